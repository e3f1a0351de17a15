/* ctm.h -- corner-transfer renormalisation (CTMRG) environments of a
 * two-site-unit-cell square-lattice iPEPS on one AMD MI355X (gfx950) GPU.
 *
 * Method: W. Lan and G. Evenbly, "Reduced Contraction Costs of
 * Corner-Transfer Methods for PEPS", arXiv:2306.08212.
 *   - problem statement (local tensors A, B of dimensions (d, D, D, D, D);
 *     environment {C^i, T^i} of boundary dimension chi; left/right/up/down
 *     moves repeated until converged): Sec. II, Figs. 1-2;
 *   - standard isometries (SVD of the half-plaquette, cost chi^3 D^6):
 *     Sec. II, Fig. 2(c);
 *   - reduced environment and sequential ket-then-bra ("sequential-order")
 *     isometries v^1, v^2, cost chi^3 D^3: Secs. III-IV, Figs. 3-4 and the
 *     Appendix (helper isometries v_l, v_r);
 *   - bond energy of the Heisenberg model: Sec. V, Eq. (1).
 *
 * Conventions (the paper's figures are not available; these are fixed here):
 *   Site tensors are row-major double arrays A[s][l][u][r][d], d * D^4
 *   values each; A sits on sublattice a, B on sublattice b (checkerboard).
 *   The environment holds 16 tensors, index e = 8*kind + 2*(i-1) + z with
 *   kind 0 = corner C^i, 1 = edge T^i, i = 1..4, z = 0 (a) or 1 (b):
 *   C1, C2, C3, C4 are the up-left, up-right, down-right, down-left corners of
 *   a z-site and T1, T2, T3, T4 the edges left of, above, right of and below
 *   it.  Index order runs clockwise around the boundary: C^i[p][q] with p the
 *   bond to T^i and q the bond to T^{i+1}; T^i[p][k][b][q] with p toward
 *   C^{i-1}, q toward C^i and (k, b) the ket and bra legs into the site
 *   (each of dimension D).  Bond dimensions start at D^2 (traced-boundary
 *   initial environment) and grow to at most chi.
 *
 * Errors: every function returns a ctm_status (CTM_OK = 0); nothing throws
 * across this interface.  With the environment variable CTM_DEBUG_HIP set,
 * the first failing HIP call of an operation is also named on stderr.  The
 * library must use the same HIP runtime as the caller's device buffers (with
 * PyTorch: load torch before this library).  All functions taking a solver
 * enqueue work on the solver's stream and return without waiting unless
 * stated otherwise.
 */
#ifndef CTM_H
#define CTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_solver ctm_solver; /* opaque, owned by the library */

enum ctm_status {
  CTM_OK = 0,
  CTM_EINVAL = 1,    /* bad argument (d < 2, D < 1, chi < D^2, NULL pointer,
                        bad enum)                                            */
  CTM_ENOMEM = 2,    /* workspace smaller than ctm_workspace_size(), or a
                        host allocation failed                              */
  CTM_EHIP = 3,      /* a HIP runtime call failed (including a failed graph
                        capture of a move)                                  */
  CTM_ENUMERIC = 4,  /* a tensor norm was zero, NaN or Inf, or a Jacobi SVD
                        of a truncation did not converge within its sweep
                        cap; reported by the next synchronising call
                        (ctm_converge, ctm_read_delta, ctm_energy) and kept
                        for the solver's lifetime                           */
  CTM_ENOTCONV = 5   /* ctm_converge reached max_iters; state stays valid    */
};

enum ctm_method {
  CTM_STANDARD = 0,   /* standard isometries every move (Sec. II)            */
  CTM_REDUCED = 1,    /* sequential-order isometries (Secs. III-IV, App.)    */
  CTM_REDUCED_ENV = 2 /* reduced-env: one 4-index isometry from the reduced
                         half-network [C1 T2 C2; T1 z T3] (Sec. III,
                         Fig. 3(a,b)), cost chi^3 D^4                        */
};

enum ctm_precision {
  CTM_FP64 = 0,      /* every contraction in FP64                            */
  CTM_FP32 = 1,      /* absorption chains on FP32 MFMA; SVDs, norms, energy FP64 */
  CTM_BF16 = 2       /* absorption chains on BF16 MFMA with FP32 accumulation */
};

enum ctm_dir { CTM_LEFT = 0, CTM_UP = 1, CTM_RIGHT = 2, CTM_DOWN = 3 };

typedef struct {
  int d;                 /* physical dimension (>= 2)                         */
  int D;                 /* virtual bond dimension (>= 1)                     */
  int chi;               /* boundary dimension chi (>= D^2: the traced-boundary
                            environment starts with bonds of dimension D^2)  */
  int method;            /* enum ctm_method                                   */
  int precision;         /* enum ctm_precision                                */
  int boot_iters;        /* leading iterations that use standard isometries
                            whatever the method (>= 0; 0 = only where the
                            reduced move could not grow a bond, by shape)    */
  double svd_cutoff;     /* relative singular-value cutoff tau (1e-14)        */
  void *stream;          /* hipStream_t the solver is bound to; NULL = null stream */
  void *workspace;       /* caller-owned device memory, >= ctm_workspace_size */
  size_t workspace_bytes;
  int chi_p;             /* chi': bond of the first-stage isometry v^1 of the
                            sequential-order split (Sec. IV: "slightly larger
                            chi'" for strongly correlated states); 0 = chi,
                            else >= chi                                      */
  int chi_pp;            /* chi'': bond of the first stage of the helper
                            isometries v_l^1, v_r^1 (App.); 0 = chi, else
                            >= chi.  Sec. V sets both to chi.                */
} ctm_config;

/* Exact peak device bytes one solver uses for cfg (all of it inside the
 * caller's workspace; the library allocates no device memory of its own).
 * Host-only; returns 0 for an invalid cfg. */
size_t ctm_workspace_size(const ctm_config *cfg);

/* Create a solver for the problem of Sec. II: the two-site unit cell {A, B}
 * of 5-index site tensors (d, D, D, D, D) and the 16 environment tensors
 * {C^i_z, T^i_z} of boundary dimension chi (Fig. 1(d)).  Copies A and B
 * (host or device pointers, ptrs_on_device; the caller keeps its buffers),
 * builds the initial environment -- the paper does not state one; here each
 * tensor is the single boundary site it stands for with its outward legs
 * traced (ket = bra), bonds D^2 -- and normalises it.  *out receives the
 * handle; free it with ctm_destroy.  Synchronises the stream once.
 * CTM_EINVAL for a bad cfg (d < 2, D < 1, chi < D^2, unknown method or
 * precision) or NULL pointers, CTM_ENOMEM when cfg->workspace_bytes is below
 * ctm_workspace_size(cfg), CTM_EHIP for a failed HIP call. */
int ctm_init(const ctm_config *cfg, const double *A, const double *B, int ptrs_on_device,
             ctm_solver **out);

/* One directional move (Sec. II, Fig. 2(a,b)): two column insertions, each
 * absorbing {T^2, site, site, T^4} into the left environment and truncating
 * the enlarged bonds with the isometries of the solver's method -- standard
 * (Sec. II, Fig. 2(c)) or sequential-order (Secs. III-IV, Figs. 3-4, App.).
 * The other directions are the left move in a frame turned dir quarter
 * turns (Sec. II, "moves in other directions can be adjusted
 * accordingly").  Asynchronous; CTM_EINVAL for a bad dir. */
int ctm_move(ctm_solver *s, int dir);

/* n full iterations (moves left, right, up, down) with no host round trip. */
int ctm_iterate(ctm_solver *s, int n);

/* Iterate the four moves until converged (Sec. II: N_CTM ~ 10-30 iterations
 * of moves in four directions).  The paper gives no convergence measure;
 * here it is delta = the largest change, over the 8 corners, of a corner's
 * singular values divided by its largest one, zero padded to chi.  Stops
 * when delta < tol (CTM_OK) or after max_iters iterations (CTM_ENOTCONV;
 * the state stays valid).  Reads one scalar per iteration (synchronises).
 * iters_done / delta may be NULL.  CTM_ENUMERIC if a norm failed or an SVD
 * did not converge. */
int ctm_converge(ctm_solver *s, int max_iters, double tol, int *iters_done, double *delta);

/* One full iteration followed by the corner-spectrum change delta, all
 * enqueued on the stream with no host wait (for schedulers that overlap many
 * solves); ctm_read_delta then synchronises the stream and returns delta, or
 * CTM_ENUMERIC if a tensor norm failed. */
int ctm_iterate_delta(ctm_solver *s);
int ctm_read_delta(ctm_solver *s, double *delta);

/* Bond energies of Sec. V, Eq. (1): e_bond = Tr(rho h) / Tr(rho) with rho
 * the two-site reduced density matrix of a nearest-neighbour bond contracted
 * from the environment (a 2 x 4 network: the two sites between their edges
 * and corners), for the four bond types, and the per-site energy
 * e_site = (sum of e_bond) / 2 (two bonds per site).  h2 is a host d^2 x d^2
 * row-major operator h[(s1 s2)][(s1' s2')] acting on (left, right) or
 * (top, bottom) sites, or NULL for S.S with S = sigma / 2 -- Eq. (1) prints
 * -S.S "with Pauli matrices", but the quoted QMC energy -0.669437 is that of
 * the spin-1/2 antiferromagnet +S.S, S = sigma / 2, which is used here.
 * e_bond order: horizontal (a left of b), horizontal (b left of a), vertical
 * (a above b), vertical (b above a).  Synchronises the stream.  CTM_ENUMERIC
 * for a non-finite or zero-trace result or a pending numeric error. */
int ctm_energy(ctm_solver *s, const double *h2, double *e_site, double e_bond[4]);

/* One-site expectation values out[0] = <op>_a, out[1] = <op>_b of a d x d
 * host operator op[s'][s] (row-major, acting on the ket index s), each from
 * the site between its four corners and four edges: <op> = tr(rho op) /
 * tr(rho).  Sec. V: the staggered magnetisation of the Heisenberg model
 * (|<S>_a - <S>_b| / 2), the order parameter m_z = <S^z> and the
 * transverse-field term <S^x> of the Ising model.  Synchronises the stream;
 * CTM_EINVAL for NULL pointers, CTM_ENUMERIC for a non-finite result. */
int ctm_expect1(ctm_solver *s, const double *op, double out[2]);

/* Connected correlation along a row, out[x-1] = <op_0 op_x> - <op_0><op_x>
 * for x = 1..L (1 <= L <= 4096), with site 0 on sublattice a and the row
 * horizontal (Sec. V, Fig. 8(b): S_zz(x) at the Ising critical point).  The
 * row between the edges above and below it is contracted column by column
 * from the left boundary of site 0 to the right boundary of site x (ket
 * layer before bra layer, chi^3 D^4 + chi^2 D^6 d per column).  op as for
 * ctm_expect1.  Synchronises the stream. */
int ctm_row_correlation(ctm_solver *s, const double *op, int L, double *out);

/* Copy environment tensor e (0..15, see above) to host memory: writes its two
 * boundary dimensions to *p, *q and, if host_out is not NULL and n is large
 * enough (p*q for corners, p*D*D*q for edges), the values.  Synchronises. */
int ctm_get_env(ctm_solver *s, int e, double *host_out, size_t n, int *p, int *q);

/* Replace environment tensor e with host data of boundary dimensions (p, q),
 * each at most max(chi, D^2) (warm start, resume). */
int ctm_set_env(ctm_solver *s, int e, const double *host_in, int p, int q);

/* Moves done so far. */
int ctm_moves_done(const ctm_solver *s);

/* Graph replay of moves (default on).  The independent branches of a move
 * (the side isometries and anchors of an insertion, the updates of its two
 * rows) each run on a stream of their own; a branch whose launch sequence
 * (fixed by direction, bond dimensions, method, precision, bootstrap state
 * and its place in the move) comes up a second time is captured into a HIP
 * graph and replayed from then on, so branches still overlap and the host
 * issues a handful of calls per branch instead of one per kernel.  Results
 * are bitwise those of eager launches.  ctm_set_graphs(s, 0) runs every move
 * eagerly; either call synchronises the stream and frees the captured
 * graphs.  Moves run eagerly while the profiler is on. */
int ctm_set_graphs(ctm_solver *s, int enable);

/* Switch the precision of the absorption chains (enum ctm_precision) for the
 * moves that follow; the environment is kept. */
int ctm_set_precision(ctm_solver *s, int precision);

/* Live kernel timing.  ctm_profile(s, 1) clears and starts recording a HIP
 * event pair around every kernel launch of the solver (0 stops); both
 * synchronise the stream.  ctm_profile_read returns, for one kernel class,
 * the launches recorded, their summed duration in ms and their algorithmic
 * flop and byte counts (synchronises).  Classes: 0 FP64 GEMM kernel, 1 FP32
 * GEMM, 2 BF16 GEMM, 3 permute/cast, 4 Jacobi SVD round kernel, 5 other SVD
 * kernels, 6 norms, scaling and split-K sums, 7 device copies, 8 the block
 * Cholesky factorisation and inverse of the orthonormalisation.  The work of
 * a Jacobi round depends on the data (which column pairs still rotate), so
 * class 4's counts are tallied by the kernel itself on the device. */
int ctm_profile(ctm_solver *s, int enable);
int ctm_profile_read(ctm_solver *s, int cls, long long *launches, double *ms, double *flops,
                     double *bytes);

void ctm_destroy(ctm_solver *s);

/* Static string for a status code (and the last HIP error of a solver, if any). */
const char *ctm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* CTM_H */

// FP64 truncated SVD for the chi-truncation of the corner-transfer move.
//
// The isometries of the move are the top-k left singular vectors of a
// reshaped sub-network (standard isometry, the split isometries v^1, v^2 and
// the helper isometries v_l, v_r).  They are computed with a QR-preconditioned
// one-sided (Hestenes) block Jacobi method:
//
//   For M (m x n, m >= n) the columns are ordered by decreasing norm and
//   orthonormalised (M P = Q R, blocked classical Gram-Schmidt applied
//   twice).  X = R^T (n x n) is then orthogonalised by plane rotations from
//   the right, X <- X J, until every pair of columns is orthogonal.  With
//   R^T J = W Sigma we have M P = (Q J) Sigma W^T, so U = Q J: the singular
//   values are the column norms of X and the left singular vectors are the
//   accumulated rotations mapped through Q (orthonormal by construction).
//   The triangular factor of a norm-ordered QR has rows of decreasing size,
//   which makes its transpose closer to column-orthogonal than M; two more
//   norm-ordered QR steps of the square factor (R^T = Q' R', then again)
//   push it further toward diagonal, and the sweeps then converge in about
//   five even for strongly graded spectra, where on M itself they crawl.  A wide M (m < n) is first reduced to the square
//   L = M Q_1 from the QR of M^T, which has the same left singular vectors.
//
// Stopping test for a pair of columns a, b with Gram entries g_aa, g_bb, g_ab:
// no rotation if either column is below the rounding noise of the rotations
// (g < 4 r eps^2 ||M||_F^2), if |g_ab| <= r eps sqrt(g_aa g_bb) (orthogonal to
// working accuracy), or if |g_ab| <= eps ||M||_F sqrt(max(g_aa, g_bb)) / 4:
// the component of one column along the other is then below a quarter of
// eps ||M||_F, under the absolute accuracy any backward-stable SVD (and
// LAPACK's) delivers.  Without that absolute floor, columns of very small norm
// chase orthogonality they cannot reach and the sweeps never end.  (With a
// floor of 4 eps ||M||_F the move's energies at D=4, chi=64 sat 2e-10 from
// LAPACK's after two reduced iterations; with eps / 4 they sit at 1e-11, and
// the sweep counts do not change.)
//
// Columns are grouped in blocks of 16; one workgroup takes a pair of blocks
// (32 columns), forms their 32 x 32 Gram matrix, applies one cyclic Jacobi
// sweep to it in LDS (the outer sweeps finish the job), and
// applies the resulting rotation to the 32 columns of X and of J.  Block
// pairs follow a round-robin tournament, so the pairs of one round are
// disjoint and run as one launch.  A device flag ends the sweeps once a full
// sweep applied no rotation.
//
// Afterwards the columns are ranked by norm (ties by index), the top kk are
// kept, columns with sigma <= tau * sigma_0 are zeroed and every kept column
// of U is sign-fixed: among the rows whose magnitude is within 1e-8
// (relative) of the largest, the lowest is made positive.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ctm_internal.h"

namespace ctm {
namespace {

constexpr int JW = 16;         // columns per block
constexpr int JP = 2 * JW;     // columns per pair
constexpr double kSignTie = 1e-8;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void rr_pair(int nb, int round, int i, int* a, int* b) {
  // circle method: block 0 fixed, the others rotate
  auto pos = [&](int k) { return ((k - 1 + round) % (nb - 1)) + 1; };
  *a = (i == 0) ? 0 : pos(i);
  *b = pos(nb - 1 - i);
}

// Reciprocal and reciprocal square root from the hardware estimates and two
// Newton steps (each squares the relative error).  A dependent FP64
// operation costs tens of cycles on this GPU, and the compiler's correctly
// rounded division and square root are chains of about ten of them, which
// set the pace of the serial steps below; these take five to seven and agree
// with the rounded results to about an ulp.  Arguments are positive and
// finite where they are used.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Orders a wave's LDS accesses for the compiler across this point (the
// hardware completes one wave's LDS operations in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane `lane`'s value of v (lane a compile-time or wave-uniform index).
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Rotation test for a column pair (see the file comment): thr = 4 eps ||M||_F.
// Compared in squares (Gram entries of normalised data are far from overflow).
__device__ __forceinline__ bool needs_rotation(double app, double aqq, double apq, double tol,
                                               double gnoise, double thr) {
  const double a2 = apq * apq;
  return fmin(app, aqq) > gnoise && a2 > tol * tol * fabs(app * aqq) &&
         a2 > thr * thr * fmax(app, aqq);
}

// in-LDS cyclic Jacobi on the symmetric positive semi-definite 32 x 32 Gram
// matrix G, at most max_sweeps sweeps; J accumulates the rotations.
// Rutishauser's update of the pivot entries (a_pp - t a_pq, a_qq + t a_pq,
// a_pq = 0) keeps small entries relatively accurate.
//
// One step applies the 16 disjoint rotations of a round-robin round as
// G <- J^T G J.  Thread t owns the 2 x 2 block of G at the rows of pair t/16
// and the columns of pair t%16, and two rows of J's columns of pair t/16;
// it computes both rotations it needs from the pivot entries itself, so a
// step is one read phase and one write phase (rows first, then columns, the
// same order of operations as a row pass followed by a column pass).
// Computed without branches (the pairs of a step diverge in whether they
// rotate): every quantity is formed and the identity selected where the
// pair needs no rotation.
__device__ __forceinline__ bool jac_rotation(double app, double aqq, double apq, double tol,
                                             double gnoise, double thr, double* c, double* s,
                                             double* tt) {
  const bool rot = needs_rotation(app, aqq, apq, tol, gnoise, thr);
  const double tau = (aqq - app) * rcp_nr(2.0 * (rot ? apq : 1.0));
  const double at = fabs(tau);
  // sqrt(1 + tau^2) = |tau| to working precision beyond 1e100
  const bool big = at > 1e100;
  const double u = fma(big ? 0.0 : tau, big ? 0.0 : tau, 1.0);
  double t = rcp_nr(big ? 2.0 * at : at + u * rsq_nr(u));
  t = tau >= 0.0 ? t : -t;
  const double cc = rsq_nr(fma(t, t, 1.0));
  *tt = rot ? t : 0.0;
  *c = rot ? cc : 1.0;
  *s = rot ? t * cc : 0.0;
  return rot;
}

__device__ void lds_sym_jacobi(double (*G)[JP + 1], double (*J)[JP + 1], double tol,
                               double gnoise, double thr, int max_sweeps, int* sflag) {
  const int t = threadIdx.x;
  for (int idx = t; idx < JP * JP; idx += blockDim.x) J[idx / JP][idx % JP] = (idx / JP == idx % JP) ? 1.0 : 0.0;
  const int bi = t >> 4, bj = t & 15;   // pair of the rows / of the columns
  const int jr = (t & 15) * 2;          // rows of J this thread rotates
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (t == 0) *sflag = 0;
    __syncthreads();
    for (int round = 0; round < JP - 1; ++round) {
      int pi, qi, pj, qj;
      rr_pair(JP, round, bi, &pi, &qi);
      if (pi > qi) { const int x = pi; pi = qi; qi = x; }
      rr_pair(JP, round, bj, &pj, &qj);
      if (pj > qj) { const int x = pj; pj = qj; qj = x; }
      const double app = G[pi][pi], aqq = G[qi][qi], apq = G[pi][qi];
      const double bpp = G[pj][pj], bqq = G[qj][qj], bpq = G[pj][qj];
      const double b00 = G[pi][pj], b01 = G[pi][qj], b10 = G[qi][pj], b11 = G[qi][qj];
      const double j00 = J[jr][pi], j01 = J[jr][qi], j10 = J[jr + 1][pi], j11 = J[jr + 1][qi];
      double ci, si, ti, cj, sj, tj;
      const bool roti = jac_rotation(app, aqq, apq, tol, gnoise, thr, &ci, &si, &ti);
      jac_rotation(bpp, bqq, bpq, tol, gnoise, thr, &cj, &sj, &tj);
      __syncthreads();   // every read of this step precedes every write
      if (bi == bj) {
        if (roti) {
          G[pi][pi] = app - ti * apq;
          G[qi][qi] = aqq + ti * apq;
          G[pi][qi] = 0.0;
          G[qi][pi] = 0.0;
        }
      } else {
        const double r00 = ci * b00 - si * b10, r01 = ci * b01 - si * b11;
        const double r10 = si * b00 + ci * b10, r11 = si * b01 + ci * b11;
        G[pi][pj] = cj * r00 - sj * r01;
        G[pi][qj] = sj * r00 + cj * r01;
        G[qi][pj] = cj * r10 - sj * r11;
        G[qi][qj] = sj * r10 + cj * r11;
      }
      if (roti) {
        J[jr][pi] = ci * j00 - si * j01;
        J[jr][qi] = si * j00 + ci * j01;
        J[jr + 1][pi] = ci * j10 - si * j11;
        J[jr + 1][qi] = si * j10 + ci * j11;
        if (bj == 0) *sflag = 1;
      }
      __syncthreads();
    }
    if (*sflag == 0) break;
    __syncthreads();
  }
}

// One round of the block tournament.  X: r rows, ld = ldx, column-major.
// V: vr rows (0 = none), ld = vr.  fro: ||X||_F on the device.
// The 32 columns of a block pair pass through LDS in chunks of CH rows; the
// Gram matrix and the rotation of the columns are FP64 matrix-core products
// (v_mfma_f64_16x16x4f64: operand lane l holds row l%16 / column l%16 at
// k = l/16; result lane l, element i is row l/16 + 4 i, column l%16).
constexpr int CH = 64;

// LDS of one block pair's step.
struct JacLds {
  double G[JP][JP + 1];
  double J[JP][JP + 1];
  double chunk[CH][JP + 1];
  double outc[CH][JP + 1];
  int any, sflag;
};

// The step of one block pair (pair of round `round`), run by a whole
// workgroup.
__device__ __forceinline__ void jac_pair(double* __restrict__ X, int r, int64_t ldx,
                                         double* __restrict__ V, int vr, int nb, int round,
                                         int pair, double tol, double tol_in, int inner_sweeps,
                                         const double* __restrict__ fro, int* __restrict__ flags,
                                         double* __restrict__ work, double thr_mult, JacLds& L) {
  double (*G)[JP + 1] = L.G;
  double (*J)[JP + 1] = L.J;
  double (*chunk)[JP + 1] = L.chunk;
  double (*outc)[JP + 1] = L.outc;
  int& any = L.any;
  int& sflag = L.sflag;
  // columns below the rounding noise of the rotations (norm < 2 sqrt(r) eps
  // ||M||_F) are not made orthogonal: their directions are not determined by
  // the data, and chasing them only spins through sweeps
  const double gnoise = 4.0 * (double)r * 4.930380657631324e-32 * fro[0] * fro[0];
  const double thr = thr_mult * 2.220446049250313e-16 * fro[0];
  int bi, bj;
  rr_pair(nb, round, pair, &bi, &bj);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  auto col = [&](int a) { return a < JW ? bi * JW + a : bj * JW + (a - JW); };

  constexpr int PER = CH * JP / 256;   // doubles per thread and chunk
  double pre[PER];
  auto fetch = [&](const double* src, int rows, int64_t ld, int row0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + 256 * q;
      const int a = e / CH, rr = e % CH;
      const int gr = row0 + rr;
      pre[q] = gr < rows ? src[(int64_t)col(a) * ld + gr] : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + 256 * q;
      chunk[e % CH][e / CH] = pre[q];
    }
  };

  // Gram: wave w computes the 16 x 16 tile (w / 2, w % 2)
  const int mt = wave >> 1, nt = wave & 1;
  d4 gacc = {0.0, 0.0, 0.0, 0.0};
  fetch(X, r, ldx, 0);
  for (int row0 = 0; row0 < r; row0 += CH) {
    stash();
    __syncthreads();
    if (row0 + CH < r) fetch(X, r, ldx, row0 + CH);
#pragma unroll
    for (int kk = 0; kk < CH; kk += 4) {
      const int kr = kk + (lane >> 4);
      gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(chunk[kr][mt * 16 + (lane & 15)],
                                                  chunk[kr][nt * 16 + (lane & 15)], gacc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) G[mt * 16 + (lane >> 4) + 4 * q][nt * 16 + (lane & 15)] = gacc[q];
  if (t == 0) any = 0;
  __syncthreads();
  {
    const int ga = t >> 3, gb = (t & 7) * 4;
    for (int q = 0; q < 4; ++q) {
      const int b = gb + q;
      if (b != ga) {
        const double gab = G[ga][b], gaa = G[ga][ga], gbb = G[b][b];
        if (needs_rotation(gaa, gbb, gab, tol, gnoise, thr)) any = 1;
      }
    }
  }
  __syncthreads();
  // algorithmic work of this block pair, for the profiler: the Gram
  // (2 r 32^2 flop, r 32 doubles read) and, when it rotates, X J and V J
  // (2 (r + vr) 32^2 flop, (r + vr) 32 doubles read and written)
  if (work != nullptr && t == 0) {
    const double rot = any ? 1.0 : 0.0;
    atomicAdd(&work[0], 2.0 * JP * JP * (r + rot * (r + vr)));
    atomicAdd(&work[1], 8.0 * JP * (r + rot * 2.0 * (r + vr)));
  }
  if (!any) return;
  lds_sym_jacobi(G, J, tol_in, gnoise, thr, inner_sweeps, &sflag);
  if (t == 0) atomicAdd(&flags[1], 1);

  // [X; V][:, cols] <- [X; V][:, cols] J, as one stream of CH-row chunks over
  // the rows of X and then of V.  Wave w forms row tiles 2 (w / 2) and
  // 2 (w / 2) + 1 of column tile w % 2; its slice of J stays in registers.
  double jb[JP / 4];
#pragma unroll
  for (int q = 0; q < JP / 4; ++q) jb[q] = J[4 * q + (lane >> 4)][nt * 16 + (lane & 15)];
  const int nx = (r + CH - 1) / CH, nv = (V != nullptr) ? (vr + CH - 1) / CH : 0;
  auto fetch_chunk = [&](int ci) {
    if (ci < nx) fetch(X, r, ldx, ci * CH);
    else fetch(V, vr, vr, (ci - nx) * CH);
  };
  fetch_chunk(0);
  for (int ci = 0; ci < nx + nv; ++ci) {
    stash();
    __syncthreads();
    if (ci + 1 < nx + nv) fetch_chunk(ci + 1);
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2) {
      const int m2 = (wave >> 1) * 2 + i2;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < JP / 4; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(chunk[m2 * 16 + (lane & 15)][4 * q + (lane >> 4)],
                                                   jb[q], acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) outc[m2 * 16 + (lane >> 4) + 4 * q][nt * 16 + (lane & 15)] = acc[q];
    }
    __syncthreads();
    const bool isx = ci < nx;
    const int row0 = isx ? ci * CH : (ci - nx) * CH;
    const int rows = isx ? r : vr;
    double* dst = isx ? X : V;
    const int64_t ld = isx ? ldx : (int64_t)vr;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + 256 * q;
      const int a = e / CH, rr = e % CH;
      if (row0 + rr < rows) dst[(int64_t)col(a) * ld + row0 + rr] = outc[rr][a];
    }
  }
}

__global__ __launch_bounds__(256) void jac_round_kernel(double* __restrict__ X, int r, int64_t ldx,
                                                        double* __restrict__ V, int vr, int nb,
                                                        int round, double tol, double tol_in,
                                                        int inner_sweeps,
                                                        const double* __restrict__ fro,
                                                        int* __restrict__ flags,
                                                        double* __restrict__ work, int xslot,
                                                        double thr_mult) {
  __shared__ JacLds L;
  // workgroups go to the 8 XCDs round robin; only those of XCD xslot work,
  // so every round of one SVD finds X and V in the same L2
  if ((int)(blockIdx.x & 7) != xslot) return;
  if (flags[0]) return;   // converged in an earlier sweep
  jac_pair(X, r, ldx, V, vr, nb, round, blockIdx.x >> 3, tol, tol_in, inner_sweeps, fro, flags,
           work, thr_mult, L);
}

// The sweeps after the first few, in one launch of one workgroup, which
// returns at once when the sweeps have converged (nearly always: the
// preconditioned sweeps converge in at most about six).  Otherwise it takes
// the remaining sweeps' block pairs one after the other, in the order the
// rounds take them (every pair of a round is disjoint from the others, so
// the order within a round does not change the result), and ends each sweep
// as jac_sweep_end does.
__global__ __launch_bounds__(256) void jac_late_kernel(double* __restrict__ X, int r, int64_t ldx,
                                                       double* __restrict__ V, int vr, int nb,
                                                       double tol, double tol_in, int inner_sweeps,
                                                       const double* __restrict__ fro,
                                                       int* __restrict__ flags,
                                                       double* __restrict__ work,
                                                       double thr_mult, int sweeps) {
  __shared__ JacLds L;
  __shared__ int done;
  const int t = threadIdx.x;
  for (int sw = 0; sw < sweeps; ++sw) {
    if (t == 0) done = flags[0];
    __syncthreads();
    if (done) return;
    for (int rd = 0; rd < nb - 1; ++rd)
      for (int p = 0; p < nb / 2; ++p) {
        jac_pair(X, r, ldx, V, vr, nb, rd, p, tol, tol_in, inner_sweeps, fro, flags, work,
                 thr_mult, L);
        // this pair's columns of X and V, and its count, before the next
        // pair reads them
        __threadfence();
        __syncthreads();
      }
    if (t == 0) {
      if (flags[0] == 0 && flags[1] == 0) flags[0] = 1;
      if (flags[0] == 0) flags[2] += 1;
      flags[1] = 0;
    }
    __threadfence();
    __syncthreads();
  }
}

__global__ void jac_sweep_end(int* flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (flags[0] == 0 && flags[1] == 0) flags[0] = 1;
    if (flags[0] == 0) flags[2] += 1;   // sweeps that rotated something
    flags[1] = 0;
  }
}

// After the last sweep: a Jacobi solve whose final sweep still rotated has
// not converged; bit 2 of the solver's numeric error word records it (the
// word is only ever set, never cleared, by kernels).
__global__ void jac_converged_check(const int* __restrict__ flags, int* __restrict__ err) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && flags[0] == 0) err[0] |= 2;
}

__global__ void jac_flags_init(int* flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
    flags[2] = 0;
  }
}

// V (col-major, vr x cp) = identity on the first vr columns, zero beyond.
__global__ __launch_bounds__(256) void eye_kernel(double* __restrict__ V, int vr, int cp) {
  const int64_t tv = (int64_t)vr * cp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tv; e += (int64_t)gridDim.x * 256) {
    const int j = (int)(e / vr), i = (int)(e % vr);
    V[e] = (i == j) ? 1.0 : 0.0;
  }
}

// Column sums of squares of row-major M (m x n) over row chunks of `rows`
// rows: part[chunk * n + j].  Fixed summation order (deterministic).
__global__ __launch_bounds__(256) void rm_colsq_kernel(const double* __restrict__ M, int m, int n,
                                                       int rows, double* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int i0 = blockIdx.y * rows, i1 = min(m, i0 + rows);
  // sixteen loads in flight, then their squares summed in row order
  double s = 0.0;
  int i = i0;
  for (; i + 16 <= i1; i += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = M[(int64_t)(i + u) * n + j];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u] * v[u];
  }
  for (; i < i1; ++i) {
    const double v = M[(int64_t)i * n + j];
    s += v * v;
  }
  part[(int64_t)blockIdx.y * n + j] = s;
}

__global__ __launch_bounds__(256) void rm_colnorm_kernel(const double* __restrict__ part,
                                                         int chunks, int n,
                                                         double* __restrict__ sig) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  int q = 0;
  for (; q + 8 <= chunks; q += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * n + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < chunks; ++q) s += part[(int64_t)q * n + j];
  sig[j] = sqrt(s);
}

// Q[:, t] = M[:, order[t]] (row-major m x n).
__global__ __launch_bounds__(256) void gather_cols_kernel(const double* __restrict__ M, int m,
                                                          int n, const int* __restrict__ order,
                                                          double* __restrict__ Q) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n;
    const int t = (int)(e % n);
    const int j = order[t];
    Q[e] = (j >= 0 && j < n) ? M[i * n + j] : 0.0;   // j is always in range (see the ranking)
  }
}

// column norms -> sig[cp]
__global__ __launch_bounds__(256) void jac_colnorm_kernel(const double* __restrict__ X, int r,
                                                          int cp, double* __restrict__ sig) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < r; i += 256) {
    const double v = X[(int64_t)j * r + i];
    s += v * v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sig[j] = sqrt(sh[0]);
}

// order[rank] = column, for ranks < kk (descending norm, ties by index)
// A NaN ranks below every number (as -inf, ties by index), so the ranks are
// always a permutation of 0..c-1 and order[] holds valid column indices
// whatever the data: the indices feed gathers.
// A workgroup ranks 64 keys; its four waves each count, for every one of
// them, the keys of one quarter of the list that precede it.  Launch with
// (c + 63) / 64 workgroups.
__global__ __launch_bounds__(256) void jac_rank_kernel(const double* __restrict__ sig, int c, int kk,
                                                       int* __restrict__ order) {
  __shared__ int part[4][64];
  const int jl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  auto key = [](double x) { return x == x ? x : -INFINITY; };
  const double v = j < c ? key(sig[j]) : 0.0;
  const int per = (c + 3) / 4, lo = q * per, hi = min(c, lo + per);
  int r4[4] = {0, 0, 0, 0};
  int i = lo;
  for (; i + 4 <= hi; i += 4)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double w = key(sig[i + u]);
      r4[u] += (w > v) || (w == v && i + u < j);
    }
  for (; i < hi; ++i) {
    const double w = key(sig[i]);
    r4[0] += (w > v) || (w == v && i < j);
  }
  part[q][jl] = (r4[0] + r4[1]) + (r4[2] + r4[3]);
  __syncthreads();
  if (q == 0 && j < c) {
    const int rank = (part[0][jl] + part[1][jl]) + (part[2][jl] + part[3][jl]);
    if (rank < kk) order[rank] = j;
  }
}

// Uj[:, t] (row-major vr x kk) = column order[t] of the accumulated
// rotations V (col-major, vr rows), S[t] its singular value; columns with
// sigma <= tau * sigma_0 (or not finite) are zero with S = 0.
__global__ __launch_bounds__(256) void jac_pick_kernel(const double* __restrict__ V, int vr,
                                                       int cp, const double* __restrict__ sig,
                                                       const int* __restrict__ order, int kk,
                                                       double tau, double* __restrict__ Uj,
                                                       double* __restrict__ S) {
  const int64_t total = (int64_t)vr * kk;
  // order[] is a permutation of 0..cp-1 (see the ranking); the range checks
  // only keep a bad index from becoming an address
  const int o0 = order[0];
  const double s0 = (o0 >= 0 && o0 < cp) ? sig[o0] : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / kk), t = (int)(e % kk);
    const int j = order[t];
    const bool inr = j >= 0 && j < cp;
    const double sj = inr ? sig[j] : 0.0;
    const bool keep = inr && (s0 > 0.0) && (sj > tau * s0) && isfinite(sj);
    Uj[e] = keep ? V[(int64_t)j * vr + i] : 0.0;
    if (i == 0) S[t] = keep ? sj : 0.0;
  }
}

// Gram-Schmidt fallback of the in-block step, as a tree (TSQR): the block's
// rows are cut into chunks of 256; each workgroup orthonormalises its chunk in
// LDS (classical Gram-Schmidt twice, then, for a column that lost more than
// half its length in those projections, a third projection that checks the
// normalised column: if it loses more than half its length again, the column
// was rounding noise and is dependent), keeping the projection coefficients as
// the chunk's R factor.  The stacked R factors are reduced the same way until
// one chunk is left; the Q factors are then multiplied back down the tree.
// Zero columns of a Q factor come with zero rows of its R factor, so the
// product stays orthonormal on the nonzero columns.  At the top of the tree
// dependence follows the block rules: on the first visit a residual at most
// 1e-13 of the column's original norm nrm0 (recorded in dead[]), on the second
// a unit column that keeps at most half its length after the re-projection.
// First-visit dependence threshold, relative to a column's original norm
// (CTM_DEBUG_DEAD_TOL overrides it for measurements).
double dead_tol() {
  if (const char* v = std::getenv("CTM_DEBUG_DEAD_TOL")) return std::atof(v);
  return 1e-13;
}

constexpr int TQ = 256;   // rows per chunk
constexpr int OBW = 64;   // columns per orthonormalisation block
constexpr int OBP = OBW + 1;

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// LDS of one chunk of the Gram-Schmidt tree, in doubles: T[TQ][OBP], then
// red[256 / OBW][OBP], coef[OBW] and sh[4].
constexpr int TSQR_LDS = TQ * OBP + (256 / OBW) * OBP + OBW + 4;

// One chunk (TQ rows from row chunk * TQ) of a level of the Gram-Schmidt
// tree, run by a whole workgroup; L is TSQR_LDS doubles of LDS.
__device__ __forceinline__ void tsqr_local_chunk(
    const double* __restrict__ src, int rows, int64_t lds, int nb, double* __restrict__ q,
    int64_t ldq, int qcols, double* __restrict__ r, int top, const double* __restrict__ nrm0,
    int c0, int* __restrict__ dead, int final, double dead_tol, int chunk, double* L, int& dep) {
  double (*T)[OBP] = reinterpret_cast<double (*)[OBP]>(L);
  double (*red)[OBP] = reinterpret_cast<double (*)[OBP]>(L + TQ * OBP);
  double* coef = L + TQ * OBP + (256 / OBW) * OBP;
  double* sh = coef + OBW;
  const int t = threadIdx.x;
  const int i0 = chunk * TQ;
  for (int e = t; e < TQ * OBW; e += 256) {
    const int rr = e / OBW, cc = e % OBW;
    T[rr][cc] = (i0 + rr < rows && cc < nb) ? src[(int64_t)(i0 + rr) * lds + cc] : 0.0;
  }
  __syncthreads();
  constexpr int NG = 256 / OBW, GR = TQ / NG;   // row groups for the coefficients
  const int ca = t % OBW, cg = t / OBW;       // coefficient a, row group cg
  // thread t < OBW accumulates R[t][j] of the current column j
  double racc = 0.0;
  auto colsq = [&](int j) {
    const double v = (t < TQ) ? T[t][j] : 0.0;
    return block_sum256(v * v, sh);
  };
  // x <- x - sum_{a<j} coef_a q_a, coefficients accumulated into R[a][j] * w
  // (four independent partial sums in the loops: the LDS loads of a loop
  // are then issued back to back instead of one round trip per term)
  auto project = [&](int j, double w) {
    double pp = 0.0;
    if (ca < j) {
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int rr = cg * GR; rr < cg * GR + GR; rr += 4)
        for (int u = 0; u < 4; ++u) p4[u] += T[rr + u][ca] * T[rr + u][j];
      pp = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    }
    red[cg][ca] = pp;
    __syncthreads();
    if (t < j) {
      double cs = 0.0;
      for (int g = 0; g < NG; ++g) cs += red[g][t];
      coef[t] = cs;
      racc += w * cs;
    }
    __syncthreads();
    if (t < TQ) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int aa = 0;
      for (; aa + 4 <= j; aa += 4)
        for (int u = 0; u < 4; ++u) s4[u] += coef[aa + u] * T[t][aa + u];
      for (; aa < j; ++aa) s4[0] += coef[aa] * T[t][aa];
      T[t][j] -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
  };
  auto put_r = [&](int j, double rjj) {
    if (r != nullptr && t < OBW)
      r[((int64_t)chunk * OBW + t) * OBW + j] = t < j ? racc : (t == j ? rjj : 0.0);
    racc = 0.0;
  };
  for (int j = 0; j < nb; ++j) {
    if (top && final && dead[c0 + j]) {
      if (t < TQ) T[t][j] = 0.0;
      put_r(j, 0.0);
      __syncthreads();
      continue;
    }
    // squared norms; r = q rsq(q) and 1 / r = rsq(q) where q > 0
    const double q0 = colsq(j);
    project(j, 1.0);
    project(j, 1.0);
    const double q1 = colsq(j);
    const double i1 = q1 > 0.0 ? rsq_nr(q1) : 0.0, r1 = q1 * i1;
    if (t == 0) {
      bool d;
      if (top) d = final ? !(r1 > 0.5) : !(r1 > dead_tol * nrm0[c0 + j]);
      else d = !(q1 > 1e-26 * q0);
      dep = d ? 1 : 0;
    }
    __syncthreads();
    double rjj = 0.0;
    if (!dep) {
      if (t < TQ) T[t][j] *= i1;
      __syncthreads();
      if (q1 >= 0.25 * q0) {
        // the column kept at least half its norm through the two
        // projections: it is orthogonal to the earlier ones to working
        // accuracy already ("twice is enough"), and a third projection
        // would only move it by rounding
        rjj = r1;
      } else {
        project(j, r1);
        const double q2 = colsq(j);
        if (t == 0) dep = (q2 > 0.25) ? 0 : 1;
        __syncthreads();
        if (!dep) {
          const double i2 = rsq_nr(q2);
          if (t < TQ) T[t][j] *= i2;
          rjj = r1 * (q2 * i2);
        }
      }
    }
    if (dep && t < TQ) T[t][j] = 0.0;
    put_r(j, rjj);
    if (t == 0 && top && !final) dead[c0 + j] = dep;
    __syncthreads();
  }
  for (int j = nb; j < OBW; ++j) put_r(j, 0.0);
  for (int e = t; e < TQ * OBW; e += 256) {
    const int rr = e / OBW, cc = e % OBW;
    if (i0 + rr < rows && cc < qcols) q[(int64_t)(i0 + rr) * ldq + cc] = T[rr][cc];
  }
}

// dst rows of chunk b = Q rows of chunk b (TQ x OBW, ld OBW) times W rows
// [OBW b, OBW b + OBW) (ld OBW); nb columns.  The chunk's rows go through
// LDS in two halves; L is LDS of at least OBW * OBP + (TQ / 2) * OBP
// doubles.  Run by a whole workgroup.
__device__ __forceinline__ void tsqr_apply_chunk(const double* __restrict__ Q, int rows,
                                                 const double* __restrict__ W, int nb,
                                                 double* __restrict__ dst, int64_t ldd, int b,
                                                 double* L) {
  constexpr int TH = TQ / 2;
  double (*Ws)[OBP] = reinterpret_cast<double (*)[OBP]>(L);
  double (*Qs)[OBP] = reinterpret_cast<double (*)[OBP]>(L + OBW * OBP);
  const int t = threadIdx.x;
  for (int e = t; e < OBW * OBW; e += 256)
    Ws[e / OBW][e % OBW] = W[((int64_t)b * OBW + e / OBW) * OBW + e % OBW];
  for (int h = 0; h < 2; ++h) {
    const int i0 = b * TQ + h * TH;
    for (int e = t; e < TH * OBW; e += 256) {
      const int rr = e / OBW, cc = e % OBW;
      Qs[rr][cc] = (i0 + rr < rows) ? Q[(int64_t)(i0 + rr) * OBW + cc] : 0.0;
    }
    __syncthreads();
    // on the FP64 matrix cores: wave w forms rows 32 w .. 32 w + 31 of the
    // half, all 64 columns, as 2 x 4 tiles of 16 x 16 (result lane l,
    // element q: row l / 16 + 4 q, column l % 16 of its tile)
    const int lane = t & 63, rw = (t >> 6) * 32;
    d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < OBW; k0 += 4) {
      const int kr = k0 + (lane >> 4);
      double av[2], bv[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = Qs[rw + 16 * i + (lane & 15)][kr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Ws[kr][16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = rw + 16 * i + (lane >> 4) + 4 * q, cc = 16 * j + (lane & 15);
          if (cc < nb && i0 + rr < rows) dst[(int64_t)(i0 + rr) * ldd + cc] = acc[i][j][q];
        }
    __syncthreads();
  }
}

// The levels of the Gram-Schmidt tree above the first (which the Cholesky
// kernel runs) and the products back down, for a block that was not
// healthy.  Level l (1 <= l <= n) factors its input rows[l] x OBW (the
// stacked R factors of level l - 1) chunk by chunk into q[l] and, below the
// top level n, r[l]; then W_n = q[n], W_l = Q_l W_{l+1} into w[l] for
// n > l >= 1, and the block of U = Q_0 W_1 with Q_0 = q[0].
constexpr int kMaxTree = 8;
struct TreeLevels {
  int n;
  int rows[kMaxTree + 1];
  double* q[kMaxTree + 1];
  double* r[kMaxTree + 1];
  double* w[kMaxTree + 1];
};
static_assert(OBW * OBP + (TQ / 2) * OBP <= TSQR_LDS, "the apply's LDS fits the chunk's");

// One launch with a workgroup per chunk of level 1, which exits at once when
// the Cholesky path took the block.  The workgroups factor their chunks of
// level 1; the last to finish (a device-scope counter, zeroed by the
// Cholesky kernel; no workgroup waits for another) then runs the levels
// above and the products down alone, one chunk after the other.  A
// healthy block thus costs this one launch whatever the depth of the tree.
__global__ __launch_bounds__(256) void tsqr_upper_kernel(TreeLevels tl, int nb,
                                                         double* __restrict__ U, int64_t kk,
                                                         int c0, const double* __restrict__ nrm0,
                                                         int* __restrict__ dead, int final,
                                                         const int* __restrict__ healthy,
                                                         int* __restrict__ count,
                                                         double dead_tol) {
  __shared__ double L[TSQR_LDS];
  __shared__ int dep, last;
  if (*healthy) return;   // the Cholesky path took this block
  const int t = threadIdx.x;
  tsqr_local_chunk(tl.r[0], tl.rows[1], OBW, nb, tl.q[1], OBW, OBW, tl.r[1], tl.n == 1 ? 1 : 0,
                   nrm0, c0, dead, final, dead_tol, blockIdx.x, L, dep);
  if (gridDim.x > 1) {
    __threadfence();   // this chunk's factors reach the device before the count
    __syncthreads();
    if (t == 0) last = atomicAdd(count, 1) == (int)gridDim.x - 1 ? 1 : 0;
    __syncthreads();
    if (!last) return;
    __threadfence();
  }
  for (int l = 2; l <= tl.n; ++l) {
    const int ch = (tl.rows[l] + TQ - 1) / TQ;
    for (int b = 0; b < ch; ++b) {
      __threadfence();
      __syncthreads();
      tsqr_local_chunk(tl.r[l - 1], tl.rows[l], OBW, nb, tl.q[l], OBW, OBW, tl.r[l],
                       l == tl.n ? 1 : 0, nrm0, c0, dead, final, dead_tol, b, L, dep);
    }
  }
  const double* W = tl.q[tl.n];
  for (int l = tl.n - 1; l >= 0; --l) {
    double* out = l == 0 ? U + c0 : tl.w[l];
    const int ch = (tl.rows[l] + TQ - 1) / TQ;
    for (int b = 0; b < ch; ++b) {
      __threadfence();
      __syncthreads();
      tsqr_apply_chunk(tl.q[l], tl.rows[l], W, l == 0 ? nb : OBW, out, l == 0 ? kk : OBW, b, L);
    }
    W = out;
  }
}

// Cholesky path of the in-block step.  G (nb x nb) is the Gram matrix of the
// block's columns after the projection of the earlier blocks.  One wave
// factors G = R^T R and inverts R.  The block is "healthy" when the
// condition number of the column-scaled block, estimated from R^{-1}, is at
// most 1e6 on the first visit (Cholesky QR then leaves orthogonality errors
// below ~1e-4, which the second visit removes) and at most twice its value
// for an orthonormal block (the number of nonzero columns) on the second,
// every nonzero column keeps a pivot d_j >= delta G_jj (delta = 1e-12, then
// 0.25: unit columns that lose more than half their length are left to the
// Gram-Schmidt fallback, which decides dependence), and on the first visit
// no column is at or below 1e-13 of its original norm.  Exactly zero columns
// are dead.  R^{-1} has its dead rows and columns zero.
//
// With shift > 0 the factorisation is of G + shift diag(G) and the block is
// taken as it comes (no condition test): Q = A R^{-1} then spans exactly the
// columns of A (R is invertible on the live columns) and is orthonormal only
// up to about shift kappa^2, which is all a power-iteration basis needs.
//
// One wave does everything, in registers, with no workgroup barrier (a
// wave's LDS operations complete in order, and the fences below only keep
// the compiler from moving LDS accesses across a step):
// * Factorisation: lane i holds row i of the trailing matrix (rows and
//   columns beyond nb are zero and give zero pivots).  Row j (lane k's
//   element j, equal to row j by symmetry) goes through LDS as Rw[j], and
//   each lane applies w_ik -= (w_ij / d_j) Rw[j][k] for k > j.  The serial
//   path is the chain of pivots: d_{j+1} = a - Rw[j][j+1]^2 / d_j with a the
//   element (j+1, j+1) before step j, formed as one FMA from values that
//   are ready earlier, then its reciprocal (hardware estimate and one cubic
//   Newton step, three FMAs).  Those FMAs sit between four groups of the
//   step's updates so their latencies overlap them, and each group's entries
//   of the next pivot row are loaded as soon as the group is done.
//   The unscaled rows Rw[j] and the pivots are kept; R[j][k] = Rw[j][k] /
//   sqrt(d_j).
// * Acceptance on the recorded pivots, then R^{-1} by forward substitution
//   on L = R^T: lane i forms row i of R^{-1} (y = L^{-1} e_i), reading the
//   rows of Rw (the columns of L) in order.  The serial path is two FMAs per
//   step (the next accumulator, then the next scaled unknown, formed before
//   the step's other updates).
// The loops are unrolled so every per-lane array stays in registers.
__device__ __forceinline__ double rcp_cubic(double x, double y0) {
  const double e = fma(-x, y0, 1.0);
  return fma(y0, fma(e, e, e), y0);
}

constexpr int RLD = OBW + 4;   // 16-byte aligned LDS rows of R^{-1} and of the applied rows

// Run by the first wave of a workgroup (lanes 0..63) once G sits in Gs (zero
// beyond nb): factors G, writes R^{-1} into Rs (row-major, zero beyond nb)
// and returns whether the block is healthy; with write_state it also
// records healthy and the dead columns.  Rw is LDS scratch.
__device__ __forceinline__ int chol_factor(int nb, int c0, const double* __restrict__ nrm0,
                                           int* __restrict__ dead, int final,
                                           int* __restrict__ healthy, double shift,
                                           double dead_tol, bool write_state,
                                           double (*Rw)[OBP], const double (*Gs)[OBP],
                                           double (*Rs)[RLD]) {
  const int i = threadIdx.x;
  const double gii = Gs[i][i];
  const double n0 = i < nb ? nrm0[c0 + i] : 0.0;

  double w[OBW], row[OBW];
#pragma unroll
  for (int k = 0; k < OBW; ++k) {
    w[k] = Gs[i][k] * (i == k ? 1.0 + shift : 1.0);
    row[k] = 0.0;
  }
  // columns with G_jj != 0, one bit per lane
  const unsigned long long gmask = __ballot(gii != 0.0);
  Rw[0][i] = w[0];
  wave_lds_sync();
#pragma unroll
  for (int k = 1; k < OBW; ++k) row[k] = Rw[0][k];
  double d = readlane_f64(w[0], 0);
  bool live = d > 0.0 && (gmask & 1ull);
  double rc = rcp_cubic(d, __builtin_amdgcn_rcp(d));   // used only when live
  double a = readlane_f64(w[1], 1);                   // element (1, 1) before step 0
  double my_d = i == 0 ? d : 0.0;
#pragma clang loop unroll(full)
  for (int j = 0; j < OBW; ++j) {
    const double ci = live ? w[j] * rc : 0.0;
    double dn = 0.0, y = 1.0;
    bool liven = false;
    if (j + 1 < OBW) {
      // next pivot: lane j + 1's own update of its element j + 1
      dn = fma(-(row[j + 1] * (live ? rc : 0.0)), row[j + 1], a);
      liven = dn > 0.0 && ((gmask >> (j + 1)) & 1ull);
      my_d = i == j + 1 ? dn : my_d;
      y = __builtin_amdgcn_rcp(dn);
      w[j + 1] = fma(-ci, row[j + 1], w[j + 1]);
      Rw[j + 1][i] = w[j + 1];
      wave_lds_sync();
    }
    // element (j + 2, j + 2) after this step, for the next pivot
    if (j + 2 < OBW) {
      w[j + 2] = fma(-ci, row[j + 2], w[j + 2]);
      a = readlane_f64(w[j + 2], j + 2);
      row[j + 2] = Rw[j + 1][j + 2];
    }
    const int k0 = j + 3, nk = OBW - k0 > 0 ? OBW - k0 : 0;
    const int q1 = k0 + nk / 4, q2 = k0 + nk / 2, q3 = k0 + (3 * nk) / 4;
    double e = 0.0;
#pragma unroll
    for (int k = k0; k < q1; ++k) w[k] = fma(-ci, row[k], w[k]);
#pragma unroll
    for (int k = k0; k < q1; ++k) row[k] = Rw[j + 1][k];
    __builtin_amdgcn_sched_barrier(0);
    e = fma(-dn, y, 1.0);
#pragma unroll
    for (int k = q1; k < q2; ++k) w[k] = fma(-ci, row[k], w[k]);
#pragma unroll
    for (int k = q1; k < q2; ++k) row[k] = Rw[j + 1][k];
    __builtin_amdgcn_sched_barrier(0);
    e = fma(e, e, e);
#pragma unroll
    for (int k = q2; k < q3; ++k) w[k] = fma(-ci, row[k], w[k]);
#pragma unroll
    for (int k = q2; k < q3; ++k) row[k] = Rw[j + 1][k];
    __builtin_amdgcn_sched_barrier(0);
    y = fma(y, e, y);
#pragma unroll
    for (int k = q3; k < OBW; ++k) w[k] = fma(-ci, row[k], w[k]);
#pragma unroll
    for (int k = q3; k < OBW; ++k) row[k] = Rw[j + 1][k];
    __builtin_amdgcn_sched_barrier(0);
    d = dn;
    rc = y;
    live = liven;
  }
  const bool live_i = my_d > 0.0 && gii != 0.0;
  const double rinv_i = live_i ? rsq_nr(my_d) : 0.0;

  // acceptance: every nonzero column keeps a pivot d_j >= delta G_jj and, on
  // the first visit, no column is at or below 1e-13 of its original norm;
  // exactly zero columns are dead
  const double delta = final ? 0.25 : 1e-12;
  const bool isdead = i < nb && gii == 0.0;
  bool good_i = true;
  if (i < nb && !isdead)
    good_i = (my_d >= delta * gii) && (final || sqrt(gii) > dead_tol * n0);
  const bool ok = __all(good_i);

  // row i of R^{-1}: acc_m collects sum_{k<m} L[m][k] y_k with
  // L[m][k] = Rw[k][m] / sqrt(d_k), i.e. Rw[k][m] z_k, z_k = y_k / sqrt(d_k)
  double acc[OBW];
#pragma unroll
  for (int k = 0; k < OBW; ++k) acc[k] = 0.0;
#pragma unroll
  for (int k = 1; k < OBW; ++k) row[k] = Rw[0][k];
  double part = 0.0;
  double rk = readlane_f64(rinv_i, 0);
  double z = (i == 0 ? 1.0 : 0.0) * (rk * rk);
#pragma clang loop unroll(full)
  for (int k = 0; k < OBW; ++k) {
    const double y = fma(-acc[k], rk, (i == k ? 1.0 : 0.0) * rk);
    double zn = 0.0, rn = 0.0;
    if (k + 1 < OBW) {
      acc[k + 1] = fma(row[k + 1], z, acc[k + 1]);
      rn = readlane_f64(rinv_i, k + 1);
      zn = fma(-acc[k + 1], rn * rn, (i == k + 1 ? 1.0 : 0.0) * (rn * rn));
    }
    const int m0 = k + 2, nm = OBW - m0 > 0 ? OBW - m0 : 0;
    const int h = m0 + nm / 2;
#pragma unroll
    for (int m = m0; m < h; ++m) acc[m] = fma(row[m], z, acc[m]);
#pragma unroll
    for (int m = m0; m < h; ++m) row[m] = Rw[k + 1][m];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = h; m < OBW; ++m) acc[m] = fma(row[m], z, acc[m]);
#pragma unroll
    for (int m = h; m < OBW; ++m) row[m] = Rw[k + 1][m];
    acc[k] = y;   // row i of R^{-1}, element k
    part = fma(y, y, part);
    __builtin_amdgcn_sched_barrier(0);
    z = zn;
    rk = rn;
  }
  // kappa of the column-scaled block: || diag(sqrt(G_jj)) R^{-1} ||_F times
  // the square root of the number of live columns
  part *= gii;
  int nlive = (i < nb && !isdead) ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) {
    part += __shfl_xor(part, off);
    nlive += __shfl_xor(nlive, off);
  }
  const double kappa = sqrt((double)nlive * part);
  const int good = shift > 0.0 ||
                   (ok && (kappa <= (final ? 2.0 * (double)(nlive > 0 ? nlive : 1) : 1e6)));
#pragma unroll
  for (int k = 0; k < OBW; ++k) Rs[i][k] = acc[k];   // zero beyond nb
  if (write_state) {
    if (i < nb && !final && good) dead[c0 + i] = isdead ? 1 : 0;
    if (i == 0) *healthy = good;
  }
  return good;
}

// The in-block Cholesky QR step: the factorisation of G (chol_factor) and
// U[:, c0 : c0 + nb] <- U[:, c0 : c0 + nb] R^{-1} (row-major, ld kk) when the
// block is healthy, in one launch.  G comes as the splits K slabs of its
// product (gemm_f64_partials; one slab: G itself), which the workgroup sums
// in slab order from 0.0 into LDS (the order the split-K sum kernel takes).
// Each workgroup takes 64 rows of U; its
// first wave factors G (every workgroup the same arithmetic on the same G,
// so the same R^{-1} and verdict; the first workgroup records them), which
// costs no time over one factorisation and saves a launch and a round trip
// of R^{-1} through memory.  While the first wave factors, the other three
// stage the workgroup's rows of the block in LDS.  Apply: the rows
// (transposed) sit in LDS next to R^{-1}, and the four waves form the 64 x 64
// product on the FP64 matrix cores.
// The nfb workgroups after the (m + 63) / 64 of the apply run the first
// level of the Gram-Schmidt fallback instead, chunk blockIdx.x - (m + 63) /
// 64 each, when the block is not healthy (tsqr_local_chunk, arguments q0,
// ldq0, qcols0, r0, top0; its later levels are a launch of their own, whose
// counter, healthy[1], the first workgroup zeroes).  The apply and the
// fallback never both run, so neither reads what the other writes.
constexpr int CHOL_LDS = 2 * OBW * OBP + 2 * OBW * RLD;
static_assert(TSQR_LDS <= CHOL_LDS, "the fallback chunk fits in the Cholesky kernel's LDS");
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void chol_apply_kernel(
    const double* __restrict__ Gp, int splits, int nb, int c0, const double* __restrict__ nrm0,
    int* __restrict__ dead, int final, int* __restrict__ healthy, double shift, double dead_tol,
    double* __restrict__ U, int m, int kk, double* __restrict__ q0, int64_t ldq0, int qcols0,
    double* __restrict__ r0, int top0) {
  __shared__ __align__(16) double L[CHOL_LDS];
  // row j of the trailing matrix as it stood at step j
  double (*Rw)[OBP] = reinterpret_cast<double (*)[OBP]>(L);
  double (*Gs)[OBP] = reinterpret_cast<double (*)[OBP]>(L + OBW * OBP);   // G, zero beyond nb
  // Rs[a][c] = R^{-1}[a][c]; Pt[a][r] = U[i0 + r][c0 + a]
  double (*Rs)[RLD] = reinterpret_cast<double (*)[RLD]>(L + 2 * OBW * OBP);
  double (*Pt)[RLD] = reinterpret_cast<double (*)[RLD]>(L + 2 * OBW * OBP + OBW * RLD);
  __shared__ int good_s, dep_s;
  const int t = threadIdx.x;
  const int napply = (m + 63) / 64;
  {
    // element (r, cc) = (t / 64 + 4 q, t % 64); clamped addresses, so every
    // load is issued and the values beyond nb are dropped
    const int cc = t & 63, ccl = cc < nb ? cc : nb - 1;
    const int64_t nn = (int64_t)nb * nb;
    double g[16];
    if (splits == 1) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r = (t >> 6) + 4 * q;
        g[q] = Gp[(r < nb ? r : nb - 1) * nb + ccl];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) g[q] = 0.0;
      // four slabs' loads in flight before their sums; a slab beyond the
      // last adds 0.0, which leaves the sum bitwise as it is (it starts
      // from +0.0, so it is never -0.0)
      for (int z = 0; z < splits; z += 4) {
        double v[4][16];
#pragma unroll
        for (int zz = 0; zz < 4; ++zz) {
          const bool in = z + zz < splits;
          const double* slab = Gp + (in ? z + zz : z) * nn;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int r = (t >> 6) + 4 * q;
            v[zz][q] = slab[(r < nb ? r : nb - 1) * nb + ccl];
            if (!in) v[zz][q] = 0.0;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int zz = 0; zz < 4; ++zz)
#pragma unroll
          for (int q = 0; q < 16; ++q) g[q] += v[zz][q];
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = (t >> 6) + 4 * q;
      Gs[r][cc] = (r < nb && cc < nb) ? g[q] : 0.0;
    }
  }
  __syncthreads();
  const int i0 = blockIdx.x * 64;
  if (t < 64) {
    const int good = chol_factor(nb, c0, nrm0, dead, final, healthy, shift, dead_tol,
                                 blockIdx.x == 0, Rw, Gs, Rs);
    if (t == 0) good_s = good;
  } else if ((int)blockIdx.x < napply) {
    // meanwhile the other three waves stage the workgroup's rows of the block,
    // transposed: Pt[a][r] = U[i0 + r][c0 + a] (zero beyond m and nb)
    constexpr int PQ = (64 * OBW + 191) / 192;
    double pv[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int e = (t - 64) + 192 * q;
      const int r = e >> 6, cc = e & 63;
      pv[q] = (e < 64 * OBW && i0 + r < m && cc < nb) ? U[(int64_t)(i0 + r) * kk + c0 + cc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int e = (t - 64) + 192 * q;
      if (e < 64 * OBW) Pt[e & 63][e >> 6] = pv[q];
    }
  }
  __syncthreads();
  const int good = good_s;
  if (blockIdx.x == 0 && t == 0) healthy[1] = 0;   // the fallback's counter
  if ((int)blockIdx.x >= napply) {
    if (good) return;
    tsqr_local_chunk(U + c0, m, kk, nb, q0, ldq0, qcols0, r0, top0, nrm0, c0, dead, final,
                     dead_tol, blockIdx.x - napply, L, dep_s);
    return;
  }
  if (!good) return;
  // the product on the FP64 matrix cores: wave w forms the 32 x 32 quadrant
  // (w / 2, w % 2) of the 64 x 64 result as 2 x 2 tiles of 16 x 16, over the
  // 64 inner indices in steps of 4 (R^{-1} and the rows are zero beyond nb)
  const int w = t >> 6, lane = t & 63;
  const int rq = (w >> 1) * 32, cq = (w & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < OBW; k0 += 4) {
    const int kr = k0 + (lane >> 4);
    const double a0 = Pt[kr][rq + (lane & 15)], a1 = Pt[kr][rq + 16 + (lane & 15)];
    const double b0 = Rs[kr][cq + (lane & 15)], b1 = Rs[kr][cq + 16 + (lane & 15)];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // result lane l, element q: row l / 16 + 4 q, column l % 16 of its tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + rq + 16 * i + (lane >> 4) + 4 * q;
        const int col = cq + 16 * j + (lane & 15);
        if (row < m && col < nb) U[(int64_t)row * kk + c0 + col] = acc[i][j][q];
      }
}

// In-place sign fix of the kk columns of row-major U (m x kk): the lowest
// row whose magnitude is within kSignTie of the column's largest is made
// positive.  Zero columns stay zero.
__global__ __launch_bounds__(256) void sign_fix_kernel(double* __restrict__ U, int m, int kk) {
  __shared__ double shm[256];
  __shared__ int shi[256];
  const int t = blockIdx.x;
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) mx = fmax(mx, fabs(U[(int64_t)i * kk + t]));
  shm[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + w]);
    __syncthreads();
  }
  const double top = shm[0];
  if (!(top > 0.0)) return;
  const double thr = (1.0 - kSignTie) * top;
  int lo = 0x7fffffff;
  for (int i = threadIdx.x; i < m; i += 256)
    if (fabs(U[(int64_t)i * kk + t]) >= thr && i < lo) lo = i;
  shi[threadIdx.x] = lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) shi[threadIdx.x] = min(shi[threadIdx.x], shi[threadIdx.x + w]);
    __syncthreads();
  }
  if (U[(int64_t)shi[0] * kk + t] < 0.0)
    for (int i = threadIdx.x; i < m; i += 256) U[(int64_t)i * kk + t] = -U[(int64_t)i * kk + t];
}

// Standard normal numbers from a counter-based generator: splitmix64 of
// (seed, index) gives two uniforms, Box-Muller turns them into a normal.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void gaussian_kernel(double* __restrict__ x, int64_t n,
                                                       uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t a = splitmix64(seed ^ splitmix64(2 * (uint64_t)i));
    const uint64_t b = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 1));
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;   // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;           // [0, 1)
    x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

__global__ void spec_finish_kernel(const double* __restrict__ S, int kk, int chi,
                                   double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= chi) return;
  const double s0 = S[0];
  out[i] = (i < kk && s0 > 0.0) ? S[i] / s0 : 0.0;
}

}  // namespace

namespace {

// The Gram-Schmidt tree for block [c0, c0 + nbk) of A above its first level,
// which the Cholesky kernel runs into q0 (m x OBW, all OBW columns, zeros
// beyond nbk) and r0 (one OBW x OBW factor per chunk of TQ rows); when m
// fits one chunk that level was the whole tree and wrote A itself.  One
// launch (tsqr_upper_kernel), which exits at once when the Cholesky path has
// taken the block; count is its counter, zeroed by the Cholesky kernel.
void tsqr_fallback(Ctx& c, double* A, int m, int kk, int c0, int nbk, const double* nrm0,
                   int* dead, int pass, const int* healthy, double* q0, double* r0, int* count) {
  const int chunks0 = (m + TQ - 1) / TQ;
  if (chunks0 == 1) return;
  const size_t mk = c.arena.mark();
  TreeLevels tl{};
  tl.rows[0] = m;
  tl.q[0] = q0;
  tl.r[0] = r0;
  int rows = chunks0 * OBW, n = 0;
  for (;;) {
    if (++n > kMaxTree) throw Error(1, "orthonormalize: too many rows");   // bad argument
    const int chunks = (rows + TQ - 1) / TQ;
    tl.rows[n] = rows;
    tl.q[n] = (double*)c.arena.alloc(sizeof(double) * (size_t)rows * OBW);
    tl.r[n] = chunks == 1 ? nullptr
                          : (double*)c.arena.alloc(sizeof(double) * (size_t)chunks * OBW * OBW);
    if (chunks == 1) break;
    rows = chunks * OBW;
  }
  tl.n = n;
  for (int l = 1; l < n; ++l)
    tl.w[l] = (double*)c.arena.alloc(sizeof(double) * (size_t)tl.rows[l] * OBW);
  if (!c.dry) {
    // the tree's work when it runs: Gram-Schmidt twice over each level and
    // the products down; it is timed whether or not it runs
    double fl = 0.0, by = 0.0;
    for (int l = 1; l <= n; ++l) fl += 6.0 * tl.rows[l] * (double)nbk * nbk;
    for (int l = 0; l < n; ++l) {
      fl += 2.0 * tl.rows[l] * (double)OBW * nbk;
      by += 8.0 * 3.0 * tl.rows[l] * OBW;
    }
    ProfScope ps(c, K_SVD_OTHER, fl, by);
    hipLaunchKernelGGL(tsqr_upper_kernel, dim3((tl.rows[1] + TQ - 1) / TQ), dim3(256), 0, c.stream,
                       tl, nbk, A, (int64_t)kk, c0, nrm0, dead, pass, healthy, count, dead_tol());
    c.check_launch();
  }
  c.arena.release(mk);
}

// Orthonormalise the kk columns of row-major A (m x kk) in place, in order,
// by block classical Gram-Schmidt applied twice (BCGS2): for each block of 64
// columns, project out the earlier blocks (one GEMM pair), orthonormalise
// inside the block (Cholesky QR when the block is well conditioned, else
// classical Gram-Schmidt twice), and repeat both steps.  With rounds = 1
// (the bases between power steps of the range finder, which need a
// normalised basis of the same span, not one orthonormal to working
// accuracy) the first in-block step is a shifted Cholesky QR.
// The second projection comes after the first in-block normalisation, so a
// nearly dependent column, which shrinks to a small residual inside the
// block, is still made orthogonal to the earlier blocks.  Columns dependent
// to working precision come out as zero columns: the nonzero columns are
// orthonormal and span the columns of A up to rounding.
void orthonormalize(Ctx& c, double* A, int m, int kk, int rounds = 2) {
  constexpr int OB = OBW;
  // one round asked for (the bases between power steps): the block's first
  // factorisation is a shifted Cholesky QR, which cannot fail and keeps the
  // span, and the second a plain one under the first-visit test (orthogonal
  // to ~1e-4 at worst), so the columns come out normalised without the
  // Gram-Schmidt tree in most blocks
  const bool loose = rounds == 1;
  if (loose) rounds = 2;
  const size_t mk = c.arena.mark();
  const int rows = 64;
  const int chunks = (m + rows - 1) / rows;
  double* part = (double*)c.arena.alloc(sizeof(double) * (size_t)chunks * kk);
  double* nrm0 = (double*)c.arena.alloc(sizeof(double) * (size_t)kk);
  int* dead = (int*)c.arena.alloc(sizeof(int) * (size_t)kk);
  double* G = (double*)c.arena.alloc(sizeof(double) * (size_t)kk * OB);
  // the block Gram's split-K slabs (the split depends on m alone: every
  // block has the same K = m and at most OB columns)
  const int gslabs = gemm_f64_split_count(OB, OB, m);
  double* Gp = (double*)c.arena.alloc(sizeof(double) * (size_t)gslabs * OB * OB);
  int* healthy = (int*)c.arena.alloc(sizeof(int) * 2);   // and the fallback's counter
  // the first level of the Gram-Schmidt fallback (run by the Cholesky
  // kernel): Q and R factors of its chunks when there are several
  const int chunks0 = (m + TQ - 1) / TQ;
  double* q0 = chunks0 > 1 ? (double*)c.arena.alloc(sizeof(double) * (size_t)m * OB) : nullptr;
  double* r0 =
      chunks0 > 1 ? (double*)c.arena.alloc(sizeof(double) * (size_t)chunks0 * OB * OB) : nullptr;
  if (!c.dry) {
    ProfScope ps(c, K_SVD_OTHER, 0.0, 8.0 * (double)m * kk);
    hipLaunchKernelGGL(rm_colsq_kernel, dim3((kk + 255) / 256, chunks), dim3(256), 0, c.stream, A,
                       m, kk, rows, part);
    hipLaunchKernelGGL(rm_colnorm_kernel, dim3((kk + 255) / 256), dim3(256), 0, c.stream, part,
                       chunks, kk, nrm0);
    c.check_launch();
  }
  for (int c0 = 0; c0 < kk; c0 += OB) {
    const int nbk = std::min(OB, kk - c0);
    for (int pass = 0; pass < rounds; ++pass) {
      if (c0 > 0) {
        gemm(c, F64, c0, nbk, m, 1.0, A, kk, 1, A + c0, kk, 0, 0.0, G, nbk);
        gemm(c, F64, m, nbk, c0, -1.0, A, kk, 0, G, nbk, 0, 1.0, A + c0, kk);
      }
      // in-block: Cholesky QR of the block when it is well conditioned,
      // classical Gram-Schmidt twice otherwise (decided on the device)
      const int gsplits = gemm_f64_partials(c, nbk, nbk, m, A + c0, kk, 1, A + c0, kk, 0, Gp);
      if (gsplits > gslabs) throw Error(2, "orthonormalize: Gram slabs beyond their buffer");
      if (!c.dry) {
        const bool shifted = loose && pass == 0;
        // Cholesky nb^3 / 3 and triangular inverse nb^3 / 3 flop (once: the
        // workgroups repeat it side by side), apply m nb^2; the slabs of G
        // in, the block read and written
        const double b3 = (double)nbk * nbk * nbk;
        ProfScope ps(c, K_CHOL, 2.0 * b3 / 3.0 + (double)m * nbk * nbk,
                     8.0 * ((double)gsplits * nbk * nbk + 2.0 * m * nbk), 1, true);
        // the shifted factorisation cannot fail: no fallback workgroups
        const int nfb = shifted ? 0 : chunks0;
        const bool one = chunks0 == 1;
        launch(ps, chol_apply_kernel, dim3((m + 63) / 64 + nfb), dim3(256), c.stream,
               (const double*)Gp, gsplits, nbk, c0, (const double*)nrm0, dead, loose ? 0 : pass,
               healthy, shifted ? 1e-12 : 0.0, dead_tol(), A, m, kk, one ? A + c0 : q0,
               (int64_t)(one ? kk : OB), one ? nbk : OB, r0, one ? 1 : 0);
        c.check_launch();
      }
      if (!(loose && pass == 0))
        tsqr_fallback(c, A, m, kk, c0, nbk, nrm0, dead, loose ? 0 : pass, healthy, q0, r0,
                      healthy + 1);
    }
  }
  c.arena.release(mk);
}

void sign_fix(Ctx& c, double* U, int m, int kk) {
  if (c.dry || kk <= 0) return;
  ProfScope ps(c, K_SVD_OTHER, 0.0, 16.0 * m * kk);
  hipLaunchKernelGGL(sign_fix_kernel, dim3(kk), dim3(256), 0, c.stream, U, m, kk);
  c.check_launch();
}

unsigned grid_for(int64_t n, int64_t cap) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

// Q = orthonormalised columns of row-major A (m x n), taken in order of
// decreasing column norm (ties by index): A P = Q R.
void orth_sorted(Ctx& c, const double* A, int m, int n, double* Q) {
  const size_t mk = c.arena.mark();
  const int rows = 64;
  const int chunks = (m + rows - 1) / rows;
  double* part = (double*)c.arena.alloc(sizeof(double) * (size_t)chunks * n);
  double* sig = (double*)c.arena.alloc(sizeof(double) * (size_t)n);
  int* order = (int*)c.arena.alloc(sizeof(int) * (size_t)n);
  if (!c.dry) {
    ProfScope ps(c, K_SVD_OTHER, 0.0, 16.0 * (double)m * n);
    hipLaunchKernelGGL(rm_colsq_kernel, dim3((n + 255) / 256, chunks), dim3(256), 0, c.stream, A,
                       m, n, rows, part);
    hipLaunchKernelGGL(rm_colnorm_kernel, dim3((n + 255) / 256), dim3(256), 0, c.stream, part,
                       chunks, n, sig);
    hipLaunchKernelGGL(jac_rank_kernel, dim3((n + 63) / 64), dim3(256), 0, c.stream, sig, n, n,
                       order);
    hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for((int64_t)m * n, 8192)), dim3(256), 0,
                       c.stream, A, m, n, order, Q);
    c.check_launch();
  }
  orthonormalize(c, Q, m, n);
  c.arena.release(mk);
}

// Truncated SVD of row-major M (m x n, m >= n): U (m x kk), S (kk).
void tsvd_core(Ctx& c, const double* M, int m, int n, int k, double tau, double* U, double* S) {
  const int kk = std::min(k, n);
  if (kk <= 0) return;
  const int r = n;                  // X = R^T is n x n
  int nb = (n + JW - 1) / JW;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  const int cp = nb * JW;
  const size_t mk = c.arena.mark();
  double* Q = (double*)c.arena.alloc(sizeof(double) * (size_t)m * n);
  double* X = (double*)c.arena.alloc(sizeof(double) * (size_t)r * cp);
  double* V = (double*)c.arena.alloc(sizeof(double) * (size_t)n * cp);
  double* sig = (double*)c.arena.alloc(sizeof(double) * (size_t)cp);
  int* order = (int*)c.arena.alloc(sizeof(int) * (size_t)kk);
  int* flags = (int*)c.arena.alloc(4 * sizeof(int));
  double* fro = (double*)c.arena.alloc(sizeof(double));
  double* Uj = (double*)c.arena.alloc(sizeof(double) * (size_t)n * kk);
  double* A1 = (double*)c.arena.alloc(sizeof(double) * (size_t)n * n);
  double* Q2 = (double*)c.arena.alloc(sizeof(double) * (size_t)n * n);
  double* A2 = (double*)c.arena.alloc(sizeof(double) * (size_t)n * n);
  double* Q3 = (double*)c.arena.alloc(sizeof(double) * (size_t)n * n);
  orth_sorted(c, M, m, n, Q);
  // Preconditioning (all matrices row-major).  M P1 = Q R1 with the column
  // order P1 of orth_sorted; A1 = M^T Q = P1 R1^T, so M = Q A1^T.  Two more
  // norm-ordered QR steps of the square factor: A1 P2 = Q2 R2 gives
  // A1^T = A2 Q2^T with A2 = A1^T Q2 (= P2 R2^T), and A2 P3 = Q3 R3 gives
  // A2 = Q3 A3^T with A3 = A2^T Q3.  So M = Q Q3 A3^T Q2^T, and the one-sided
  // Jacobi method on the columns of A3 (A3 J = W Sigma) yields
  // U = Q Q3 J.  Each step R -> R^T and back is a step of the Cholesky LR
  // iteration on the column Gram matrix (R^T R -> R R^T): it moves weight to
  // the diagonal, so the sweeps that follow are fewer (on the move's
  // 256 x 256 truncation inputs 13 -> 5 sweeps for the row M', 9 -> 6 for a
  // side product).  The Jacobi input is A3 in column-major order, i.e. the
  // row-major product Q3^T A2.
  gemm(c, F64, n, n, m, 1.0, M, n, 1, Q, n, 0, 0.0, A1, n);              // A1 = M^T Q
  orth_sorted(c, A1, n, n, Q2);
  gemm(c, F64, n, n, n, 1.0, A1, n, 1, Q2, n, 0, 0.0, A2, n);            // A2 = A1^T Q2
  orth_sorted(c, A2, n, n, Q3);
  gemm(c, F64, n, n, n, 1.0, Q3, n, 1, A2, n, 0, 0.0, X, n);             // X = Q3^T A2
  if (cp > n) fill(c, X + (size_t)n * n, F64, (int64_t)(cp - n) * n, 0.0);
  norm2(c, X, (int64_t)n * n, fro);
  if (!c.dry) {
    hipLaunchKernelGGL(eye_kernel, dim3(grid_for((int64_t)n * cp, 4096)), dim3(256), 0, c.stream,
                       V, n, cp);
    hipLaunchKernelGGL(jac_flags_init, dim3(1), dim3(1), 0, c.stream, flags);
    const double eps = 2.220446049250313e-16;
    // relative orthogonality test r eps and absolute floor eps ||M||_F / 4
    // (CTM_DEBUG_JAC_TOL / CTM_DEBUG_JAC_THR override the two multipliers
    // for measurements)
    double tolf = std::max((double)r, 4.0), thr_mult = 0.25;
    if (const char* v = std::getenv("CTM_DEBUG_JAC_TOL")) tolf = std::max(2.0, std::atof(v));
    if (const char* v = std::getenv("CTM_DEBUG_JAC_THR")) thr_mult = std::atof(v);
    const double tol = tolf * eps;
    // inner test strictly below the outer one, so a block the inner solve
    // leaves converged also passes the outer test
    const double tol_in = std::min(32.0, 0.5 * tolf) * eps;
    const int inner_sweeps = 1;
    // CTM_DEBUG_MAX_SWEEPS lowers the cap (tests of the non-convergence status)
    int max_sweeps = 14;
    if (const char* ms = std::getenv("CTM_DEBUG_MAX_SWEEPS")) max_sweeps = std::max(1, std::min(14, std::atoi(ms)));
    // XCD of this SVD's Jacobi rounds (concurrent SVDs have their buffers
    // megabytes apart, so they mostly land on different XCDs)
    const int xslot = (int)(((uintptr_t)X >> 20) & 7);
    // the first sweeps one launch per round; the rest, which converged
    // sweeps make no-ops, in one launch (CTM_DEBUG_PAR_SWEEPS moves the split
    // for the tests of that launch)
    int par_sweeps = 8;
    if (const char* ps = std::getenv("CTM_DEBUG_PAR_SWEEPS")) par_sweeps = std::max(1, std::atoi(ps));
    par_sweeps = std::min(par_sweeps, max_sweeps);
    for (int sw = 0; sw < par_sweeps; ++sw) {
      for (int rd = 0; rd < nb - 1; ++rd) {
        // each round timed by its own dispatch; its work is data dependent,
        // so the kernel tallies it on the device
        ProfScope ps(c, K_SVD_ROUND, 0.0, 0.0, 1, true);
        launch(ps, jac_round_kernel, dim3(8 * (nb / 2)), dim3(256), c.stream, X, r, (int64_t)r, V,
               n, nb, rd, tol, tol_in, inner_sweeps, fro, flags, c.prof ? c.work : nullptr, xslot,
               thr_mult);
      }
      hipLaunchKernelGGL(jac_sweep_end, dim3(1), dim3(1), 0, c.stream, flags);
    }
    if (max_sweeps > par_sweeps) {
      ProfScope ps(c, K_SVD_ROUND, 0.0, 0.0, 1, true);
      launch(ps, jac_late_kernel, dim3(1), dim3(256), c.stream, X, r, (int64_t)r, V, n, nb, tol,
             tol_in, inner_sweeps, fro, flags, c.prof ? c.work : nullptr, thr_mult,
             max_sweeps - par_sweeps);
    }
    if (c.dev_flags)
      hipLaunchKernelGGL(jac_converged_check, dim3(1), dim3(1), 0, c.stream, flags, c.dev_flags);
    if (std::getenv("CTM_DEBUG_SWEEPS")) {   // diagnostics only: blocks the host
      int f[3] = {0, 0, 0};
      c.check(hipMemcpyAsync(f, flags, sizeof(f), hipMemcpyDeviceToHost, c.stream));
      c.check(hipStreamSynchronize(c.stream));
      std::fprintf(stderr, "tsvd_core m=%d n=%d: %d rotating sweeps, converged %d\n", m, n, f[2],
                   f[0]);
    }
    ProfScope ps(c, K_SVD_OTHER, 0.0, 8.0 * (double)r * cp + 16.0 * (double)n * kk);
    hipLaunchKernelGGL(jac_colnorm_kernel, dim3(cp), dim3(256), 0, c.stream, X, r, cp, sig);
    hipLaunchKernelGGL(jac_rank_kernel, dim3((cp + 63) / 64), dim3(256), 0, c.stream, sig, cp,
                       kk, order);
    hipLaunchKernelGGL(jac_pick_kernel, dim3(grid_for((int64_t)n * kk, 4096)), dim3(256), 0,
                       c.stream, V, n, cp, sig, order, kk, tau, Uj, S);
    c.check_launch();
  }
  gemm(c, F64, n, kk, n, 1.0, Q3, n, 0, Uj, kk, 0, 0.0, A1, kk);        // Q3 J
  gemm(c, F64, m, kk, n, 1.0, Q, n, 0, A1, kk, 0, 0.0, U, kk);          // U = Q Q3 J
  sign_fix(c, U, m, kk);
  c.arena.release(mk);
}

// Left singular vectors of a wide M (m < n): M^T P = Q1 R1 gives
// M = P R1^T Q1^T, so L = M Q1 (m x m) has the left singular vectors and
// singular values of M.
void tsvd_wide(Ctx& c, const double* M, int m, int n, int k, double tau, double* U, double* S) {
  const size_t mk = c.arena.mark();
  double* MT = (double*)c.arena.alloc(sizeof(double) * (size_t)m * n);
  double* Q1 = (double*)c.arena.alloc(sizeof(double) * (size_t)n * m);
  double* L = (double*)c.arena.alloc(sizeof(double) * (size_t)m * m);
  {
    Tensor tM = make_view((void*)M, F64, {m, n}), tT = make_view(MT, F64, {n, m});
    const int pr[2] = {1, 0};
    permute(c, tM, pr, tT);
  }
  orth_sorted(c, MT, n, m, Q1);
  gemm(c, F64, m, m, n, 1.0, M, n, 0, Q1, m, 0, 0.0, L, m);             // L = M Q1
  tsvd_core(c, L, m, m, k, tau, U, S);
  c.arena.release(mk);
}

}  // namespace

// Dispatch: large problems are first narrowed to a small factor whose SVD the
// preconditioned Jacobi method then takes.
//  - 128 <= k <= min(m, n) / 4 with min(m, n) >= 768: randomised range finder
//    with one power iteration (subspace of b = 2k columns, Gaussian test
//    matrix from a counter-based generator);
//    with Y = Q the range basis, B = Q^T M is wide and B^T = M^T Q; then
//    L = B Q_B from the QR of B^T is b x b with the left singular vectors of
//    B, and U = Q U_L.
//  - m >= n: QR-preconditioned Jacobi on M.
//  - m < n: reduction to the square L = M Q_1 first.
void tsvd(Ctx& c, const double* M, int m, int n, int k, double tau, double* U, double* S) {
  const int mn = std::min(m, n);
  const int kk = std::min(k, mn);
  if (kk <= 0) return;
  if (mn >= 768 && kk >= 128 && kk <= mn / 4) {
    // oversampling p = k: on the move's own truncation inputs (spectra of
    // the side product and of M' at D = 6 and 8) one power step on a 2k
    // subspace gives every kept singular value to rounding and the kept
    // projector to ~1e-12 of ||M||; with p = k / 4 the side product at
    // D = 6 kept only ~1e-10 and ~2e-8
    const int b = std::min(mn, 2 * kk);
    const size_t mk = c.arena.mark();
    double* Y = (double*)c.arena.alloc(sizeof(double) * (size_t)m * b);
    double* Z = (double*)c.arena.alloc(sizeof(double) * (size_t)n * b);
    double* QB = (double*)c.arena.alloc(sizeof(double) * (size_t)n * b);
    double* L = (double*)c.arena.alloc(sizeof(double) * (size_t)b * b);
    double* UL = (double*)c.arena.alloc(sizeof(double) * (size_t)b * kk);
    if (!c.dry) {
      const uint64_t seed = 0x5eedull + 0x100000001b3ull * (uint64_t)(++c.rng_calls);
      hipLaunchKernelGGL(gaussian_kernel, dim3(grid_for((int64_t)n * b, 4096)), dim3(256), 0,
                         c.stream, Z, (int64_t)n * b, seed);
      c.check_launch();
    }
    gemm(c, F64, m, b, n, 1.0, M, n, 0, Z, b, 0, 0.0, Y, b);            // Y = M Om
    // one power step; it only needs a well-conditioned basis: one
    // Gram-Schmidt round (orthogonal to ~1e-4 at worst) instead of two
    for (int it = 0; it < 1; ++it) {
      orthonormalize(c, Y, m, b, 1);
      gemm(c, F64, n, b, m, 1.0, M, n, 1, Y, b, 0, 0.0, Z, b);          // Z = M^T Y
      orthonormalize(c, Z, n, b, 1);
      gemm(c, F64, m, b, n, 1.0, M, n, 0, Z, b, 0, 0.0, Y, b);          // Y = M Z
    }
    orthonormalize(c, Y, m, b);                              // Q
    gemm(c, F64, n, b, m, 1.0, M, n, 1, Y, b, 0, 0.0, Z, b);            // B^T = M^T Q
    orth_sorted(c, Z, n, b, QB);                                         // B^T P = Q_B R
    gemm(c, F64, b, b, n, 1.0, Z, b, 1, QB, b, 0, 0.0, L, b);           // L = B Q_B
    tsvd_core(c, L, b, b, kk, tau, UL, S);
    gemm(c, F64, m, kk, b, 1.0, Y, b, 0, UL, kk, 0, 0.0, U, kk);        // U = Q U_L
    sign_fix(c, U, m, kk);
    c.arena.release(mk);
    return;
  }
  if (m >= n)
    tsvd_core(c, M, m, n, k, tau, U, S);
  else
    tsvd_wide(c, M, m, n, k, tau, U, S);
}

void range_basis(Ctx& c, const double* M, int m, int n, double* Q) { orth_sorted(c, M, m, n, Q); }

void corner_spectrum(Ctx& c, const double* C, int p, int q, int chi, double* out) {
  const int kk = std::min(chi, std::min(p, q));
  const size_t mk = c.arena.mark();
  double* U = (double*)c.arena.alloc((size_t)p * std::max(kk, 1) * sizeof(double));
  double* S = (double*)c.arena.alloc((size_t)std::max(kk, 1) * sizeof(double));
  tsvd(c, C, p, q, chi, 0.0, U, S);
  if (!c.dry) {
    hipLaunchKernelGGL(spec_finish_kernel, dim3((chi + 255) / 256), dim3(256), 0, c.stream, S, kk,
                       chi, out);
    c.check_launch();
  }
  c.arena.release(mk);
}

}  // namespace ctm

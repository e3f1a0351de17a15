// Corner-transfer solver: schedule of one move and the C-ABI entry points.
//
// Every step runs in this library's kernels (GEMM, permute, SVD, norms); the
// host only sequences launches on the solver's stream and tracks bond
// dimensions, which are fixed by shapes alone (a truncation of an m x n
// matrix to k keeps min(k, m, n) columns), so no host round trip is needed
// inside a move.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <exception>
#include <stdexcept>
#include <thread>
#include <vector>

#include "../../include/ctm.h"
#include "ctm_internal.h"

using namespace ctm;

struct ctm_solver {
  Ctx ctx;
  int d = 2, D = 1, chi = 1, method = CTM_REDUCED, precision = CTM_FP64, boot_iters = 1;
  // first-stage bonds of the sequential-order split: chi_p of the anchors'
  // v^1 (Sec. IV), chi_pp of the helper isometries v_l^1, v_r^1 (App.)
  int chi_p = 1, chi_pp = 1;
  double tau = 1e-14;
  int cap = 1;        // largest bond dimension any tensor can take
  int moves = 0;
  double* env[16] = {nullptr};
  int pd[16] = {0}, qd[16] = {0};
  double* site[2] = {nullptr, nullptr};
  double* site_rot[4][2] = {};
  void* sT1[4][2] = {};
  void* sT2[4][2] = {};
  double* spec[2] = {nullptr, nullptr};
  int spec_cur = 0;
  bool spec_valid = false;
  double* scal = nullptr;    // device scalars
  double* h4 = nullptr;      // device d^4 operator
  size_t persist = 0;
  Profiler prof;
  // independent truncations of one insertion run concurrently on these
  // streams (default priority), forked from and joined to ctx.stream
  static constexpr int kAux = 4, kMaxBranch = 8;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kMaxBranch] = {};
  // moves replayed from captured HIP graphs, keyed by everything the launch
  // sequence of a move depends on (see run_move)
  bool graphs = true;
  std::string move_tag;   // key of the move being issued ("" = no replay)
  int branch_call = 0;    // run_branches calls so far in that move
  std::map<std::string, hipGraphExec_t> gexec;
  std::map<std::string, int> gseen;
  void drop_graphs() {
    for (auto& kv : gexec) (void)hipGraphExecDestroy(kv.second);
    gexec.clear();
    gseen.clear();
  }
  ~ctm_solver() {
    drop_graphs();
    for (hipStream_t& st : aux)
      if (st) (void)hipStreamDestroy(st);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (hipEvent_t& e : ev_join)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr int kC = 0, kT = 1;
constexpr int kMaxCorrLength = 4096;   // longest row of ctm_row_correlation

inline int env_index(int kind, int i, int z) { return 8 * kind + 2 * (i - 1) + z; }
inline int stored_i(int i, int r) { return (i - 1 + r) % 4 + 1; }

int cdt(const ctm_solver* s) {
  return s->precision == CTM_FP64 ? F64 : (s->precision == CTM_FP32 ? F32 : BF16);
}

Tensor env_view(ctm_solver* s, int kind, int role_i, int z, int r) {
  const int e = env_index(kind, stored_i(role_i, r), z);
  if (kind == kC) return make_view(s->env[e], F64, {s->pd[e], s->qd[e]});
  return make_view(s->env[e], F64, {s->pd[e], s->D, s->D, s->qd[e]});
}

Tensor site_view(ctm_solver* s, int r, int z) {
  const int64_t d = s->d, D = s->D;
  return make_view(s->site_rot[r][z], F64, {d, D, D, D, D});
}

// Copy t to dst and return the view at dst (device to device, stream ordered).
Tensor keep(Ctx& c, const Tensor& t, void* dst) {
  Tensor out = t;
  out.p = dst;
  if (!c.dry && t.p != dst && t.bytes() > 0) {
    ProfScope ps(c, K_COPY, 0.0, 2.0 * t.bytes());
    copy_bytes(c, dst, t.p, t.bytes());
  }
  return out;
}

Tensor reshape(const Tensor& t, std::initializer_list<int64_t> dims) {
  Tensor o = make_view(t.p, t.dt, dims);
  if (o.numel() != t.numel()) throw std::runtime_error("reshape: size mismatch");
  return o;
}

// Runs independent pieces of work concurrently.  Each branch gets its own
// slice of the workspace (sized by a dry run of the branch), its own stream
// and its own range of random-generator calls, so its kernels and results do
// not depend on the other branches or on their timing.  Branches write their
// results into buffers the caller allocated before the fork.
void run_branches(ctm_solver* s, const std::vector<std::function<void(Ctx&)>>& fs) {
  Ctx& c = s->ctx;
  const int n = (int)fs.size();
  if (n > ctm_solver::kMaxBranch) throw std::runtime_error("too many branches");
  std::vector<size_t> need(n);
  for (int b = 0; b < n; ++b) {
    Ctx d;
    d.dry = true;
    d.arena.dry = true;
    fs[b](d);
    need[b] = d.arena.peak + 256;
  }
  // the slices are released on return: every later use of that memory is
  // ordered after the join on ctx.stream.  With CTM_DEBUG_GUARD set, each
  // slice is followed by a guard region checked after the join (a write
  // past a slice would land in the next branch's memory and make results
  // depend on timing); a hit sets bit 4 of the error word.
  const bool guard = std::getenv("CTM_DEBUG_GUARD") != nullptr;
  const size_t gbytes = guard ? ((size_t)1 << 16) : 0;
  const size_t mk = c.arena.mark();
  std::vector<char*> base(n), gbase(n);
  for (int b = 0; b < n; ++b) {
    base[b] = (char*)c.arena.alloc(need[b]);
    gbase[b] = gbytes ? (char*)c.arena.alloc(gbytes) : nullptr;
  }
  if (gbytes && !c.dry)
    for (int b = 0; b < n; ++b) guard_fill(c, gbase[b], gbytes);
  if (c.dry && std::getenv("CTM_DEBUG_MEM"))
    for (int b = 0; b < n; ++b)
      std::fprintf(stderr, "  branch %d/%d needs %.1f MB (top %.1f MB)\n", b, n, need[b] / 1e6,
                   c.arena.top / 1e6);
  const uint64_t r0 = c.rng_calls;
  c.rng_calls = r0 + 64 * (uint64_t)(n + 1);
  if (c.dry || c.arena.overflow) {
    c.arena.release(mk);
    return;
  }
  // CTM_DEBUG_SERIAL_BRANCHES runs the branches one after the other on the
  // solver's stream (determinism diagnostics)
  const bool par = s->ev_fork != nullptr && !std::getenv("CTM_DEBUG_SERIAL_BRANCHES");
  if (par) c.check(hipEventRecord(s->ev_fork, c.stream));
  std::vector<Ctx> ks(n);
  for (int b = 0; b < n; ++b) {
    Ctx& k = ks[b];
    k.stream = par ? s->aux[b % ctm_solver::kAux] : c.stream;
    k.prof = c.prof;
    k.dev_flags = c.dev_flags;
    k.work = c.work;
    k.arena.base = base[b];
    k.arena.cap = need[b];
    k.rng_calls = r0 + 64 * (uint64_t)(b + 1);
  }
  // A branch whose key (the move's key, this fork point and the branch) has
  // come up before is captured into a HIP graph on its stream and replayed
  // from then on: the branch function then runs in dry mode over the same
  // workspace slice, which reproduces its host-side results (shapes and
  // buffer addresses of its outputs) without a launch.  The fork and join
  // stay eager, so replayed branches still run concurrently.
  const bool replay = par && !s->move_tag.empty() && c.prof == nullptr;
  const int call = s->branch_call++;
  auto issue = [&](int b) {
    Ctx& k = ks[b];
    if (par) k.check(hipStreamWaitEvent(k.stream, s->ev_fork, 0));
    hipGraphExec_t ex = nullptr;
    std::string key;
    if (replay) {
      key = s->move_tag + "#" + std::to_string(call) + "." + std::to_string(b);
      auto it = s->gexec.find(key);
      if (it != s->gexec.end()) ex = it->second;
    }
    if (ex != nullptr) {
      k.dry = true;
      fs[b](k);
      k.dry = false;
      k.check(hipGraphLaunch(ex, k.stream));
    } else if (replay && s->gseen[key] >= 1) {
      hipGraph_t g = nullptr;
      k.check(hipStreamBeginCapture(k.stream, hipStreamCaptureModeRelaxed));
      try {
        fs[b](k);
      } catch (...) {
        (void)hipStreamEndCapture(k.stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      k.check(hipStreamEndCapture(k.stream, &g));
      if (g != nullptr && k.hip_err == hipSuccess) k.check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      if (g) (void)hipGraphDestroy(g);
      if (ex == nullptr) throw Error(CTM_EHIP, "branch capture failed");
      s->gexec[key] = ex;
      k.check(hipGraphLaunch(ex, k.stream));
    } else {
      if (replay) s->gseen[key] += 1;
      fs[b](k);
    }
    if (par) k.check(hipEventRecord(s->ev_join[b], k.stream));
  };
  // each branch is issued from its own host thread (kernel launches cost
  // host time, and the branches share no host state); with the profiler on,
  // or when a branch is captured or seen for the first time (the graph maps
  // are shared), they are issued in order from this thread
  bool threads = par && c.prof == nullptr && n > 1;
  if (replay)
    for (int b = 0; b < n && threads; ++b)
      if (!s->gexec.count(s->move_tag + "#" + std::to_string(call) + "." + std::to_string(b)))
        threads = false;
  std::vector<std::exception_ptr> errs(n);
  if (threads) {
    std::vector<std::thread> th;
    for (int b = 1; b < n; ++b)
      th.emplace_back([&, b] {
        try {
          issue(b);
        } catch (...) {
          errs[b] = std::current_exception();
        }
      });
    try {
      issue(0);
    } catch (...) {
      errs[0] = std::current_exception();
    }
    for (std::thread& t : th) t.join();
  } else {
    for (int b = 0; b < n; ++b) issue(b);
  }
  for (int b = 0; b < n; ++b) {
    c.check(ks[b].hip_err);
    if (ks[b].arena.overflow) c.arena.overflow = true;
  }
  if (par)
    for (int b = 0; b < n; ++b) c.check(hipStreamWaitEvent(c.stream, s->ev_join[b], 0));
  if (gbytes)
    for (int b = 0; b < n; ++b) guard_check(c, gbase[b], gbytes);
  c.arena.release(mk);
  for (int b = 0; b < n; ++b)
    if (errs[b]) std::rethrow_exception(errs[b]);
}

// Truncated isometry of a row-major m x n F64 matrix: U (m x kk) at dst,
// kk = min(k, m, n) (k = chi unless given).
Tensor isometry(ctm_solver* s, Ctx& c, const Tensor& M, int64_t m, int64_t n, void* dst,
                int k = 0) {
  if (k <= 0) k = s->chi;
  const int kk = (int)std::min<int64_t>(k, std::min(m, n));
  const size_t mk = c.arena.mark();
  double* S = (double*)c.arena.alloc(sizeof(double) * std::max(kk, 1));
  tsvd(c, M.d(), (int)m, (int)n, k, s->tau, (double*)dst, S);
  c.arena.release(mk);
  return make_view(dst, F64, {m, kk});
}

Tensor double_layer(Ctx& c, const Tensor& S) {
  return contract(c, S, "slurd", S, "sLURD", "lLuUrRdD", F64, F64);
}

// ---------------------------------------------------------------- anchors

// Standard 4-index isometry v_z[j, kd, bd, nu] (Sec. II, Fig. 2(c)).
Tensor anchor_standard(ctm_solver* s, Ctx& c, int r, int z, void* dst) {
  const int w = 1 - z;
  const int64_t D = s->D;
  Tensor C1 = env_view(s, kC, 1, z, r), T1 = env_view(s, kT, 1, z, r), T2 = env_view(s, kT, 2, z, r);
  Tensor T2w = env_view(s, kT, 2, w, r), C2w = env_view(s, kC, 2, w, r), T3w = env_view(s, kT, 3, w, r);
  const int64_t nj = T1.dims[0], nq = T2.dims[3], nj2 = T3w.dims[3];
  const size_t mk = c.arena.mark();
  Tensor az = double_layer(c, site_view(s, r, z));
  Tensor X = contract(c, C1, "mn", T2, "nuvq", "muvq", F64, F64);
  Tensor Y = contract(c, T1, "jklm", X, "muvq", "jkluvq", F64, F64);
  Tensor Q1 = contract(c, Y, "jkluvq", az, "kluvrRdD", "jdDqrR", F64, F64);
  Tensor aw = double_layer(c, site_view(s, r, w));
  Tensor X2 = contract(c, T2w, "quvn", C2w, "nm", "quvm", F64, F64);
  Tensor Y2 = contract(c, X2, "quvm", T3w, "mrRj", "quvrRj", F64, F64);
  Tensor Q2 = contract(c, Y2, "quvrRj", aw, "lLuvrRdD", "qlLdDj", F64, F64);
  const int64_t m = nj * D * D, k = nq * D * D, n = D * D * nj2;
  Tensor M = c.alloc(F64, {m, n});
  gemm(c, F64, (int)m, (int)n, (int)k, 1.0, Q1.p, k, 0, Q2.p, n, 0, 0.0, M.p, n);
  Tensor U = isometry(s, c, M, m, n, dst);
  c.arena.release(mk);
  return make_view(dst, F64, {nj, D, D, U.dims[1]});
}

// Reduced-env 4-index isometry v_z[j, kd, bd, nu] (Sec. III, Fig. 3(a,b)):
// in a converged environment the right half of the half-plaquette,
// {w, T2_w, C2_w, T3_w}, is stood in for by the anchor's own {C2_z, T3_z}
// (the right move's isometry that would follow is dropped: multiplying by a
// co-isometry from the right leaves the left singular vectors unchanged).
// The reduced half-network [C1 T2 C2; T1 z T3] is contracted with the ket
// layer of z before the bra layer, so it costs chi^3 D^4 + chi^2 D^6 d,
// reshaped (chi D^2) x chi and truncated to its top chi left singular
// vectors.
Tensor anchor_reduced_env(ctm_solver* s, Ctx& c, int r, int z, void* dst) {
  const int64_t D = s->D;
  Tensor C1 = env_view(s, kC, 1, z, r), T1 = env_view(s, kT, 1, z, r), T2 = env_view(s, kT, 2, z, r);
  Tensor C2 = env_view(s, kC, 2, z, r), T3 = env_view(s, kT, 3, z, r);
  const int64_t nj = T1.dims[0], nj2 = T3.dims[3];
  const size_t mk = c.arena.mark();
  Tensor Az = site_view(s, r, z);
  Tensor L = contract(c, C1, "mi", T1, "jklm", "iklj", F64, F64);
  Tensor R = contract(c, C2, "im", T3, "mklj", "iklj", F64, F64);
  Tensor X = contract(c, L, "iklj", T2, "iuvn", "kljuvn", F64, F64);
  X = contract(c, X, "kljuvn", Az, "skurd", "ljvnsrd", F64, F64);     // ket layer
  X = contract(c, X, "ljvnsrd", Az, "slvRD", "jnrdRD", F64, F64);     // bra layer
  Tensor M = contract(c, X, "jnrdRD", R, "nrRk", "jdDk", F64, F64);
  Tensor U = isometry(s, c, M, nj * D * D, nj2, dst);
  c.arena.release(mk);
  return make_view(dst, F64, {nj, D, D, U.dims[1]});
}

// Absorption of one site into an edge with 4-index isometries on both bonds
// (Sec. II, Fig. 2(b)), ket layer then bra layer: T[p,k,b,q] with the
// q-side bond (q, ku, bu) truncated by vq[q,u,v,n] and the p-side bond
// (p, kd, bd) by vp[p,d,D,m]; site A[s,l,u,r,d] of the frame, its l leg on
// T's (k, b).  Returns out[m, kr, br, n] in F64; the contractions run in
// the compute type cp (chi^3 D^4 + chi^2 D^6 d, no double-layer tensor).
Tensor absorb4(Ctx& c, const Tensor& T, const Tensor& A, const Tensor& vp, const Tensor& vq, int cp) {
  Tensor Z = contract(c, T, "pklq", vq, "quvn", "pkluvn", cp, cp);
  Z = contract(c, Z, "pkluvn", A, "skurd", "plvnsrd", cp, cp);         // ket layer
  Z = contract(c, Z, "plvnsrd", A, "slvRD", "pnrdRD", cp, cp);         // bra layer
  return contract(c, Z, "pnrdRD", vp, "pdDm", "mrRn", cp, F64);
}

// Two-stage isometry of X[i,k,b,j] (bonded on (i,k,b)): v1 [i,k,mu], v2
// [mu,b,nu], X''[nu,j] (Appendix, Fig. A(c)).  Outputs at the given buffers.
//
// The side isometries enter the move only through M' = C'1 T'2 C'2, where
// the second-stage bond nu is summed over between X'' = v2^T X' and the v2
// of the absorption chain: M' depends on v2 only through the projector
// v2 v2^T.  When the second stage keeps every column (chi >= the columns of
// X', cutoff at rounding level) that projector is the one onto the range of
// X', so any orthonormal basis of the range serves: the norm-ordered QR
// basis that the SVD would start from, without its Jacobi sweeps.
void split_iso(ctm_solver* s, Ctx& c, const Tensor& X, void* d1, void* d2, void* dxx,
               Tensor* v1o, Tensor* v2o, Tensor* xxo) {
  const int64_t ni = X.dims[0], D = X.dims[1], nj = X.dims[3];
  const size_t mk = c.arena.mark();
  Tensor v1 = isometry(s, c, X, ni * D, D * nj, d1, s->chi_pp);
  const int64_t c1 = v1.dims[1];
  v1 = reshape(v1, {ni, D, c1});
  Tensor Xp = contract(c, v1, "ikm", X, "iklj", "mlj", F64, F64);
  const bool full_range = s->chi >= nj && c1 * D >= nj && s->tau <= 1e-12;
  Tensor v2;
  if (full_range) {
    range_basis(c, Xp.d(), (int)(c1 * D), (int)nj, (double*)d2);
    v2 = make_view(d2, F64, {c1 * D, nj});
  } else {
    v2 = isometry(s, c, Xp, c1 * D, nj, d2);
  }
  const int64_t c2 = v2.dims[1];
  v2 = reshape(v2, {c1, D, c2});
  Tensor Xpp = contract(c, v2, "mln", Xp, "mlj", "nj", F64, F64);
  *xxo = keep(c, Xpp, dxx);
  c.arena.release(mk);
  *v1o = v1;
  *v2o = v2;
}

// Sequential ket-then-bra absorption of one site into an edge (Sec. IV,
// Fig. 4(b)): T[p,k,b,q], site S[s, in, p-side, open, q-side] in the compute
// type; the p-side bond takes (vp1, vp2), the q-side bond (vq1, vq2).
// Returns out[nu_p, ko, bo, nu_q] in F64.
Tensor chain(ctm_solver* s, Ctx& c, const Tensor& T, const Tensor& S, const Tensor& vp1,
             const Tensor& vp2, const Tensor& vq1, const Tensor& vq2) {
  const int cp = cdt(s);
  Tensor X1 = contract(c, T, "pkbq", vp1, "pim", "kbqim", cp, cp);
  Tensor X2 = contract(c, X1, "kbqim", S, "skioj", "bqmsoj", cp, cp);
  Tensor X3 = contract(c, X2, "bqmsoj", vq1, "qjn", "bmson", cp, cp);
  Tensor X4 = contract(c, X3, "bmson", vp2, "mIv", "vIbson", cp, cp);
  Tensor X5 = contract(c, X4, "vIbson", S, "sbIOJ", "vonOJ", cp, cp);
  return contract(c, X5, "vonOJ", vq2, "nJw", "voOw", cp, F64);
}

struct SplitV {
  Tensor v1, v2;
};

// Helper isometries and compressed corner of one side of the reduced
// half-network [C1 T2 C2; T1 z T3] (Appendix, Fig. A(c)): side 0 splits
// {C1, T1}, side 1 splits {C2, T3}.
struct SideIso {
  Tensor v1, v2, cc;
  void *b1 = nullptr, *b2 = nullptr, *bc = nullptr;
};

void side_iso(ctm_solver* s, Ctx& c, int r, int z, int side, SideIso* o) {
  const size_t mk = c.arena.mark();
  Tensor X;
  if (side == 0) {
    Tensor C1 = env_view(s, kC, 1, z, r), T1 = env_view(s, kT, 1, z, r);
    X = contract(c, C1, "mi", T1, "jklm", "iklj", F64, F64);
  } else {
    Tensor C2 = env_view(s, kC, 2, z, r), T3 = env_view(s, kT, 3, z, r);
    X = contract(c, C2, "im", T3, "mklj", "iklj", F64, F64);
  }
  split_iso(s, c, X, o->b1, o->b2, o->bc, &o->v1, &o->v2, &o->cc);
  c.arena.release(mk);
}

// Split isometries (v^1_z[j,kd,mu], v^2_z[mu,bd,nu]) of the reduced move
// (Secs. III-IV, Figs. 3-4): T'2 from the sequential ket-then-bra absorption
// of z into T2 between the two sides' helper isometries, M' = C'1 T'2 C'2,
// v^1 from M' as (chi D) x (D chi), v^2 from N = v^1^T M' as (chi' D) x chi.
SplitV anchor_reduced(ctm_solver* s, Ctx& c, int r, int z, const SideIso& L, const SideIso& R,
                      void* d1, void* d2) {
  const int64_t D = s->D;
  Tensor T2 = env_view(s, kT, 2, z, r), T1 = env_view(s, kT, 1, z, r);
  Tensor T3 = env_view(s, kT, 3, z, r);
  const int64_t nj = T1.dims[0], nj2 = T3.dims[3];
  const size_t mk = c.arena.mark();
  const int cp = cdt(s);
  Tensor S = make_view(s->sT2[r][z], cp, {s->d, D, D, D, D});
  Tensor Tp2 = chain(s, c, T2, S, L.v1, L.v2, R.v1, R.v2);
  Tensor Mp = contract(c, L.cc, "nj", Tp2, "ndDo", "jdDo", F64, F64);
  Mp = contract(c, Mp, "jdDo", R.cc, "ok", "jdDk", F64, F64);
  Tensor v1 = isometry(s, c, Mp, nj * D, D * nj2, d1, s->chi_p);
  const int64_t c1 = v1.dims[1];
  v1 = reshape(v1, {nj, D, c1});
  Tensor N = contract(c, v1, "jdm", Mp, "jdDk", "mDk", F64, F64);
  Tensor v2 = isometry(s, c, N, c1 * D, nj2, d2);
  const int64_t c2 = v2.dims[1];
  v2 = reshape(v2, {c1, D, c2});
  c.arena.release(mk);
  return SplitV{v1, v2};
}

// Whether an insertion in frame r uses the standard isometries: always for
// the standard method and during the first boot_iters iterations, and
// otherwise whenever the reduced rule would leave a new bond smaller, by
// shape, than the standard one (the reduced sub-networks have rank at most
// the far-side bond T3.q, so they cannot grow a bond).
bool insertion_standard(const ctm_solver* s, int r) {
  if (s->method == CTM_STANDARD) return true;
  if (s->moves / 4 < s->boot_iters) return true;
  const int64_t D = s->D, chi = s->chi;
  for (int z = 0; z < 2; ++z) {
    const int64_t nj = s->pd[env_index(kT, stored_i(1, r), z)];
    const int64_t nj2 = s->qd[env_index(kT, stored_i(3, r), z)];
    const int64_t sd = std::min({chi, nj * D * D, D * D * nj2});
    int64_t rd;
    if (s->method == CTM_REDUCED_ENV) {
      rd = std::min({chi, nj * D * D, nj2});
    } else {
      const int64_t c1 = std::min({(int64_t)s->chi_p, nj * D, D * nj2});
      rd = std::min({chi, c1 * D, nj2});
    }
    if (rd < sd) return true;
  }
  return false;
}

void store_env(ctm_solver* s, int e, const Tensor& t) {
  Ctx& c = s->ctx;
  double* nrm = s->scal + e;   // one scalar slot per tensor
  norm2(c, t.d(), t.numel(), nrm);
  keep(c, t, s->env[e]);
  scale_by_inv(c, s->env[e], t.numel(), nrm);
  s->pd[e] = (int)t.dims[0];
  s->qd[e] = (int)t.dims[t.nd - 1];
}

// Insert one column into the left environment (frame r) and truncate.
// Independent work runs as concurrent branches: the two anchors (standard
// move) or the side isometries and then the two split anchors (reduced
// move), and finally the updates of the two rows x = a, b.  The right-side
// isometries (from C2_z and T3_z, which a left move leaves unchanged) are
// the same for both insertions of a move: they are kept in rside, computed
// by the first reduced insertion (have_r false) and reused by the second.
void insert_column(ctm_solver* s, int r, SideIso* rside, bool have_r) {
  Ctx& c = s->ctx;
  const int64_t D = s->D, cap = s->cap, chi = s->chi;
  const bool stdm = insertion_standard(s, r);
  // 4-index isometries: standard (Sec. II) or reduced-env (Sec. III)
  const bool four = stdm || s->method == CTM_REDUCED_ENV;
  // the standard move's (chi D^2) x (D^2 chi) objects dominate the
  // workspace; when they are large its branches run one after the other
  const bool big_standard = stdm && (double)cap * D * D * cap * D * D * 8.0 > 1e9;
  const size_t mk = c.arena.mark();
  // anchors
  Tensor V4[2];
  SplitV VS[2];
  if (four) {
    void* dv[2];
    for (int z = 0; z < 2; ++z) dv[z] = c.arena.alloc(sizeof(double) * cap * D * D * chi);
    auto a0 = [&](Ctx& k) {
      V4[0] = stdm ? anchor_standard(s, k, r, 0, dv[0]) : anchor_reduced_env(s, k, r, 0, dv[0]);
    };
    auto a1 = [&](Ctx& k) {
      V4[1] = stdm ? anchor_standard(s, k, r, 1, dv[1]) : anchor_reduced_env(s, k, r, 1, dv[1]);
    };
    if (big_standard) {
      run_branches(s, {a0});
      run_branches(s, {a1});
    } else {
      run_branches(s, {a0, a1});
    }
  } else {
    SideIso side[2][2];   // [z][side]
    for (int z = 0; z < 2; ++z) {
      side[z][0].b1 = c.arena.alloc(sizeof(double) * cap * D * s->chi_pp);
      side[z][0].b2 = c.arena.alloc(sizeof(double) * s->chi_pp * D * chi);
      side[z][0].bc = c.arena.alloc(sizeof(double) * chi * cap);
      side[z][1] = rside[z];
    }
    std::vector<std::function<void(Ctx&)>> fs;
    for (int z = 0; z < 2; ++z)
      for (int sd = 0; sd < 2; ++sd)
        if (sd == 0 || !have_r)
          fs.push_back([&, z, sd](Ctx& k) { side_iso(s, k, r, z, sd, &side[z][sd]); });
    run_branches(s, fs);
    for (int z = 0; z < 2; ++z) rside[z] = side[z][1];
    void* d1[2];
    void* d2[2];
    for (int z = 0; z < 2; ++z) {
      d1[z] = c.arena.alloc(sizeof(double) * cap * D * s->chi_p);
      d2[z] = c.arena.alloc(sizeof(double) * s->chi_p * D * chi);
    }
    run_branches(s, {[&](Ctx& k) { VS[0] = anchor_reduced(s, k, r, 0, side[0][0], side[0][1], d1[0], d2[0]); },
                     [&](Ctx& k) { VS[1] = anchor_reduced(s, k, r, 1, side[1][0], side[1][1], d1[1], d2[1]); }});
  }
  // new tensors, staged until all six are done
  Tensor nC1[2], nT1[2], nC4[2];
  void *bC1[2], *bT1[2], *bC4[2];
  for (int y = 0; y < 2; ++y) {
    bC1[y] = c.arena.alloc(sizeof(double) * cap * cap);
    bT1[y] = c.arena.alloc(sizeof(double) * cap * D * D * cap);
    bC4[y] = c.arena.alloc(sizeof(double) * cap * cap);
  }
  const int cp = cdt(s);
  auto update_row = [&](Ctx& k, int x) {
    const int y = 1 - x;
    Tensor C1x = env_view(s, kC, 1, x, r), T2x = env_view(s, kT, 2, x, r);
    Tensor T1x = env_view(s, kT, 1, x, r);
    Tensor C4x = env_view(s, kC, 4, x, r), T4x = env_view(s, kT, 4, x, r);
    {
      const size_t m2 = k.arena.mark();
      Tensor G = contract(k, C1x, "jm", T2x, "mubq", "jubq", F64, F64);
      Tensor t;
      if (four) {
        t = contract(k, G, "jubq", V4[y], "jubn", "nq", F64, F64);
      } else {
        Tensor G1 = contract(k, G, "jubq", VS[y].v1, "jum", "mbq", F64, F64);
        t = contract(k, G1, "mbq", VS[y].v2, "mbn", "nq", F64, F64);
      }
      nC1[y] = keep(k, t, bC1[y]);
      k.arena.release(m2);
    }
    {
      const size_t m2 = k.arena.mark();
      Tensor t;
      if (four) {
        // the standard bootstrap stays FP64; the reduced-env method absorbs
        // in the compute type, like the sequential chains
        t = absorb4(k, T1x, site_view(s, r, x), V4[x], V4[y], stdm ? F64 : cp);
      } else {
        Tensor S = make_view(s->sT1[r][x], cp, {s->d, D, D, D, D});
        t = chain(s, k, T1x, S, VS[x].v1, VS[x].v2, VS[y].v1, VS[y].v2);
      }
      nT1[y] = keep(k, t, bT1[y]);
      k.arena.release(m2);
    }
    {
      const size_t m2 = k.arena.mark();
      Tensor G4 = contract(k, C4x, "mj", T4x, "pkbm", "jkbp", F64, F64);
      Tensor t;
      if (four) {
        t = contract(k, G4, "jkbp", V4[x], "jkbn", "pn", F64, F64);
      } else {
        Tensor G5 = contract(k, G4, "jkbp", VS[x].v1, "jkm", "mbp", F64, F64);
        t = contract(k, G5, "mbp", VS[x].v2, "mbn", "pn", F64, F64);
      }
      nC4[y] = keep(k, t, bC4[y]);
      k.arena.release(m2);
    }
  };
  auto u0 = [&](Ctx& k) { update_row(k, 0); };
  auto u1 = [&](Ctx& k) { update_row(k, 1); };
  if (big_standard) {
    run_branches(s, {u0});
    run_branches(s, {u1});
  } else {
    run_branches(s, {u0, u1});
  }
  for (int y = 0; y < 2; ++y) {
    store_env(s, env_index(kC, stored_i(1, r), y), nC1[y]);
    store_env(s, env_index(kT, stored_i(1, r), y), nT1[y]);
    store_env(s, env_index(kC, stored_i(4, r), y), nC4[y]);
  }
  c.arena.release(mk);
}

void do_move(ctm_solver* s, int r) {
  // random test matrices of the truncations depend only on their position in
  // the move, so a move from a given state is reproducible in any precision
  s->ctx.rng_calls = 0;
  Ctx& c = s->ctx;
  const int64_t D = s->D, cap = s->cap, chi = s->chi;
  const size_t mk = c.arena.mark();
  SideIso rside[2];
  for (int z = 0; z < 2; ++z) {
    rside[z].b1 = c.arena.alloc(sizeof(double) * cap * D * s->chi_pp);
    rside[z].b2 = c.arena.alloc(sizeof(double) * s->chi_pp * D * chi);
    rside[z].bc = c.arena.alloc(sizeof(double) * chi * cap);
  }
  bool have_r = false;
  for (int k = 0; k < 2; ++k) {
    const bool stdm = insertion_standard(s, r);
    insert_column(s, r, rside, have_r);
    have_r = have_r || !stdm;
  }
  c.arena.release(mk);
  s->moves++;
}

// Everything the launch sequence of a move in frame r depends on: the
// schedule follows from the bond dimensions, method, precision and bootstrap
// state alone; buffers sit at fixed places in the workspace and the random
// test matrices depend only on their position in the move.
std::string move_key(const ctm_solver* s, int r) {
  std::string k = std::to_string(r) + "/" + std::to_string(s->precision) + "/" +
                  std::to_string(s->method) + "/" + std::to_string(s->moves / 4 < s->boot_iters);
  for (int e = 0; e < 16; ++e) k += "/" + std::to_string(s->pd[e]) + "x" + std::to_string(s->qd[e]);
  return k;
}

// One move.  With graph replay on, the concurrent branches of the move are
// captured and replayed per branch (see run_branches) under the move's key.
void run_move(ctm_solver* s, int r) {
  s->move_tag = (s->graphs && s->ctx.prof == nullptr) ? move_key(s, r) : std::string();
  s->branch_call = 0;
  try {
    do_move(s, r);
  } catch (...) {
    s->move_tag.clear();
    throw;
  }
  s->move_tag.clear();
}

void do_iteration(ctm_solver* s) {
  static const int order[4] = {CTM_LEFT, CTM_RIGHT, CTM_UP, CTM_DOWN};
  for (int i = 0; i < 4; ++i) run_move(s, order[i]);
}

// normalised corner spectra of the 8 corners into spec[cur]
void corner_spectra(ctm_solver* s) {
  Ctx& c = s->ctx;
  double* out = s->spec[s->spec_cur];
  for (int z = 0; z < 2; ++z)
    for (int i = 1; i <= 4; ++i) {
      const int e = env_index(kC, i, z);
      corner_spectrum(c, s->env[e], s->pd[e], s->qd[e], s->chi, out + (size_t)(i - 1 + 4 * z) * s->chi);
    }
}

// Half of the bond network on the side of site x (frame r):
// H[s, c, r1, i, S, R1] with c / i the bonds to T2 / T4 of the other half,
// r1 / R1 the ket / bra legs toward the other site, s / S the physical
// indices.  The ket site is absorbed one physical slice at a time, so no
// intermediate exceeds chi^2 D^4 entries.
Tensor half_network(ctm_solver* s, int x, int r, void* dst) {
  Ctx& c = s->ctx;
  const int64_t d = s->d, D = s->D;
  const int64_t D4 = D * D * D * D;
  Tensor C1 = env_view(s, kC, 1, x, r), T1 = env_view(s, kT, 1, x, r), C4 = env_view(s, kC, 4, x, r);
  Tensor T2 = env_view(s, kT, 2, x, r), T4 = env_view(s, kT, 4, x, r);
  const int64_t nc = T2.dims[3], ni = T4.dims[0];
  Tensor H = make_view(dst, F64, {d, nc, D, ni, d, D});
  const size_t mk = c.arena.mark();
  Tensor L = contract(c, C1, "ab", T1, "fkla", "bfkl", F64, F64);
  L = contract(c, L, "bfkl", C4, "hf", "bklh", F64, F64);
  Tensor P2 = contract(c, L, "bklh", T2, "buUc", "klhuUc", F64, F64);
  Tensor P2p = relabel(c, P2, "klhuUc", "lhUcku", F64);
  Tensor Ax = site_view(s, r, x);
  for (int64_t sl = 0; sl < d; ++sl) {
    const size_t m2 = c.arena.mark();
    Tensor As = make_view((double*)Ax.p + sl * D4, F64, {D, D, D, D});
    Tensor P3 = contract(c, P2p, "lhUcku", As, "kurd", "lhUcrd", F64, F64);
    Tensor P4 = contract(c, P3, "lhUcrd", T4, "idDh", "lUcriD", F64, F64);
    Tensor Hs = contract(c, P4, "lUcriD", Ax, "SlURD", "criSR", F64, F64);
    keep(c, Hs, (double*)dst + sl * (nc * D * ni * d * D));
    c.arena.release(m2);
  }
  c.arena.release(mk);
  return H;
}

// <h> numerator and trace for the bond (x, right neighbour) in frame r -> out[0..1]
void bond_energy(ctm_solver* s, int x, int r, double* out) {
  Ctx& c = s->ctx;
  const int y = 1 - x;
  const int64_t d = s->d, D = s->D;
  const size_t mk = c.arena.mark();
  // left half: site x in frame r; right half: site y seen from the mirrored
  // frame r + 2, where its environment C3, T4, C2, T3, T2 plays C1, T2, C4,
  // T1, T4 and the other site is on its left
  const int rm = (r + 2) % 4;
  const int64_t ncL = env_view(s, kT, 2, x, r).dims[3], niL = env_view(s, kT, 4, x, r).dims[0];
  const int64_t ncR = env_view(s, kT, 2, y, rm).dims[3], niR = env_view(s, kT, 4, y, rm).dims[0];
  void* bl = c.arena.alloc(sizeof(double) * d * ncL * D * niL * d * D);
  void* br = c.arena.alloc(sizeof(double) * d * ncR * D * niR * d * D);
  Tensor HL = half_network(s, x, r, bl);
  Tensor HR = half_network(s, y, rm, br);
  // HL[s, c, r1, i, S, R1] with c -> T2_y.p, i -> T4_y.q; in the mirrored
  // frame the right half's T2-bond index is the T4_y.q bond of frame r and
  // its T4-bond index the T2_y.p bond: HR[t, i, r1, c, T, R1]
  Tensor rho = contract(c, HL, "scriSR", HR, "tircTR", "stST", F64, F64);
  rho_energy(c, rho.d(), s->h4, s->d, out);
  c.arena.release(mk);
}

// Right boundary column {C2, T3, C3} of site x in frame r:
// Rb[c, r1, R1, i] with c the bond to T2_x.q, (r1, R1) the legs into the
// site's right leg and i the bond to T4_x.p.
Tensor right_boundary(ctm_solver* s, Ctx& c, int x, int r) {
  Tensor C2 = env_view(s, kC, 2, x, r), T3 = env_view(s, kT, 3, x, r), C3 = env_view(s, kC, 3, x, r);
  Tensor X = contract(c, C2, "bn", T3, "ntTe", "btTe", F64, F64);
  return contract(c, X, "btTe", C3, "eg", "btTg", F64, F64);
}

// Unnormalised one-site reduced density matrix rho[s, S] of an x-site (the
// site between its four corners and four edges, Sec. II, Fig. 1(c)) into
// out (d x d, device): the left half of the bond network closed by the
// site's own right boundary.
void site_rdm(ctm_solver* s, int x, double* out) {
  Ctx& c = s->ctx;
  const int64_t d = s->d, D = s->D;
  const size_t mk = c.arena.mark();
  const int64_t nc = env_view(s, kT, 2, x, 0).dims[3], ni = env_view(s, kT, 4, x, 0).dims[0];
  void* bl = c.arena.alloc(sizeof(double) * d * nc * D * ni * d * D);
  Tensor HL = half_network(s, x, 0, bl);
  Tensor Rb = right_boundary(s, c, x, 0);
  Tensor rho = contract(c, HL, "scriSR", Rb, "crRi", "sS", F64, F64);
  keep(c, rho, out);
  c.arena.release(mk);
}

// Absorb the column {T2_z, z, T4_z} (frame 0, identity on the site's
// physical legs) into a left vector V[c, r, R, f]: c / f the bonds to the
// next T2 / T4, (r, R) the ket / bra legs toward the next site.  Ket layer
// before bra layer (chi^3 D^4 + chi^2 D^6 d).
Tensor absorb_column(ctm_solver* s, Ctx& c, const Tensor& V, int z) {
  Tensor T2 = env_view(s, kT, 2, z, 0), T4 = env_view(s, kT, 4, z, 0);
  Tensor A = site_view(s, 0, z);
  Tensor X = contract(c, V, "crRf", T2, "cuUb", "rRfuUb", F64, F64);
  X = contract(c, X, "rRfuUb", A, "srutd", "RfUbstd", F64, F64);
  X = contract(c, X, "RfUbstd", A, "sRUTD", "fbtdTD", F64, F64);
  return contract(c, X, "fbtdTD", T4, "gdDf", "btTg", F64, F64);
}

// <op> numerators and traces of the a- and b-site into out[0..3]
// (numerator a, trace a, numerator b, trace b); op is d x d on the device.
void expect1_impl(ctm_solver* s, const double* op, double* out) {
  Ctx& c = s->ctx;
  const int d = s->d;
  const size_t mk = c.arena.mark();
  double* rho = (double*)c.arena.alloc(sizeof(double) * d * d);
  for (int z = 0; z < 2; ++z) {
    site_rdm(s, z, rho);
    rho1_expect(c, rho, op, d, out + 2 * z);
  }
  c.arena.release(mk);
}

// Connected correlation C(x) = <op_0 op_x> - <op_0><op_x> along a row of
// frame 0 for x = 1..L into out (device), site 0 on sublattice a (Sec. V,
// Fig. 8(b)).  Two left vectors, with op and with the identity on site 0,
// are carried along the row column by column (both divided by the norm of
// the identity one after each column, so their ratios are unchanged); at
// each x they are closed with the right half of the site at x.
void row_corr_impl(ctm_solver* s, const double* op, int L, double* out) {
  Ctx& c = s->ctx;
  const int64_t d = s->d, D = s->D, cap = s->cap;
  const size_t mk = c.arena.mark();
  double* nrm = (double*)c.arena.alloc(sizeof(double));
  Tensor opT = make_view((void*)op, F64, {d, d});
  Tensor I = c.alloc(F64, {d, d});
  fill(c, I.p, F64, d * d, 0.0);
  for (int64_t k = 0; k < d; ++k) fill(c, I.d() + k * (d + 1), F64, 1, 1.0);
  Tensor HR[2];
  for (int z = 0; z < 2; ++z) {
    const int64_t nc = env_view(s, kT, 2, z, 2).dims[3], ni = env_view(s, kT, 4, z, 2).dims[0];
    void* b = c.arena.alloc(sizeof(double) * d * nc * D * ni * d * D);
    HR[z] = half_network(s, z, 2, b);
  }
  const size_t vbytes = sizeof(double) * cap * D * D * cap;
  void* vo_buf = c.arena.alloc(vbytes);
  void* vi_buf = c.arena.alloc(vbytes);
  Tensor VO, VI;
  {
    const size_t m2 = c.arena.mark();
    const int64_t nc = env_view(s, kT, 2, 0, 0).dims[3], ni = env_view(s, kT, 4, 0, 0).dims[0];
    void* bl = c.arena.alloc(sizeof(double) * d * nc * D * ni * d * D);
    Tensor HL = half_network(s, 0, 0, bl);
    VO = keep(c, contract(c, HL, "scriSR", opT, "Ss", "crRi", F64, F64), vo_buf);
    VI = keep(c, contract(c, HL, "scriSR", I, "Ss", "crRi", F64, F64), vi_buf);
    c.arena.release(m2);
  }
  for (int x = 1; x <= L; ++x) {
    const int z = (x % 2 == 0) ? 0 : 1;
    const size_t m2 = c.arena.mark();
    Tensor RO = contract(c, VO, "crRi", HR[z], "tircTR", "tT", F64, F64);
    Tensor RI = contract(c, VI, "crRi", HR[z], "tircTR", "tT", F64, F64);
    corr_finish(c, RO.d(), RI.d(), op, (int)d, out + (x - 1));
    if (x < L) {
      Tensor nO = absorb_column(s, c, VO, z);
      Tensor nI = absorb_column(s, c, VI, z);
      norm2(c, nI.d(), nI.numel(), nrm);
      VO = keep(c, nO, vo_buf);
      VI = keep(c, nI, vi_buf);
      scale_by_inv(c, VO.d(), VO.numel(), nrm);
      scale_by_inv(c, VI.d(), VI.numel(), nrm);
    }
    c.arena.release(m2);
  }
  c.arena.release(mk);
}

// site layouts used by the absorption chains, in the compute type:
// S[s, in, p-side, open, q-side] for the T1 chain and the T2 chain
void rebuild_chain_sites(ctm_solver* s) {
  Ctx& c = s->ctx;
  const int64_t d = s->d, D = s->D;
  const int cp = cdt(s);
  for (int r = 0; r < 4; ++r)
    for (int z = 0; z < 2; ++z) {
      Tensor rot = make_view(s->site_rot[r][z], F64, {d, D, D, D, D});
      const int p1[5] = {0, 1, 4, 3, 2}, p2[5] = {0, 2, 1, 4, 3};
      Tensor o1 = make_view(s->sT1[r][z], cp, {d, D, D, D, D});
      Tensor o2 = make_view(s->sT2[r][z], cp, {d, D, D, D, D});
      permute(c, rot, p1, o1);
      permute(c, rot, p2, o2);
    }
}

void perm_rot(int r, int* p) {
  // r quarter turns of (s,l,u,r,d) -> (s,u,r,d,l)
  int cur[5] = {0, 1, 2, 3, 4};
  const int one[5] = {0, 2, 3, 4, 1};
  for (int t = 0; t < r; ++t) {
    int nxt[5];
    for (int i = 0; i < 5; ++i) nxt[i] = cur[one[i]];
    std::memcpy(cur, nxt, sizeof(cur));
  }
  std::memcpy(p, cur, sizeof(cur));
}

// layout: persistent buffers, then sites and the traced-boundary environment
void setup(ctm_solver* s, const double* A, const double* B, int on_device) {
  Ctx& c = s->ctx;
  const int64_t d = s->d, D = s->D, cap = s->cap, chi = s->chi;
  for (int e = 0; e < 16; ++e) {
    const size_t n = (e < 8) ? (size_t)cap * cap : (size_t)cap * D * D * cap;
    s->env[e] = (double*)c.arena.alloc(n * sizeof(double));
  }
  const size_t ns = (size_t)(d * D * D * D * D);
  for (int z = 0; z < 2; ++z) s->site[z] = (double*)c.arena.alloc(ns * sizeof(double));
  for (int r = 0; r < 4; ++r)
    for (int z = 0; z < 2; ++z) {
      s->site_rot[r][z] = (double*)c.arena.alloc(ns * sizeof(double));
      s->sT1[r][z] = c.arena.alloc(ns * sizeof(double));
      s->sT2[r][z] = c.arena.alloc(ns * sizeof(double));
    }
  s->spec[0] = (double*)c.arena.alloc(8 * chi * sizeof(double));
  s->spec[1] = (double*)c.arena.alloc(8 * chi * sizeof(double));
  s->scal = (double*)c.arena.alloc(64 * sizeof(double));
  s->h4 = (double*)c.arena.alloc(d * d * d * d * sizeof(double));
  c.dev_flags = (int*)c.arena.alloc(16 * sizeof(int));
  c.work = (double*)c.arena.alloc(8 * sizeof(double));
  s->persist = c.arena.mark();
  if (c.arena.overflow) return;
  if (!c.dry) {
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    c.check(hipMemcpyAsync(s->site[0], A, ns * sizeof(double), kind, c.stream));
    c.check(hipMemcpyAsync(s->site[1], B, ns * sizeof(double), kind, c.stream));
    fill(c, c.dev_flags, F32, 16, 0.0);   // 16 ints, zero bit pattern
  }
  for (int r = 0; r < 4; ++r)
    for (int z = 0; z < 2; ++z) {
      int p[5];
      perm_rot(r, p);
      Tensor in = make_view(s->site[z], F64, {d, D, D, D, D});
      Tensor out = make_view(s->site_rot[r][z], F64, {d, D, D, D, D});
      permute(c, in, p, out);
    }
  rebuild_chain_sites(s);
  // traced-boundary environment (frame 0)
  const int64_t D2 = D * D;
  for (int z = 0; z < 2; ++z) {
    Tensor X = site_view(s, 0, z), Y = site_view(s, 0, 1 - z);
    const size_t mk = c.arena.mark();
    struct Spec { int kind, i; const Tensor* t; const char* lb; const char* lo; };
    const Spec sp[8] = {
        {kC, 1, &X, "sluRD", "dDrR"},   {kC, 2, &X, "sLurD", "lLdD"},
        {kC, 3, &X, "sLUrd", "uUlL"},   {kC, 4, &X, "slURd", "rRuU"},
        {kT, 1, &Y, "slURD", "dDrRuU"}, {kT, 2, &Y, "sLuRD", "lLdDrR"},
        {kT, 3, &Y, "sLUrD", "uUlLdD"}, {kT, 4, &Y, "sLURd", "rRuUlL"}};
    for (const Spec& q : sp) {
      const size_t m2 = c.arena.mark();
      Tensor t = contract(c, *q.t, "slurd", *q.t, q.lb, q.lo, F64, F64);
      Tensor v = q.kind == kC ? reshape(t, {D2, D2}) : reshape(t, {D2, D, D, D2});
      store_env(s, env_index(q.kind, q.i, z), v);
      c.arena.release(m2);
    }
    c.arena.release(mk);
  }
}

// Status for the exception being handled (call inside a catch block):
// the code an Error carries, CTM_ENOMEM for a failed host allocation, and
// otherwise CTM_EHIP when a HIP call has failed, CTM_EINVAL if not.
int fail_status(const ctm_solver* s) {
  try {
    throw;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    return CTM_ENOMEM;
  } catch (...) {
    if (s && s->ctx.hip_err != hipSuccess) return CTM_EHIP;
    return CTM_EINVAL;
  }
}

int status_from(ctm_solver* s) {
  if (s->ctx.arena.overflow) return CTM_ENOMEM;
  if (s->ctx.hip_err != hipSuccess) return CTM_EHIP;
  return CTM_OK;
}

bool valid_cfg(const ctm_config* cfg) {
  if (!cfg) return false;
  if (cfg->d < 2 || cfg->D < 1 || cfg->chi < 1) return false;
  // the traced-boundary environment starts with bonds of dimension D^2
  if ((int64_t)cfg->chi < (int64_t)cfg->D * cfg->D) return false;
  if (cfg->method != CTM_STANDARD && cfg->method != CTM_REDUCED && cfg->method != CTM_REDUCED_ENV)
    return false;
  if (cfg->precision < CTM_FP64 || cfg->precision > CTM_BF16) return false;
  if (cfg->boot_iters < 0) return false;
  // chi' and chi'' (0 = chi) may not be below chi: the second stages keep chi
  if (cfg->chi_p < 0 || cfg->chi_pp < 0) return false;
  if ((cfg->chi_p > 0 && cfg->chi_p < cfg->chi) || (cfg->chi_pp > 0 && cfg->chi_pp < cfg->chi))
    return false;
  if (!(cfg->svd_cutoff >= 0.0) || cfg->svd_cutoff >= 1.0) return false;
  // every dimension product must stay well inside 32-bit GEMM sizes
  const double cap = std::max<double>(cfg->chi, (double)cfg->D * cfg->D);
  if (cap * cfg->D * cfg->D * cfg->D * cfg->d > 2.0e9) return false;
  const double cpm = std::max<double>(std::max(cfg->chi_p, cfg->chi_pp), cfg->chi);
  if (cpm * cfg->D * cfg->D * cfg->D * cfg->d * cfg->D > 4.0e10) return false;
  return true;
}

void fill_from_cfg(ctm_solver* s, const ctm_config* cfg) {
  s->d = cfg->d;
  s->D = cfg->D;
  s->chi = cfg->chi;
  s->chi_p = cfg->chi_p > 0 ? cfg->chi_p : cfg->chi;
  s->chi_pp = cfg->chi_pp > 0 ? cfg->chi_pp : cfg->chi;
  s->method = cfg->method;
  s->precision = cfg->precision;
  s->boot_iters = cfg->boot_iters;
  s->tau = cfg->svd_cutoff;
  s->cap = cfg->chi;   // valid_cfg requires chi >= D^2
  s->ctx.stream = (hipStream_t)cfg->stream;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

size_t ctm_workspace_size(const ctm_config* cfg) {
  if (!valid_cfg(cfg)) return 0;
  try {
    ctm_solver s;
    fill_from_cfg(&s, cfg);
    s.ctx.dry = true;
    s.ctx.arena.dry = true;
    setup(&s, nullptr, nullptr, 0);
    // shapes settle after the first iteration; two more cover the steady state
    const int iters = std::max(1, s.boot_iters) + 2;
    const bool dbg = std::getenv("CTM_DEBUG_MEM") != nullptr;
    for (int it = 0; it < iters; ++it) {
      for (int mv : {CTM_LEFT, CTM_RIGHT, CTM_UP, CTM_DOWN}) {
        const bool stdm = insertion_standard(&s, mv);
        do_move(&s, mv);
        if (dbg) std::fprintf(stderr, "iter %d move %d std %d peak %.1f MB\n", it, mv, (int)stdm, s.ctx.arena.peak / 1e6);
      }
    }
    corner_spectra(&s);
    if (dbg) std::fprintf(stderr, "spectra peak %.1f MB\n", s.ctx.arena.peak / 1e6);
    for (int k = 0; k < 4; ++k) bond_energy(&s, k & 1, k >> 1, s.scal);
    if (dbg) std::fprintf(stderr, "energy peak %.1f MB\n", s.ctx.arena.peak / 1e6);
    // observables: one-site expectations and a row correlation (its peak
    // is reached at the first column; later columns reuse the same space)
    {
      const size_t mk = s.ctx.arena.mark();
      double* dop = (double*)s.ctx.arena.alloc(sizeof(double) * s.d * s.d);
      double* dout = (double*)s.ctx.arena.alloc(sizeof(double) * kMaxCorrLength);
      expect1_impl(&s, dop, s.scal);
      row_corr_impl(&s, dop, 2, dout);
      s.ctx.arena.release(mk);
    }
    if (dbg) std::fprintf(stderr, "observables peak %.1f MB\n", s.ctx.arena.peak / 1e6);
    return s.ctx.arena.peak + 4096;
  } catch (...) {
    return 0;
  }
}

int ctm_init(const ctm_config* cfg, const double* A, const double* B, int ptrs_on_device,
             ctm_solver** out) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  if (!valid_cfg(cfg) || !A || !B || !cfg->workspace) return CTM_EINVAL;
  const size_t need = ctm_workspace_size(cfg);
  if (need == 0) return CTM_EINVAL;
  if (cfg->workspace_bytes < need) return CTM_ENOMEM;
  ctm_solver* s = new (std::nothrow) ctm_solver();
  if (!s) return CTM_ENOMEM;
  try {
    fill_from_cfg(s, cfg);
    s->ctx.arena.base = (char*)cfg->workspace;
    s->ctx.arena.cap = cfg->workspace_bytes;
    for (hipStream_t& st : s->aux) s->ctx.check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    s->ctx.check(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    for (hipEvent_t& e : s->ev_join) s->ctx.check(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    setup(s, A, B, ptrs_on_device);
    s->ctx.check(hipStreamSynchronize(s->ctx.stream));
    int st = status_from(s);
    if (st == CTM_OK) {
      int flag = 0;
      s->ctx.check(hipMemcpy(&flag, s->ctx.dev_flags, sizeof(int), hipMemcpyDeviceToHost));
      if (flag) st = CTM_ENUMERIC;
      st = st == CTM_OK ? status_from(s) : st;
    }
    if (st != CTM_OK) {
      delete s;
      return st;
    }
  } catch (...) {
    const int st = fail_status(s);
    delete s;
    return st;
  }
  *out = s;
  return CTM_OK;
}

int ctm_move(ctm_solver* s, int dir) {
  if (!s || dir < 0 || dir > 3) return CTM_EINVAL;
  try {
    run_move(s, dir);
  } catch (...) {
    return fail_status(s);
  }
  s->spec_valid = false;
  return status_from(s);
}

int ctm_iterate(ctm_solver* s, int n) {
  if (!s || n < 0) return CTM_EINVAL;
  try {
    for (int i = 0; i < n; ++i) do_iteration(s);
  } catch (...) {
    return fail_status(s);
  }
  s->spec_valid = false;
  return status_from(s);
}

int ctm_converge(ctm_solver* s, int max_iters, double tol, int* iters_done, double* delta) {
  if (!s || max_iters < 0) return CTM_EINVAL;
  Ctx& c = s->ctx;
  double dl = INFINITY;
  int it = 0;
  try {
    if (!s->spec_valid) {
      corner_spectra(s);
      s->spec_valid = true;
    }
    for (it = 0; it < max_iters;) {
      do_iteration(s);
      ++it;
      s->spec_cur ^= 1;
      corner_spectra(s);
      max_abs_diff(c, s->spec[s->spec_cur], s->spec[s->spec_cur ^ 1], 8 * s->chi, s->scal + 32);
      int flag = 0;
      c.check(hipMemcpyAsync(&dl, s->scal + 32, sizeof(double), hipMemcpyDeviceToHost, c.stream));
      c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
      c.check(hipStreamSynchronize(c.stream));
      if (status_from(s) != CTM_OK) break;
      if (flag) {
        if (iters_done) *iters_done = it;
        if (delta) *delta = dl;
        return CTM_ENUMERIC;
      }
      if (dl < tol) break;
    }
  } catch (...) {
    return fail_status(s);
  }
  if (iters_done) *iters_done = it;
  if (delta) *delta = dl;
  const int st = status_from(s);
  if (st != CTM_OK) return st;
  return (dl < tol) ? CTM_OK : CTM_ENOTCONV;
}

int ctm_iterate_delta(ctm_solver* s) {
  if (!s) return CTM_EINVAL;
  Ctx& c = s->ctx;
  try {
    if (!s->spec_valid) {
      corner_spectra(s);
      s->spec_valid = true;
    }
    do_iteration(s);
    s->spec_cur ^= 1;
    corner_spectra(s);
    max_abs_diff(c, s->spec[s->spec_cur], s->spec[s->spec_cur ^ 1], 8 * s->chi, s->scal + 32);
  } catch (...) {
    return fail_status(s);
  }
  return status_from(s);
}

int ctm_read_delta(ctm_solver* s, double* delta) {
  if (!s) return CTM_EINVAL;
  Ctx& c = s->ctx;
  double dl = INFINITY;
  int flag = 0;
  c.check(hipMemcpyAsync(&dl, s->scal + 32, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  c.check(hipStreamSynchronize(c.stream));
  if (delta) *delta = dl;
  const int st = status_from(s);
  if (st != CTM_OK) return st;
  return flag ? CTM_ENUMERIC : CTM_OK;
}

int ctm_expect1(ctm_solver* s, const double* op, double out[2]) {
  if (!s || !op || !out) return CTM_EINVAL;
  Ctx& c = s->ctx;
  const int d = s->d;
  double res[4];
  int flag = 0;
  try {
    const size_t mk = c.arena.mark();
    double* dop = (double*)c.arena.alloc(sizeof(double) * d * d);
    c.check(hipMemcpyAsync(dop, op, sizeof(double) * d * d, hipMemcpyHostToDevice, c.stream));
    expect1_impl(s, dop, s->scal + 48);
    c.check(hipMemcpyAsync(res, s->scal + 48, sizeof(res), hipMemcpyDeviceToHost, c.stream));
    c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    c.check(hipStreamSynchronize(c.stream));
    c.arena.release(mk);
  } catch (...) {
    return fail_status(s);
  }
  const int st = status_from(s);
  if (st != CTM_OK) return st;
  bool bad = flag != 0;
  for (int z = 0; z < 2; ++z) {
    out[z] = res[2 * z] / res[2 * z + 1];
    if (!std::isfinite(out[z])) bad = true;
  }
  return bad ? CTM_ENUMERIC : CTM_OK;
}

int ctm_row_correlation(ctm_solver* s, const double* op, int L, double* out) {
  if (!s || !op || !out || L < 1 || L > kMaxCorrLength) return CTM_EINVAL;
  Ctx& c = s->ctx;
  const int d = s->d;
  std::vector<double> res((size_t)L, 0.0);
  int flag = 0;
  try {
    const size_t mk = c.arena.mark();
    double* dop = (double*)c.arena.alloc(sizeof(double) * d * d);
    double* dout = (double*)c.arena.alloc(sizeof(double) * L);
    c.check(hipMemcpyAsync(dop, op, sizeof(double) * d * d, hipMemcpyHostToDevice, c.stream));
    row_corr_impl(s, dop, L, dout);
    c.check(hipMemcpyAsync(res.data(), dout, sizeof(double) * L, hipMemcpyDeviceToHost, c.stream));
    c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    c.check(hipStreamSynchronize(c.stream));
    c.arena.release(mk);
  } catch (...) {
    return fail_status(s);
  }
  const int st = status_from(s);
  if (st != CTM_OK) return st;
  bool bad = flag != 0;
  for (int x = 0; x < L; ++x) {
    out[x] = res[x];
    if (!std::isfinite(res[x])) bad = true;
  }
  return bad ? CTM_ENUMERIC : CTM_OK;
}

int ctm_energy(ctm_solver* s, const double* h2, double* e_site, double e_bond[4]) {
  if (!s) return CTM_EINVAL;
  Ctx& c = s->ctx;
  const int d = s->d;
  std::vector<double> h(d * d * d * d, 0.0);
  if (h2) {
    std::memcpy(h.data(), h2, h.size() * sizeof(double));
  } else {
    if (d != 2) return CTM_EINVAL;
    // S.S = (sx sx + sy sy + sz sz) / 4 in the basis (up, down)
    const double v[16] = {0.25, 0, 0, 0, 0, -0.25, 0.5, 0, 0, 0.5, -0.25, 0, 0, 0, 0, 0.25};
    std::memcpy(h.data(), v, sizeof(v));
  }
  double res[8];
  int flag = 0;
  try {
    c.check(hipMemcpyAsync(s->h4, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    for (int k = 0; k < 4; ++k) bond_energy(s, k & 1, k >> 1, s->scal + 40 + 2 * k);
    c.check(hipMemcpyAsync(res, s->scal + 40, sizeof(res), hipMemcpyDeviceToHost, c.stream));
    c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    c.check(hipStreamSynchronize(c.stream));
  } catch (...) {
    return fail_status(s);
  }
  const int st = status_from(s);
  if (st != CTM_OK) return st;
  double sum = 0.0;
  bool bad = flag != 0;
  for (int k = 0; k < 4; ++k) {
    const double e = res[2 * k] / res[2 * k + 1];
    if (!std::isfinite(e)) bad = true;
    if (e_bond) e_bond[k] = e;
    sum += e;
  }
  if (e_site) *e_site = 0.5 * sum;
  return bad ? CTM_ENUMERIC : CTM_OK;
}

int ctm_get_env(ctm_solver* s, int e, double* host_out, size_t n, int* p, int* q) {
  if (!s || e < 0 || e > 15) return CTM_EINVAL;
  if (p) *p = s->pd[e];
  if (q) *q = s->qd[e];
  const size_t cnt = (e < 8) ? (size_t)s->pd[e] * s->qd[e]
                             : (size_t)s->pd[e] * s->D * s->D * s->qd[e];
  if (host_out) {
    if (n < cnt) return CTM_EINVAL;
    s->ctx.check(hipMemcpyAsync(host_out, s->env[e], cnt * sizeof(double), hipMemcpyDeviceToHost,
                                s->ctx.stream));
    s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  }
  return status_from(s);
}

int ctm_set_env(ctm_solver* s, int e, const double* host_in, int p, int q) {
  if (!s || e < 0 || e > 15 || !host_in || p < 1 || q < 1 || p > s->cap || q > s->cap)
    return CTM_EINVAL;
  const size_t cnt = (e < 8) ? (size_t)p * q : (size_t)p * s->D * s->D * q;
  s->ctx.check(hipMemcpyAsync(s->env[e], host_in, cnt * sizeof(double), hipMemcpyHostToDevice,
                              s->ctx.stream));
  s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  s->pd[e] = p;
  s->qd[e] = q;
  s->spec_valid = false;
  return status_from(s);
}

int ctm_moves_done(const ctm_solver* s) { return s ? s->moves : -1; }


int ctm_set_precision(ctm_solver* s, int precision) {
  if (!s || precision < CTM_FP64 || precision > CTM_BF16) return CTM_EINVAL;
  if (precision == s->precision) return CTM_OK;
  // the chain layouts of the sites are kept in the compute type; the
  // buffers were sized for FP64, the widest type
  s->precision = precision;
  rebuild_chain_sites(s);
  return status_from(s);
}

int ctm_set_graphs(ctm_solver* s, int enable) {
  if (!s) return CTM_EINVAL;
  s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  s->drop_graphs();
  s->graphs = enable != 0;
  return status_from(s);
}

int ctm_profile(ctm_solver* s, int enable) {
  if (!s) return CTM_EINVAL;
  s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  s->prof.clear();
  s->ctx.prof = enable ? &s->prof : nullptr;
  if (enable) {
    fill(s->ctx, s->ctx.work, F64, 8, 0.0);
    s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  }
  return status_from(s);
}

int ctm_profile_read(ctm_solver* s, int cls, long long* launches, double* ms, double* flops,
                     double* bytes) {
  if (!s || cls < 0 || cls >= K_NCLASS) return CTM_EINVAL;
  s->ctx.check(hipStreamSynchronize(s->ctx.stream));
  s->prof.collect();
  double f = s->prof.flops[cls], b = s->prof.bytes[cls];
  if (cls == K_SVD_ROUND) {   // data-dependent work, tallied on the device
    double w[2] = {0.0, 0.0};
    s->ctx.check(hipMemcpy(w, s->ctx.work, sizeof(w), hipMemcpyDeviceToHost));
    f = w[0];
    b = w[1];
  }
  if (launches) *launches = s->prof.n[cls];
  if (ms) *ms = s->prof.ms[cls];
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  return status_from(s);
}

void ctm_destroy(ctm_solver* s) {
  if (s) s->prof.clear();
  delete s;
}

const char* ctm_status_string(int status) {
  switch (status) {
    case CTM_OK: return "ok";
    case CTM_EINVAL: return "invalid argument";
    case CTM_ENOMEM: return "workspace too small";
    case CTM_EHIP: return "HIP runtime error";
    case CTM_ENUMERIC: return "numerical failure (zero, NaN or Inf norm, or a Jacobi SVD that did not converge)";
    case CTM_ENOTCONV: return "not converged within max_iters";
    default: return "unknown status";
  }
}

}  // extern "C"

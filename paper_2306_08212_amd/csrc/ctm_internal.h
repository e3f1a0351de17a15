// Internal declarations of the corner-transfer library: device tensors,
// the workspace arena, and the launch wrappers of every kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>

namespace ctm {

enum DType : int { F64 = 0, F32 = 1, BF16 = 2 };

// An error that carries the ctm_status the C-ABI returns for it (workspace
// exhausted, a failed HIP call such as a graph capture).
struct Error : std::runtime_error {
  int code;
  Error(int c, const char* what) : std::runtime_error(what), code(c) {}
};

inline size_t dtype_size(int dt) { return dt == F64 ? 8 : (dt == F32 ? 4 : 2); }

constexpr int kMaxDims = 8;

// A dense row-major tensor living in the workspace (or a dry-run stand-in).
struct Tensor {
  void* p = nullptr;
  int dt = F64;
  int nd = 0;
  int64_t dims[kMaxDims] = {0};
  int64_t numel() const {
    int64_t n = 1;
    for (int i = 0; i < nd; ++i) n *= dims[i];
    return n;
  }
  size_t bytes() const { return (size_t)numel() * dtype_size(dt); }
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
};

Tensor make_view(void* p, int dt, std::initializer_list<int64_t> dims);
Tensor make_view(void* p, int dt, const std::vector<int64_t>& dims);

// Bump allocator over caller-owned device memory.  In dry-run mode it only
// tracks the high-water mark; pointers are offsets from a fake base and no
// kernel is launched.  Outside dry runs an allocation beyond the capacity
// sets `overflow` and throws Error(CTM_ENOMEM = 2), so no kernel is ever
// launched on memory the arena does not own.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t top = 0;
  size_t peak = 0;
  bool dry = false;
  bool overflow = false;
  void* alloc(size_t bytes);
  size_t mark() const { return top; }
  void release(size_t m) { top = m; }
};

// Kernel classes for live timing (HIP events around launches on the stream).
enum KClass : int {
  K_GEMM_F64 = 0, K_GEMM_F32, K_GEMM_BF16, K_PERMUTE, K_SVD_ROUND, K_SVD_OTHER, K_REDUCE,
  K_COPY, K_CHOL, K_NCLASS
};

struct Profiler {
  struct Rec {
    int cls;
    double flops, bytes;
    hipEvent_t e0, e1;
    int launches;
  };
  std::vector<Rec> recs;
  long long n[K_NCLASS] = {0};
  double ms[K_NCLASS] = {0}, flops[K_NCLASS] = {0}, bytes[K_NCLASS] = {0};
  // resolve recorded events (the stream must have been synchronised)
  void collect();
  void clear();
};

struct Ctx {
  hipStream_t stream = nullptr;
  Profiler* prof = nullptr;
  Arena arena;
  bool dry = false;
  hipError_t hip_err = hipSuccess;
  int* dev_flags = nullptr;   // [0] error bits (1 bad norm, 2 SVD not converged, 4 guard hit)
  double* work = nullptr;     // device tallies of data-dependent work (profiling)
  uint64_t rng_calls = 0;     // counter of randomised truncations (seeds)
  void check(hipError_t e) {
    if (e != hipSuccess && hip_err == hipSuccess) {
      hip_err = e;
      if (std::getenv("CTM_DEBUG_HIP")) std::fprintf(stderr, "ctm: HIP error %s\n", hipGetErrorString(e));
    }
  }
  void check_launch() { check(hipGetLastError()); }
  Tensor alloc(int dt, std::initializer_list<int64_t> dims);
  Tensor alloc(int dt, const std::vector<int64_t>& dims);
};

// Launches a kernel that holds the stream for ~40 us (profiling only).
void prof_gate(hipStream_t stream);

// Records one launch (or a short sequence counted as `launches` launches of
// class cls) when profiling is on.  Two ways of timing:
// * a single kernel launched through launch(ps, ...) below carries the two
//   events in its own dispatch (hipExtLaunchKernelGGL), so they read the
//   kernel's start and end, the interval a kernel tracer reports;
// * otherwise HIP events are recorded on the stream around the scope, with a
//   gate kernel ahead of the start event that lets the host enqueue the
//   events and the launches before the stream reaches them (the interval
//   then holds the kernels and the event markers, not host issue time).
struct ProfScope {
  Ctx& c;
  int cls;
  double flops, bytes;
  int launches;
  bool ext;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(Ctx& cx, int k, double f, double b, int nl = 1, bool ext_launch = false)
      : c(cx), cls(k), flops(f), bytes(b), launches(nl), ext(ext_launch) {
    if (c.prof && !c.dry) {
      c.check(hipEventCreate(&e0));
      c.check(hipEventCreate(&e1));
      if (!ext) {
        prof_gate(c.stream);
        c.check(hipEventRecord(e0, c.stream));
      }
    }
  }
  ~ProfScope() {
    if (c.prof && !c.dry && e0) {
      if (!ext) c.check(hipEventRecord(e1, c.stream));
      c.prof->recs.push_back({cls, flops, bytes, e0, e1, launches});
    }
  }
};

// One kernel launch on `stream`; under a profiling scope made with
// ext_launch = true the scope's events ride on the dispatch.
template <typename F, typename... Args>
void launch(ProfScope& ps, F kernel, dim3 grid, dim3 block, hipStream_t stream, Args... args) {
  if (ps.ext && ps.e0 != nullptr)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ps.e0, ps.e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, args...);
}

// ---------------------------------------------------------------- kernels

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], row-major; op(A) is m x k.
// ta: A stored k x m (lda = row stride); tb: B stored n x k.
// dtype: F64 (A,B,C double), F32 (A,B,C float), BF16 (A,B bf16, C float).
void gemm(Ctx& c, int dtype, int m, int n, int k, double alpha, const void* A,
          int64_t lda, int ta, const void* B, int64_t ldb, int tb, double beta,
          void* C, int64_t ldc, int batch = 1, int64_t sA = 0, int64_t sB = 0,
          int64_t sC = 0);

// Most K slabs an FP64 product is split into.
constexpr int kMaxF64Splits = 32;

// The FP64 product op(A) op(B) (m x n, row-major) over K split into slabs
// of at least 128 (gemm() takes 64), for a consumer that sums the slabs
// itself: slab z of part (at z * m * n) holds the product over the z-th K
// range.  With one slab part holds the product itself.  part has
// room for gemm_f64_split_count(m, n, k) slabs (at most kMaxF64Splits).
// Returns the number of slabs.
int gemm_f64_split_count(int m, int n, int k);
int gemm_f64_partials(Ctx& c, int m, int n, int k, const double* A, int64_t lda, int ta,
                      const double* B, int64_t ldb, int tb, double* part);

// out = permute(in): out dims are in.dims[perm[i]]; dtype conversion allowed
// (F64 <-> F32 <-> BF16) with an optional scale applied on the way.
void permute(Ctx& c, const Tensor& in, const int* perm, Tensor& out,
             double scale = 1.0);

void fill(Ctx& c, void* p, int dt, int64_t n, double v);
void copy_bytes(Ctx& c, void* dst, const void* src, size_t bytes);

// Frobenius norm of x (F64) into *nrm (device); x *= 1/norm afterwards with
// normalize(); a zero or non-finite norm raises the numeric error flag.
void norm2(Ctx& c, const double* x, int64_t n, double* nrm);
void scale_by_inv(Ctx& c, double* x, int64_t n, const double* nrm);

// Truncated SVD of the row-major m x n F64 matrix M: U (m x kk, row-major)
// holds the top kk = min(k, m, n) left singular vectors (cutoff tau relative
// to sigma_0 zeroes columns; sign fixed), S (kk) the singular values.
// M is left unchanged.
void tsvd(Ctx& c, const double* M, int m, int n, int k, double tau, double* U,
          double* S);

// An orthonormal basis of the column space of the row-major m x n F64
// matrix M (m >= n) at Q (m x n, row-major): the columns of M in order of
// decreasing norm, orthonormalised; columns dependent on the earlier ones to
// working precision come out zero.
void range_basis(Ctx& c, const double* M, int m, int n, double* Q);

// Normalised singular values of a p x q corner, zero padded to chi.
void corner_spectrum(Ctx& c, const double* C, int p, int q, int chi, double* out);

// delta = max |a - b| over n entries, written to *out.
void max_abs_diff(Ctx& c, const double* a, const double* b, int n, double* out);

// Contract the reduced density matrix with h: out[0] = sum rho*h, out[1] = tr rho.
void rho_energy(Ctx& c, const double* rho, const double* h4, int d, double* out);

// One-site density matrix rho[s, S] with op[S, s] (d x d): out[0] = sum
// rho op, out[1] = tr rho.
void rho1_expect(Ctx& c, const double* rho, const double* op, int d, double* out);

// Connected correlation <op op> - <op><op> from the d x d right-end
// matrices with op (RO) and with the identity (RI) on the left site.
void corr_finish(Ctx& c, const double* RO, const double* RI, const double* op, int d,
                 double* out);

// Debug guard regions: fill with a sentinel; check sets bit 4 of the error
// word if any byte changed.
void guard_fill(Ctx& c, void* p, size_t bytes);
void guard_check(Ctx& c, const void* p, size_t bytes);

// General contraction helper: out(lo) = A(la) * B(lb), labels are single
// characters; no label may appear in all three.  compute: F64/F32/BF16;
// the result is written in out_dt.
Tensor contract(Ctx& c, const Tensor& A, const char* la, const Tensor& B,
                const char* lb, const char* lo, int compute, int out_dt);

// Permute to a label order.
Tensor relabel(Ctx& c, const Tensor& A, const char* la, const char* lo, int out_dt);

}  // namespace ctm

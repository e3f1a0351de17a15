// Index permutes, casts and reductions (HBM-bound kernels).
//
// The permute regroups tensor legs between the contractions of the move so
// that contracted legs are contiguous for the GEMM.  When the innermost leg
// survives it is a streaming copy; otherwise a 64 x 64 LDS tile transposes the
// run of trailing input legs against the run of output-innermost legs, so
// that both the reads and the writes are coalesced 64-element rows.  All
// reductions are two-pass with a fixed block count and a fixed summation
// order, so results are bitwise reproducible.
#include <cmath>

#include <cstdio>
#include <cstdlib>

#include "ctm_internal.h"

namespace ctm {
namespace {

struct PermArgs {
  int nd;
  int64_t dims[kMaxDims];   // by input dim
  int64_t sin[kMaxDims];    // input stride of each input dim
  int64_t sout[kMaxDims];   // output stride of each input dim
};

template <typename T> __device__ __forceinline__ double ld(const T* p, int64_t i) {
  return (double)p[i];
}
template <> __device__ __forceinline__ double ld<__bf16>(const __bf16* p, int64_t i) {
  return (double)(float)p[i];
}
template <typename T> __device__ __forceinline__ void st(T* p, int64_t i, double v) {
  p[i] = (T)v;
}
template <> __device__ __forceinline__ void st<float>(float* p, int64_t i, double v) {
  p[i] = (float)v;
}
template <> __device__ __forceinline__ void st<__bf16>(__bf16* p, int64_t i, double v) {
  p[i] = (__bf16)(float)v;
}

// innermost input dim is also the innermost output dim: rows are copied
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void permute_rows_kernel(const Ti* __restrict__ in,
                                                            To* __restrict__ out, PermArgs a,
                                                            int64_t total, double scale) {
  const int64_t inner = a.dims[a.nd - 1];
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * 256) {
    int64_t rem = o / inner;
    const int64_t x = o - rem * inner;
    int64_t oi = x, oo = x;
    for (int d = a.nd - 2; d >= 0; --d) {
      const int64_t cd = rem % a.dims[d];
      rem /= a.dims[d];
      oi += cd * a.sin[d];
      oo += cd * a.sout[d];
    }
    st(out, oo, ld(in, oi) * scale);
  }
}

// Composite tiles.  When the innermost input leg is also innermost in the
// output and shorter than 64 it is carried as a payload of P elements;
// otherwise P = 1.  A is the run of input legs just above the payload
// (contiguous in the input, so unit a sits at input offset a*P) and B the run
// of legs just above the payload in the output (unit b at output offset b*P).
// A tile holds TA units of A (TA*P <= 64 elements) by 64 units of B: every
// read is a run of TA*P contiguous input elements and every write a run of
// 64*P contiguous output elements, even when each leg is only as long as the
// bond dimension D.  The other offset of each side comes from decomposing the
// composite index once per workgroup.
struct PermTile {
  int na, nb, nr;
  int P, TA;                                // TA = 64 / P
  int64_t A, B;                             // lengths of the runs, in units
  int64_t adim[kMaxDims], aout[kMaxDims];   // A legs, innermost first; output strides
  int64_t bdim[kMaxDims], bin[kMaxDims];    // B legs, output-innermost first; input strides
  int64_t rdim[kMaxDims], rin[kMaxDims], rout[kMaxDims];   // the other legs
};

// PP: the payload length when fixed at compile time (1, or the bond
// dimension 8), 0 when it is read from p.P.
template <typename Ti, typename To, int PP>
__global__ __launch_bounds__(256) void permute_ctile_kernel(const Ti* __restrict__ in,
                                                             To* __restrict__ out, PermTile p,
                                                             int64_t ntA, int64_t ntB,
                                                             double scale) {
  __shared__ double tile[64][65];
  __shared__ int64_t aoff_out[64], boff_in[64];
  int64_t bid = blockIdx.x;
  const int64_t tA = bid % ntA;
  bid /= ntA;
  const int64_t tB = bid % ntB;
  int64_t rest = bid / ntB;
  int64_t bi = 0, bo = 0;
  for (int d = p.nr - 1; d >= 0; --d) {
    const int64_t cd = rest % p.rdim[d];
    rest /= p.rdim[d];
    bi += cd * p.rin[d];
    bo += cd * p.rout[d];
  }
  const int t = threadIdx.x;
  const int P = PP ? PP : p.P;
  const int TA = 64 / P;
  if (t < TA) {
    int64_t x = tA * TA + t, o = 0;
    for (int k = 0; k < p.na; ++k) {
      const int64_t q = x / p.adim[k];
      o += (x - q * p.adim[k]) * p.aout[k];
      x = q;
    }
    aoff_out[t] = o;
  } else if (t >= 64 && t < 128) {
    int64_t x = tB * 64 + (t - 64), o = 0;
    for (int k = 0; k < p.nb; ++k) {
      const int64_t q = x / p.bdim[k];
      o += (x - q * p.bdim[k]) * p.bin[k];
      x = q;
    }
    boff_in[t - 64] = o;
  }
  __syncthreads();
  // read: row j of the tile is B unit tB*64 + j, column c element c of the
  // A units tA*TA ... (TA*P contiguous input elements)
  const int tx = t & 63, ty = t >> 6;
  const int W = TA * P;
  const int64_t abase = tA * TA;
  const bool cin = tx < W && abase + tx / P < p.A;
  const int64_t ioff = bi + abase * P + tx;
#pragma unroll 4
  for (int j = ty; j < 64; j += 4) {
    double v = 0.0;
    if (cin && tB * 64 + j < p.B) v = ld(in, ioff + boff_in[j]);
    tile[j][tx] = v;
  }
  __syncthreads();
  // write: A unit al gets 64*P contiguous output elements
  const int R = 64 * P;
#pragma unroll 4
  for (int w = t; w < TA * R; w += 256) {
    const int al = w / R, rem = w - al * R;
    const int b = rem / P, e = rem - b * P;
    const int64_t ya = abase + al, yb = tB * 64 + b;
    if (ya < p.A && yb < p.B) st(out, bo + aoff_out[al] + yb * P + e, tile[b][al * P + e] * scale);
  }
}

template <typename Ti, typename To>
void launch_permute(Ctx& c, ProfScope& ps, const void* in, void* out, const PermArgs& a,
                    double scale) {
  int64_t total = 1;
  for (int d = 0; d < a.nd; ++d) total *= a.dims[d];
  if (total == 0) return;
  // which input dim is innermost in the output?
  int ib = 0;
  for (int d = 0; d < a.nd; ++d)
    if (a.sout[d] == 1 && a.dims[d] > 1) ib = d;
  const int ia = a.nd - 1;
  const bool shared = ib == ia || a.dims[ib] == 1;
  if (a.nd == 1 || (shared && a.dims[ia] >= 64)) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    launch(ps, permute_rows_kernel<Ti, To>, dim3((unsigned)blocks), dim3(256), c.stream,
           (const Ti*)in, (To*)out, a, total, scale);
  } else {
    // payload: the shared innermost leg (if any); B: the leg just above the
    // payload in the output and those that follow it there, up to 64 units,
    // leaving the leg just above the payload in the input to A; A: the input
    // legs above the payload not in B, up to 64 elements with the payload
    PermTile p;
    const int top = shared ? ia - 1 : ia;   // innermost leg of A
    p.P = shared ? (int)a.dims[ia] : 1;
    bool inb[kMaxDims] = {false}, ina[kMaxDims] = {false};
    int start = -1;
    for (int d = 0; d < a.nd; ++d)
      if (d != ia || !shared)
        if (a.sout[d] == p.P && a.dims[d] > 1) start = d;
    p.nb = 0;
    p.B = 1;
    for (int d = start; d >= 0 && p.B < 64;) {
      inb[d] = true;
      p.bdim[p.nb] = a.dims[d];
      p.bin[p.nb] = a.sin[d];
      ++p.nb;
      p.B *= a.dims[d];
      const int64_t next = a.sout[d] * a.dims[d];
      int nx = -1;
      for (int e = 0; e < a.nd; ++e)
        if (!inb[e] && e != top && a.sout[e] == next && a.dims[e] > 1) nx = e;
      d = nx;
    }
    p.na = 0;
    p.A = 1;
    for (int d = top; d >= 0 && !inb[d] && p.A * p.P < 64; --d) {
      ina[d] = true;
      p.adim[p.na] = a.dims[d];
      p.aout[p.na] = a.sout[d];
      ++p.na;
      p.A *= a.dims[d];
    }
    p.nr = 0;
    for (int d = 0; d < top + 1; ++d)
      if (!ina[d] && !inb[d]) {
        p.rdim[p.nr] = a.dims[d];
        p.rin[p.nr] = a.sin[d];
        p.rout[p.nr] = a.sout[d];
        ++p.nr;
      }
    p.TA = 64 / p.P;
    const int64_t ntA = (p.A + p.TA - 1) / p.TA, ntB = (p.B + 63) / 64;
    const dim3 grid((unsigned)(ntA * ntB * (total / (p.A * p.B * p.P))));
    if (p.P == 1)
      launch(ps, permute_ctile_kernel<Ti, To, 1>, grid, dim3(256), c.stream, (const Ti*)in,
             (To*)out, p, ntA, ntB, scale);
    else if (p.P == 8)
      launch(ps, permute_ctile_kernel<Ti, To, 8>, grid, dim3(256), c.stream, (const Ti*)in,
             (To*)out, p, ntA, ntB, scale);
    else
      launch(ps, permute_ctile_kernel<Ti, To, 0>, grid, dim3(256), c.stream, (const Ti*)in,
             (To*)out, p, ntA, ntB, scale);
  }
  c.check_launch();
}

__global__ void fill_kernel_f64(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}
__global__ void fill_kernel_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}
__global__ void fill_kernel_bf16(__bf16* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = (__bf16)v;
}

constexpr int kRedBlocks = 512;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // 256 threads: wave reduction via LDS tree (fixed order)
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void sumsq_partial(const double* __restrict__ x, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kRedBlocks * 256) {
    const double v = x[i];
    s += v * v;
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void sumsq_final(const double* __restrict__ part,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += 256) s += part[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = sqrt(t);
}

__global__ __launch_bounds__(256) void scale_inv_kernel(double* __restrict__ x, int64_t n,
                                                        const double* __restrict__ nrm,
                                                        int* __restrict__ flags) {
  const double v = nrm[0];
  const bool bad = !(v > 0.0) || !isfinite(v);
  if (bad) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flags[0] |= 1;
    return;
  }
  const double s = 1.0 / v;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    x[i] *= s;
}

__global__ __launch_bounds__(256) void max_abs_diff_kernel(const double* a, const double* b, int n,
                                                           double* out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(a[i] - b[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// rho[s1,s2,s1',s2'] (ket first); h4[s1',s2',s1,s2] = h[(s1' s2'),(s1 s2)]
__global__ void rho_energy_kernel(const double* rho, const double* h4, int d, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int s = 0; s < d; ++s)
    for (int t = 0; t < d; ++t) {
      den += rho[((s * d + t) * d + s) * d + t];
      for (int S = 0; S < d; ++S)
        for (int T = 0; T < d; ++T)
          num += rho[((s * d + t) * d + S) * d + T] * h4[((S * d + T) * d + s) * d + t];
    }
  out[0] = num;
  out[1] = den;
}

// one-site: out[0] = sum rho[s,S] op[S,s], out[1] = sum rho[s,s]
__global__ void rho1_expect_kernel(const double* rho, const double* op, int d, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int s = 0; s < d; ++s) {
    den += rho[s * d + s];
    for (int S = 0; S < d; ++S) num += rho[s * d + S] * op[S * d + s];
  }
  out[0] = num;
  out[1] = den;
}

// connected correlation from the right-end density matrices with op (RO)
// and with the identity (RI) on the left site:
// out = <op op> / <1 1> - (<op 1> / <1 1>) (<1 op> / <1 1>)
__global__ void corr_finish_kernel(const double* RO, const double* RI, const double* op, int d,
                                   double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double oo = 0.0, oi = 0.0, io = 0.0, ii = 0.0;
  for (int t = 0; t < d; ++t) {
    oi += RO[t * d + t];
    ii += RI[t * d + t];
    for (int T = 0; T < d; ++T) {
      oo += RO[t * d + T] * op[T * d + t];
      io += RI[t * d + T] * op[T * d + t];
    }
  }
  out[0] = oo / ii - (oi / ii) * (io / ii);
}

// guard regions (debug mode): a sentinel word everywhere, checked later
constexpr uint64_t kGuardWord = 0xA5A5A5A5A5A5A5A5ull;

__global__ __launch_bounds__(256) void guard_fill_kernel(uint64_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = kGuardWord;
}

__global__ __launch_bounds__(256) void guard_check_kernel(const uint64_t* p, int64_t n, int* flags) {
  bool bad = false;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad |= p[i] != kGuardWord;
  if (bad) atomicOr(flags, 4);
}

// Profiling gate: holds the stream for about `ticks` periods of the
// constant-rate wall clock (bounded by an iteration cap whatever the clock
// does), so the host has enqueued the timing events and the kernel behind
// it before the stream reaches them.
__global__ void prof_gate_kernel(long long ticks) {
  const long long t0 = wall_clock64();
  for (int it = 0; it < 200000; ++it) {
    if (wall_clock64() - t0 >= ticks) break;
    __builtin_amdgcn_s_sleep(2);
  }
}

}  // namespace

void prof_gate(hipStream_t stream) {
  static const long long ticks = [] {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    return (long long)khz * 40 / 1000;   // 40 microseconds
  }();
  hipLaunchKernelGGL(prof_gate_kernel, dim3(1), dim3(64), 0, stream, ticks);
}

void guard_fill(Ctx& c, void* p, size_t bytes) {
  if (c.dry || bytes < 8) return;
  hipLaunchKernelGGL(guard_fill_kernel, dim3(64), dim3(256), 0, c.stream, (uint64_t*)p,
                     (int64_t)(bytes / 8));
  c.check_launch();
}

void guard_check(Ctx& c, const void* p, size_t bytes) {
  if (c.dry || bytes < 8 || !c.dev_flags) return;
  hipLaunchKernelGGL(guard_check_kernel, dim3(64), dim3(256), 0, c.stream, (const uint64_t*)p,
                     (int64_t)(bytes / 8), c.dev_flags);
  c.check_launch();
}

void rho1_expect(Ctx& c, const double* rho, const double* op, int d, double* out) {
  if (c.dry) return;
  hipLaunchKernelGGL(rho1_expect_kernel, dim3(1), dim3(64), 0, c.stream, rho, op, d, out);
  c.check_launch();
}

void corr_finish(Ctx& c, const double* RO, const double* RI, const double* op, int d,
                 double* out) {
  if (c.dry) return;
  hipLaunchKernelGGL(corr_finish_kernel, dim3(1), dim3(64), 0, c.stream, RO, RI, op, d, out);
  c.check_launch();
}

Tensor make_view(void* p, int dt, std::initializer_list<int64_t> dims) {
  Tensor t;
  t.p = p;
  t.dt = dt;
  t.nd = 0;
  for (int64_t d : dims) t.dims[t.nd++] = d;
  return t;
}

Tensor make_view(void* p, int dt, const std::vector<int64_t>& dims) {
  Tensor t;
  t.p = p;
  t.dt = dt;
  t.nd = (int)dims.size();
  for (int i = 0; i < t.nd; ++i) t.dims[i] = dims[i];
  return t;
}

void* Arena::alloc(size_t bytes) {
  const size_t al = 256;
  size_t off = (top + al - 1) / al * al;
  top = off + bytes;
  if (top > peak) peak = top;
  if (!dry && top > cap) {
    overflow = true;
    throw Error(2, "workspace exhausted");
  }
  return (void*)(base + off);
}

Tensor Ctx::alloc(int dt, std::initializer_list<int64_t> dims) {
  Tensor t = make_view(nullptr, dt, dims);
  t.p = arena.alloc(t.bytes());
  return t;
}

Tensor Ctx::alloc(int dt, const std::vector<int64_t>& dims) {
  Tensor t = make_view(nullptr, dt, dims);
  t.p = arena.alloc(t.bytes());
  return t;
}

void Profiler::collect() {
  for (Rec& r : recs) {
    float ms_ = 0.0f;
    if (hipEventElapsedTime(&ms_, r.e0, r.e1) == hipSuccess) {
      n[r.cls] += r.launches;
      ms[r.cls] += ms_;
      flops[r.cls] += r.flops;
      bytes[r.cls] += r.bytes;
    }
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  recs.clear();
}

void Profiler::clear() {
  for (Rec& r : recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  recs.clear();
  for (int i = 0; i < K_NCLASS; ++i) {
    n[i] = 0;
    ms[i] = flops[i] = bytes[i] = 0.0;
  }
}

void permute(Ctx& c, const Tensor& in, const int* perm, Tensor& out, double scale) {
  if (std::getenv("CTM_DEBUG_PERM") && in.numel() >= (1 << 20)) {
    std::fprintf(stderr, "permute dt %d->%d dims", in.dt, out.dt);
    for (int i = 0; i < in.nd; ++i) std::fprintf(stderr, " %lld", (long long)in.dims[i]);
    std::fprintf(stderr, " perm");
    for (int i = 0; i < in.nd; ++i) std::fprintf(stderr, " %d", perm[i]);
    std::fprintf(stderr, "\n");
  }
  if (c.dry || in.numel() == 0) return;
  ProfScope ps(c, K_PERMUTE, 0.0,
               (double)in.numel() * (double)(dtype_size(in.dt) + dtype_size(out.dt)), 1, true);
  // merge input dims that stay adjacent and in order; drop size-1 dims
  int nd = in.nd;
  int64_t ostr[kMaxDims];
  {
    int64_t s = 1;
    for (int i = nd - 1; i >= 0; --i) {
      ostr[perm[i]] = s;
      s *= in.dims[perm[i]];
    }
  }
  PermArgs a;
  a.nd = 0;
  int64_t istr[kMaxDims];
  {
    int64_t s = 1;
    for (int i = nd - 1; i >= 0; --i) {
      istr[i] = s;
      s *= in.dims[i];
    }
  }
  for (int i = 0; i < nd; ++i) {
    if (in.dims[i] == 1) continue;
    if (a.nd > 0) {
      const int j = a.nd - 1;
      // previous kept dim j can absorb dim i if dim i follows it in both orders
      if (a.sin[j] == istr[i] * in.dims[i] && a.sout[j] == ostr[i] * in.dims[i]) {
        a.dims[j] *= in.dims[i];
        a.sin[j] = istr[i];
        a.sout[j] = ostr[i];
        continue;
      }
    }
    a.dims[a.nd] = in.dims[i];
    a.sin[a.nd] = istr[i];
    a.sout[a.nd] = ostr[i];
    ++a.nd;
  }
  if (a.nd == 0) {
    a.nd = 1;
    a.dims[0] = 1;
    a.sin[0] = 1;
    a.sout[0] = 1;
  }
#define CTM_PERM(TI, TO) launch_permute<TI, TO>(c, ps, in.p, out.p, a, scale)
  if (in.dt == F64 && out.dt == F64) CTM_PERM(double, double);
  else if (in.dt == F64 && out.dt == F32) CTM_PERM(double, float);
  else if (in.dt == F64 && out.dt == BF16) CTM_PERM(double, __bf16);
  else if (in.dt == F32 && out.dt == F64) CTM_PERM(float, double);
  else if (in.dt == F32 && out.dt == F32) CTM_PERM(float, float);
  else if (in.dt == F32 && out.dt == BF16) CTM_PERM(float, __bf16);
  else if (in.dt == BF16 && out.dt == F64) CTM_PERM(__bf16, double);
  else if (in.dt == BF16 && out.dt == F32) CTM_PERM(__bf16, float);
  else CTM_PERM(__bf16, __bf16);
#undef CTM_PERM
}

__global__ __launch_bounds__(256) void copy_u64_kernel(uint64_t* __restrict__ dst,
                                                       const uint64_t* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void copy_u8_kernel(unsigned char* __restrict__ dst,
                                                      const unsigned char* __restrict__ src,
                                                      int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

// Device-to-device copy as a kernel (a plain kernel node when captured).
void copy_bytes(Ctx& c, void* dst, const void* src, size_t bytes) {
  if (c.dry || bytes == 0) return;
  const bool w8 = bytes % 8 == 0 && ((uintptr_t)dst % 8) == 0 && ((uintptr_t)src % 8) == 0;
  const int64_t n = w8 ? (int64_t)(bytes / 8) : (int64_t)bytes;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (w8)
    hipLaunchKernelGGL(copy_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (uint64_t*)dst, (const uint64_t*)src, n);
  else
    hipLaunchKernelGGL(copy_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (unsigned char*)dst, (const unsigned char*)src, n);
  c.check_launch();
}

void fill(Ctx& c, void* p, int dt, int64_t n, double v) {
  if (c.dry || n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (dt == F64)
    hipLaunchKernelGGL(fill_kernel_f64, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (double*)p, n, v);
  else if (dt == F32)
    hipLaunchKernelGGL(fill_kernel_f32, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (float*)p, n, (float)v);
  else
    hipLaunchKernelGGL(fill_kernel_bf16, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (__bf16*)p, n, (float)v);
  c.check_launch();
}

void norm2(Ctx& c, const double* x, int64_t n, double* nrm) {
  double* part = (double*)c.arena.alloc(kRedBlocks * sizeof(double));
  if (c.dry) return;
  ProfScope ps(c, K_REDUCE, 2.0 * n, 8.0 * n);
  hipLaunchKernelGGL(sumsq_partial, dim3(kRedBlocks), dim3(256), 0, c.stream, x, n, part);
  hipLaunchKernelGGL(sumsq_final, dim3(1), dim3(256), 0, c.stream, part, nrm);
  c.check_launch();
}

void scale_by_inv(Ctx& c, double* x, int64_t n, const double* nrm) {
  if (c.dry) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  ProfScope ps(c, K_REDUCE, (double)n, 16.0 * n);
  hipLaunchKernelGGL(scale_inv_kernel, dim3((unsigned)blocks), dim3(256), 0, c.stream, x, n, nrm,
                     c.dev_flags);
  c.check_launch();
}

void max_abs_diff(Ctx& c, const double* a, const double* b, int n, double* out) {
  if (c.dry) return;
  hipLaunchKernelGGL(max_abs_diff_kernel, dim3(1), dim3(256), 0, c.stream, a, b, n, out);
  c.check_launch();
}

void rho_energy(Ctx& c, const double* rho, const double* h4, int d, double* out) {
  if (c.dry) return;
  hipLaunchKernelGGL(rho_energy_kernel, dim3(1), dim3(64), 0, c.stream, rho, h4, d, out);
  c.check_launch();
}

}  // namespace ctm

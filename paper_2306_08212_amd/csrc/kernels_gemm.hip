// Dense GEMM kernels on the gfx950 matrix cores.
//
// Every contraction of the corner-transfer move (the enlarged-corner products,
// the ket-then-bra absorption chain, the projector applications and the
// energy networks) is lowered to C = alpha * op(A) op(B) + beta * C on
// row-major operands.  Three element types:
//   F64  : v_mfma_f64_16x16x4f64, 64 x 64 tile per workgroup
//   F32  : v_mfma_f32_32x32x2f32, 128 x 128 tile
//   BF16 : v_mfma_f32_32x32x16_bf16 (bf16 in, fp32 accumulate/out), 128 x 128
// Ragged edges are zero-filled on the way into LDS; nothing is read or
// written outside [0,m) x [0,n).
#include <algorithm>

#include <cstdio>
#include <cstdlib>

#include "ctm_internal.h"

namespace ctm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- FP64

constexpr int F64_BM = 64, F64_BN = 64, F64_BK = 32;
constexpr int F64_PER = F64_BM * F64_BK / 256;   // elements of each operand per thread

// Split-K: blockIdx.z takes K range [z * kchunk, min(K, (z + 1) * kchunk)).
// With part != nullptr the raw partial products go to part (one M x N slab
// per (z, batch) pair) and a separate pass sums them in a fixed order.
// The next K tile is fetched into registers while the current one is
// multiplied from LDS.
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, int64_t lda, int ta,
    const double* __restrict__ B, int64_t ldb, int tb, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sA, int64_t sB, int64_t sC, int tiles_n, int kchunk,
    double* __restrict__ part) {
  __shared__ double As[F64_BK][F64_BM + 2];
  __shared__ double Bs[F64_BK][F64_BN + 2];
  const int bz = blockIdx.y;
  A += sA * bz;
  B += sB * bz;
  C += sC * bz;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tile = blockIdx.x;
  const int m0 = (tile / tiles_n) * F64_BM, n0 = (tile % tiles_n) * F64_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[F64_PER], rb[F64_PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < F64_PER; ++q) {
      const int e = tid + 256 * q;
      int mm, kk;
      if (!ta) { mm = e / F64_BK; kk = e % F64_BK; } else { kk = e / F64_BM; mm = e % F64_BM; }
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < M && gk < kend) ? (ta ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0;
      int nn, kb;
      if (!tb) { kb = e / F64_BN; nn = e % F64_BN; } else { nn = e / F64_BK; kb = e % F64_BK; }
      const int gn = n0 + nn, gkb = k0 + kb;
      rb[q] = (gn < N && gkb < kend) ? (tb ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn]) : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < F64_PER; ++q) {
      const int e = tid + 256 * q;
      int mm, kk;
      if (!ta) { mm = e / F64_BK; kk = e % F64_BK; } else { kk = e / F64_BM; mm = e % F64_BM; }
      As[kk][mm] = ra[q];
      int nn, kb;
      if (!tb) { kb = e / F64_BN; nn = e % F64_BN; } else { nn = e / F64_BK; kb = e % F64_BK; }
      Bs[kb][nn] = rb[q];
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += F64_BK) {
    stash();
    __syncthreads();
    if (k0 + F64_BK < kend) fetch(k0 + F64_BK);
#pragma unroll
    for (int kk = 0; kk < F64_BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a0 = As[kr][wm + (lane & 15)];
      const double a1 = As[kr][wm + 16 + (lane & 15)];
      const double b0 = Bs[kr][wn + (lane & 15)];
      const double b1 = Bs[kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of 16x16x4 f64 (checked on gfx950): lane l, element r ->
  // row l/16 + 4*r, col l%16
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          if (part != nullptr) {
            part[(((int64_t)blockIdx.z * gridDim.y + bz) * M + gm) * N + gn] = acc[i][j][r];
          } else {
            double* cp = C + (int64_t)gm * ldc + gn;
            const double v = alpha * acc[i][j][r];
            *cp = (beta == 0.0) ? v : v + beta * (*cp);
          }
        }
      }
}

// C = alpha * sum_z part[z] + beta * C, summed in z order.
__global__ __launch_bounds__(256) void gemm_f64_splitk_sum(int M, int N, int batch, int splits,
                                                           double alpha,
                                                           const double* __restrict__ part,
                                                           double beta, double* __restrict__ C,
                                                           int64_t ldc, int64_t sC) {
  const int64_t per = (int64_t)M * N, total = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    // eight slabs' loads in flight, summed in z order
    double acc = 0.0;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * total + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; z < splits; ++z) acc += part[(int64_t)z * total + e];
    const int64_t bz = e / per, r = e % per;
    const int gm = (int)(r / N), gn = (int)(r % N);
    double* cp = C + sC * bz + (int64_t)gm * ldc + gn;
    const double v = alpha * acc;
    *cp = (beta == 0.0) ? v : v + beta * (*cp);
  }
}

// ---------------------------------------------------------------- FP32

constexpr int F32_BM = 128, F32_BN = 128, F32_BK = 16;

__global__ __launch_bounds__(256) void gemm_f32_kernel(
    int M, int N, int K, float alpha, const float* __restrict__ A, int64_t lda, int ta,
    const float* __restrict__ B, int64_t ldb, int tb, float beta, float* __restrict__ C,
    int64_t ldc, int64_t sA, int64_t sB, int64_t sC, int tiles_n) {
  __shared__ float As[F32_BK][F32_BM + 4];
  __shared__ float Bs[F32_BK][F32_BN + 4];
  const int bz = blockIdx.y;
  A += sA * bz;
  B += sB * bz;
  C += sC * bz;
  const int tile = blockIdx.x;
  const int m0 = (tile / tiles_n) * F32_BM, n0 = (tile % tiles_n) * F32_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f16v acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  // tiles are fetched as 16-byte vectors along the operand's contiguous
  // dimension (two per operand and thread) when the leading dimension and
  // the base keep them aligned; ragged edges fall back to guarded scalars
  const bool va = (lda % 4 == 0) && (((uintptr_t)A & 15) == 0);
  const bool vb = (ldb % 4 == 0) && (((uintptr_t)B & 15) == 0);
  float4 ra[2], rb[2];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q4 = tid + 256 * h;
      // A: ta = 0 is m x k (quads along k), ta = 1 is k x m (quads along m)
      {
        const int mm = ta ? (q4 % (F32_BM / 4)) * 4 : q4 / (F32_BK / 4);
        const int kk = ta ? q4 / (F32_BM / 4) : (q4 % (F32_BK / 4)) * 4;
        const int gm = m0 + mm, gk = k0 + kk;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (!ta) {
          if (va && gm < M && gk + 3 < K) {
            v = *reinterpret_cast<const float4*>(A + (int64_t)gm * lda + gk);
          } else if (gm < M) {
            const float* p = A + (int64_t)gm * lda;
            v.x = gk < K ? p[gk] : 0.0f;
            v.y = gk + 1 < K ? p[gk + 1] : 0.0f;
            v.z = gk + 2 < K ? p[gk + 2] : 0.0f;
            v.w = gk + 3 < K ? p[gk + 3] : 0.0f;
          }
        } else {
          if (va && gk < K && gm + 3 < M) {
            v = *reinterpret_cast<const float4*>(A + (int64_t)gk * lda + gm);
          } else if (gk < K) {
            const float* p = A + (int64_t)gk * lda;
            v.x = gm < M ? p[gm] : 0.0f;
            v.y = gm + 1 < M ? p[gm + 1] : 0.0f;
            v.z = gm + 2 < M ? p[gm + 2] : 0.0f;
            v.w = gm + 3 < M ? p[gm + 3] : 0.0f;
          }
        }
        ra[h] = v;
      }
      // B: tb = 0 is k x n (quads along n), tb = 1 is n x k (quads along k)
      {
        const int nn = tb ? q4 / (F32_BK / 4) : (q4 % (F32_BN / 4)) * 4;
        const int kk = tb ? (q4 % (F32_BK / 4)) * 4 : q4 / (F32_BN / 4);
        const int gn = n0 + nn, gk = k0 + kk;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (!tb) {
          if (vb && gk < K && gn + 3 < N) {
            v = *reinterpret_cast<const float4*>(B + (int64_t)gk * ldb + gn);
          } else if (gk < K) {
            const float* p = B + (int64_t)gk * ldb;
            v.x = gn < N ? p[gn] : 0.0f;
            v.y = gn + 1 < N ? p[gn + 1] : 0.0f;
            v.z = gn + 2 < N ? p[gn + 2] : 0.0f;
            v.w = gn + 3 < N ? p[gn + 3] : 0.0f;
          }
        } else {
          if (vb && gn < N && gk + 3 < K) {
            v = *reinterpret_cast<const float4*>(B + (int64_t)gn * ldb + gk);
          } else if (gn < N) {
            const float* p = B + (int64_t)gn * ldb;
            v.x = gk < K ? p[gk] : 0.0f;
            v.y = gk + 1 < K ? p[gk + 1] : 0.0f;
            v.z = gk + 2 < K ? p[gk + 2] : 0.0f;
            v.w = gk + 3 < K ? p[gk + 3] : 0.0f;
          }
        }
        rb[h] = v;
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q4 = tid + 256 * h;
      {
        const int mm = ta ? (q4 % (F32_BM / 4)) * 4 : q4 / (F32_BK / 4);
        const int kk = ta ? q4 / (F32_BM / 4) : (q4 % (F32_BK / 4)) * 4;
        if (!ta) {
          As[kk][mm] = ra[h].x;
          As[kk + 1][mm] = ra[h].y;
          As[kk + 2][mm] = ra[h].z;
          As[kk + 3][mm] = ra[h].w;
        } else {
          *reinterpret_cast<float4*>(&As[kk][mm]) = ra[h];
        }
      }
      {
        const int nn = tb ? q4 / (F32_BK / 4) : (q4 % (F32_BN / 4)) * 4;
        const int kk = tb ? (q4 % (F32_BK / 4)) * 4 : q4 / (F32_BN / 4);
        if (!tb) {
          *reinterpret_cast<float4*>(&Bs[kk][nn]) = rb[h];
        } else {
          Bs[kk][nn] = rb[h].x;
          Bs[kk + 1][nn] = rb[h].y;
          Bs[kk + 2][nn] = rb[h].z;
          Bs[kk + 3][nn] = rb[h].w;
        }
      }
    }
  };
  load_tiles(0);
  for (int k0 = 0; k0 < K; k0 += F32_BK) {
    store_tiles();
    __syncthreads();
    if (k0 + F32_BK < K) load_tiles(k0 + F32_BK);
#pragma unroll
    for (int kk = 0; kk < F32_BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float a0 = As[kr][wm + (lane & 31)];
      const float a1 = As[kr][wm + 32 + (lane & 31)];
      const float b0 = Bs[kr][wn + (lane & 31)];
      const float b1 = Bs[kr][wn + 32 + (lane & 31)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of 32x32 f32 (checked on gfx950): lane l, element j ->
  // row 8*(j/4) + 4*(l/32) + j%4, col l%32
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn + j * 32 + (lane & 31);
        if (gm < M && gn < N) {
          float* cp = C + (int64_t)gm * ldc + gn;
          const float v = alpha * acc[i][j][r];
          *cp = (beta == 0.0f) ? v : v + beta * (*cp);
        }
      }
}

// ---------------------------------------------------------------- BF16

constexpr int B16_BM = 128, B16_BN = 128, B16_BK = 32;

// LDS holds A as [m][k] and B as [n][k] so each lane's 8 consecutive k
// values are one 16-byte read.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(
    int M, int N, int K, float alpha, const __bf16* __restrict__ A, int64_t lda, int ta,
    const __bf16* __restrict__ B, int64_t ldb, int tb, float beta, float* __restrict__ C,
    int64_t ldc, int64_t sA, int64_t sB, int64_t sC, int tiles_n) {
  __shared__ __attribute__((aligned(16))) __bf16 As[B16_BM][B16_BK + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[B16_BN][B16_BK + 8];
  const int bz = blockIdx.y;
  A += sA * bz;
  B += sB * bz;
  C += sC * bz;
  const int tile = blockIdx.x;
  const int m0 = (tile / tiles_n) * B16_BM, n0 = (tile % tiles_n) * B16_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f16v acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  const __bf16 zero = (__bf16)0.0f;
  for (int k0 = 0; k0 < K; k0 += B16_BK) {
    for (int e = tid; e < B16_BM * B16_BK; e += 256) {
      int mm, kk;
      if (!ta) { mm = e / B16_BK; kk = e % B16_BK; } else { kk = e / B16_BM; mm = e % B16_BM; }
      const int gm = m0 + mm, gk = k0 + kk;
      __bf16 v = zero;
      if (gm < M && gk < K) v = ta ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[mm][kk] = v;
      int nn;
      if (!tb) { kk = e / B16_BN; nn = e % B16_BN; } else { nn = e / B16_BK; kk = e % B16_BK; }
      const int gn = n0 + nn, gk2 = k0 + kk;
      __bf16 w = zero;
      if (gn < N && gk2 < K) w = tb ? B[(int64_t)gn * ldb + gk2] : B[(int64_t)gk2 * ldb + gn];
      Bs[nn][kk] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < B16_BK; kk += 16) {
      const int kc = kk + (lane >> 5) * 8;
      const bf8 a0 = *(const bf8*)&As[wm + (lane & 31)][kc];
      const bf8 a1 = *(const bf8*)&As[wm + 32 + (lane & 31)][kc];
      const bf8 b0 = *(const bf8*)&Bs[wn + (lane & 31)][kc];
      const bf8 b1 = *(const bf8*)&Bs[wn + 32 + (lane & 31)][kc];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn + j * 32 + (lane & 31);
        if (gm < M && gn < N) {
          float* cp = C + (int64_t)gm * ldc + gn;
          const float v = alpha * acc[i][j][r];
          *cp = (beta == 0.0f) ? v : v + beta * (*cp);
        }
      }
}

// K split of an FP64 product whose grid cannot fill the chip: the number of
// slabs (1: none) and the K extent of each, at least kmin.  These products
// are short latency chains per workgroup, so slabs of 64 (two K tiles) make
// them fastest; the block Grams of the QR steps take 128, because every
// workgroup of the Cholesky kernel sums all their slabs.
int f64_splits(int m, int n, int k, int batch, int* kchunk, int kmin = 64) {
  *kchunk = k;
  const int64_t tiles = (int64_t)((m + F64_BM - 1) / F64_BM) * ((n + F64_BN - 1) / F64_BN) * batch;
  if (tiles >= 256 || k < 256) return 1;
  int64_t want = (512 + tiles - 1) / tiles;
  want = std::min<int64_t>(want, std::min<int64_t>(kMaxF64Splits, k / kmin));
  if (want <= 1) return 1;
  *kchunk = (int)(((k + want - 1) / want + F64_BK - 1) / F64_BK) * F64_BK;
  return (k + *kchunk - 1) / *kchunk;
}

}  // namespace

int gemm_f64_split_count(int m, int n, int k) {
  int kchunk = k;
  return f64_splits(m, n, std::max(k, 0), 1, &kchunk, 128);
}

int gemm_f64_partials(Ctx& c, int m, int n, int k, const double* A, int64_t lda, int ta,
                      const double* B, int64_t ldb, int tb, double* part) {
  if (m <= 0 || n <= 0) return 0;
  if (k < 0) k = 0;
  int kchunk = k;
  const int splits = f64_splits(m, n, k, 1, &kchunk, 128);
  if (c.dry) return splits;
  const int tm = (m + F64_BM - 1) / F64_BM, tn = (n + F64_BN - 1) / F64_BN;
  ProfScope ps(c, K_GEMM_F64, 2.0 * m * n * (double)k,
               ((double)m * k + (double)k * n) * 8.0 + (double)m * n * 8.0 * splits, 1, true);
  // one slab: the product itself (alpha = 1, beta = 0, which the kernel
  // stores as alpha * acc, i.e. acc); several: the raw slabs
  launch(ps, gemm_f64_kernel, dim3(tm * tn, 1, splits), dim3(256), c.stream, m, n, k, 1.0, A, lda,
         ta, B, ldb, tb, 0.0, splits > 1 ? (double*)nullptr : part, (int64_t)n, (int64_t)0, (int64_t)0, (int64_t)0, tn, kchunk,
         splits > 1 ? part : (double*)nullptr);
  return splits;
}

void gemm(Ctx& c, int dtype, int m, int n, int k, double alpha, const void* A, int64_t lda,
          int ta, const void* B, int64_t ldb, int tb, double beta, void* C, int64_t ldc,
          int batch, int64_t sA, int64_t sB, int64_t sC) {
  if (m <= 0 || n <= 0 || batch <= 0) return;
  if (k < 0) k = 0;
  if (std::getenv("CTM_DEBUG_GEMM") && (double)m * n * k * batch >= 1e9 && !c.dry)
    std::fprintf(stderr, "gemm dt %d m %d n %d k %d batch %d ta %d tb %d\n", dtype, m, n, k, batch,
                 ta, tb);
  // FP64 grids that cannot fill the chip split K (partials in the arena,
  // summed in a fixed order by a second pass, so results stay bitwise
  // reproducible)
  int splits = 1, kchunk = k;
  double* part = nullptr;
  size_t mk = c.arena.mark();
  if (dtype == F64) {
    const bool have_arena = c.arena.dry || c.arena.base != nullptr;
    if (have_arena) splits = f64_splits(m, n, k, batch, &kchunk);
    if (splits > 1) {
      part = (double*)c.arena.alloc(sizeof(double) * (size_t)splits * batch * m * n);
      if (part == nullptr && !c.dry) {   // no room: one pass over K
        splits = 1;
        kchunk = k;
      }
    }
  }
  if (c.dry) {
    c.arena.release(mk);
    return;
  }
  // k == 0 needs no special case: the K loop is empty and C = beta * C.
  const double es = dtype == F64 ? 8.0 : (dtype == F32 ? 4.0 : 2.0);
  const double eo = dtype == F64 ? 8.0 : 4.0;
  if (dtype == F64) {
    const int tm = (m + F64_BM - 1) / F64_BM, tn = (n + F64_BN - 1) / F64_BN;
    dim3 grid(tm * tn, batch, splits);
    {
      ProfScope ps(c, K_GEMM_F64, 2.0 * m * n * (double)k * batch,
                   ((double)m * k + (double)k * n) * es * batch +
                       (double)m * n * eo * batch * splits, 1, true);
      launch(ps, gemm_f64_kernel, grid, dim3(256), c.stream, m, n, k, alpha,
                         (const double*)A, lda, ta, (const double*)B, ldb, tb, beta, (double*)C,
                         ldc, sA, sB, sC, tn, kchunk, part);
    }
    if (splits > 1) {
      ProfScope ps(c, K_REDUCE, (double)m * n * batch * splits,
                   (double)m * n * batch * 8.0 * (splits + 1), 1, true);
      int64_t blocks = ((int64_t)m * n * batch + 255) / 256;
      if (blocks > 4096) blocks = 4096;
      launch(ps, gemm_f64_splitk_sum, dim3((unsigned)blocks), dim3(256), c.stream, m, n,
                         batch, splits, alpha, part, beta, (double*)C, ldc, sC);
    }
  } else if (dtype == F32) {
    ProfScope ps(c, K_GEMM_F32, 2.0 * m * n * (double)k * batch,
                 ((double)m * k + (double)k * n) * es * batch + (double)m * n * eo * batch, 1,
                 true);
    const int tm = (m + F32_BM - 1) / F32_BM, tn = (n + F32_BN - 1) / F32_BN;
    dim3 grid(tm * tn, batch);
    launch(ps, gemm_f32_kernel, grid, dim3(256), c.stream, m, n, k, (float)alpha,
                       (const float*)A, lda, ta, (const float*)B, ldb, tb, (float)beta,
                       (float*)C, ldc, sA, sB, sC, tn);
  } else {
    ProfScope ps(c, K_GEMM_BF16, 2.0 * m * n * (double)k * batch,
                 ((double)m * k + (double)k * n) * es * batch + (double)m * n * eo * batch, 1,
                 true);
    const int tm = (m + B16_BM - 1) / B16_BM, tn = (n + B16_BN - 1) / B16_BN;
    dim3 grid(tm * tn, batch);
    launch(ps, gemm_bf16_kernel, grid, dim3(256), c.stream, m, n, k, (float)alpha,
                       (const __bf16*)A, lda, ta, (const __bf16*)B, ldb, tb, (float)beta,
                       (float*)C, ldc, sA, sB, sC, tn);
  }
  c.check_launch();
  c.arena.release(mk);
}

}  // namespace ctm

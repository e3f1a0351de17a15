// Kernel-level C-ABI: thin argument checks around the launch wrappers.
#include "../../include/ctm.h"
#include "../../include/ctm_kernels.h"
#include "ctm_internal.h"

#include <mutex>

using namespace ctm;

// Device-resident scratch of the allocation-free truncation
// (ctm_kernel_tsvd_static): one copy per GPU, held until the process ends.
// Host code never uses the symbol's name as an address: the device address
// is looked up once per device with hipGetSymbolAddress and kept below.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch (looked up on the first call on
// that device, with that device current), or nullptr on a HIP error.
void* scratch_of_current_device(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int ctm_kernel_gemm(int dtype, int m, int n, int k, double alpha, const void* A, int64_t lda,
                    int ta, const void* B, int64_t ldb, int tb, double beta, void* C,
                    int64_t ldc, void* stream) {
  if (dtype < 0 || dtype > 2 || m < 0 || n < 0 || k < 0 || !C) return CTM_EINVAL;
  if (k > 0 && (!A || !B)) return CTM_EINVAL;
  Ctx c;
  c.stream = (hipStream_t)stream;
  gemm(c, dtype, m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc);
  return c.hip_err == hipSuccess ? CTM_OK : CTM_EHIP;
}

// The truncation with its error word (one int in the workspace, cleared
// first): set when a Jacobi solve did not converge.
static void tsvd_flagged(Ctx& c, const double* M, int m, int n, int k, double tau, double* U,
                         double* S) {
  c.dev_flags = (int*)c.arena.alloc(sizeof(int) * 4);
  if (!c.dry) fill(c, c.dev_flags, F32, 4, 0.0);   // zero bit pattern
  tsvd(c, M, m, n, k, tau, U, S);
}

size_t ctm_kernel_tsvd_workspace(int m, int n, int k) {
  if (m < 1 || n < 1 || k < 1) return 0;
  Ctx c;
  c.dry = true;
  c.arena.dry = true;
  tsvd_flagged(c, nullptr, m, n, k, 0.0, nullptr, nullptr);
  return c.arena.peak + 256;
}

int ctm_kernel_tsvd(const double* M, int m, int n, int k, double tau, double* U, double* S,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!M || !U || !S || m < 1 || n < 1 || k < 1 || !(tau >= 0.0)) return CTM_EINVAL;
  if (!workspace || workspace_bytes < ctm_kernel_tsvd_workspace(m, n, k)) return CTM_ENOMEM;
  Ctx c;
  c.stream = (hipStream_t)stream;
  c.arena.base = (char*)workspace;
  c.arena.cap = workspace_bytes;
  try {
    tsvd_flagged(c, M, m, n, k, tau, U, S);
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return c.hip_err == hipSuccess ? CTM_EINVAL : CTM_EHIP;
  }
  int flag = 0;
  c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  c.check(hipStreamSynchronize(c.stream));
  if (c.hip_err != hipSuccess) return CTM_EHIP;
  return flag ? CTM_ENUMERIC : CTM_OK;
}

size_t ctm_kernel_tsvd_static_max(void) { return kStaticScratchBytes; }

int ctm_kernel_tsvd_static(const double* M, int m, int n, int k, double tau, double* U, double* S,
                           void* stream) {
  if (!M || !U || !S || m < 1 || n < 1 || k < 1 || !(tau >= 0.0)) return CTM_EINVAL;
  const size_t need = ctm_kernel_tsvd_workspace(m, n, k);
  if (need == 0 || need > kStaticScratchBytes) return CTM_ENOMEM;
  hipError_t err = hipSuccess;
  void* ws = scratch_of_current_device(&err);
  if (ws == nullptr) return CTM_EHIP;
  Ctx c;
  c.stream = (hipStream_t)stream;
  c.arena.base = (char*)ws;
  c.arena.cap = kStaticScratchBytes;
  try {
    tsvd_flagged(c, M, m, n, k, tau, U, S);
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return c.hip_err == hipSuccess ? CTM_EINVAL : CTM_EHIP;
  }
  int flag = 0;
  c.check(hipMemcpyAsync(&flag, c.dev_flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  c.check(hipStreamSynchronize(c.stream));
  if (c.hip_err != hipSuccess) return CTM_EHIP;
  return flag ? CTM_ENUMERIC : CTM_OK;
}

int ctm_kernel_permute(int dt_in, const void* in, int nd, const int64_t* dims, const int* perm,
                       int dt_out, void* out, double scale, void* stream) {
  if (!in || !out || !dims || !perm || nd < 1 || nd > kMaxDims) return CTM_EINVAL;
  if (dt_in < 0 || dt_in > 2 || dt_out < 0 || dt_out > 2) return CTM_EINVAL;
  bool seen[kMaxDims] = {false};
  std::vector<int64_t> vd(dims, dims + nd), od;
  for (int i = 0; i < nd; ++i) {
    if (perm[i] < 0 || perm[i] >= nd || seen[perm[i]] || dims[i] < 0) return CTM_EINVAL;
    seen[perm[i]] = true;
    od.push_back(dims[perm[i]]);
  }
  Ctx c;
  c.stream = (hipStream_t)stream;
  Tensor ti = make_view(const_cast<void*>(in), dt_in, vd);
  Tensor to = make_view(out, dt_out, od);
  permute(c, ti, perm, to, scale);
  return c.hip_err == hipSuccess ? CTM_OK : CTM_EHIP;
}

}  // extern "C"

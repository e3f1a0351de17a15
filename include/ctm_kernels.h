/* ctm_kernels.h -- the hot kernels of the corner-transfer move, exposed one by
 * one so they can be tested and timed in isolation.  All pointers are device
 * pointers except where noted; all calls are asynchronous on `stream`
 * (hipStream_t, NULL = null stream) and return a ctm_status (ctm.h).
 *
 * Method: W. Lan and G. Evenbly, arXiv:2306.08212.
 */
#ifndef CTM_KERNELS_H
#define CTM_KERNELS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dense contraction step C = alpha * op(A) op(B) + beta * C, row-major: op(A)
 * is m x k (stored k x m with row stride lda when ta != 0, else m x k),
 * op(B) is k x n (stored n x k when tb != 0).  Every contraction of the move
 * -- the ket-then-bra absorption chain of Sec. IV / Fig. 4(b), the
 * enlarged-corner products of Sec. II and the Appendix -- reduces to this.
 * dtype: 0 = FP64, 1 = FP32, 2 = BF16 inputs with FP32 accumulation and FP32
 * C.  beta = 0 never reads C.  CTM_EINVAL for negative sizes or NULL. */
int ctm_kernel_gemm(int dtype, int m, int n, int k, double alpha, const void *A, int64_t lda,
                    int ta, const void *B, int64_t ldb, int tb, double beta, void *C,
                    int64_t ldc, void *stream);

/* Truncation of Sec. II / Sec. IV: top kk = min(k, m, n) left singular
 * vectors of the row-major FP64 m x n matrix M into U (m x kk, row-major) and
 * the singular values into S (kk); columns with sigma <= tau * sigma_0 are
 * zeroed; each kept column is sign-fixed (lowest row within 1e-8 relative of
 * the largest magnitude is positive).  M is not modified.  workspace is
 * caller-owned device memory of at least ctm_kernel_tsvd_workspace(m, n, k)
 * bytes.  CTM_ENOMEM if it is smaller.  Unlike the other calls this one
 * synchronises the stream at the end, to read the solver's error word:
 * CTM_ENUMERIC when a Jacobi solve inside did not converge within its sweep
 * cap (the outputs are then an orthonormal basis that is not the top-k
 * singular subspace). */
int ctm_kernel_tsvd(const double *M, int m, int n, int k, double tau, double *U, double *S,
                    void *workspace, size_t workspace_bytes, void *stream);
size_t ctm_kernel_tsvd_workspace(int m, int n, int k);

/* Allocation-free variant of ctm_kernel_tsvd, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and statuses as
 * ctm_kernel_tsvd, bitwise, but the workspace is a fixed device array inside
 * the library, one copy per GPU (its address is looked up on the first call
 * on each device), of ctm_kernel_tsvd_static_max() bytes (64 MiB: every
 * truncation of the move up to d=2, D=8, chi=256, e.g. 2048 x 2048 to 256,
 * fits).  Calls no hipMalloc or hipFree.  CTM_ENOMEM when
 * ctm_kernel_tsvd_workspace(m, n, k) exceeds that size.  Every call on one
 * GPU shares that GPU's array and overwrites it (the error word it needs is
 * cleared by each call): calls that overlap on one GPU -- on different
 * streams or from different host threads -- race and must not be issued.
 * Synchronises the stream at the end, as ctm_kernel_tsvd does. */
int ctm_kernel_tsvd_static(const double *M, int m, int n, int k, double tau, double *U, double *S,
                           void *stream);
size_t ctm_kernel_tsvd_static_max(void);

/* Index permute between contractions: out[i_0..] = scale * in[...] with out
 * dimension j equal to input dimension perm[j]; nd <= 8; dims are the input
 * dimensions (host array).  dt_in / dt_out as for ctm_kernel_gemm (2 = BF16)
 * -- the permute also converts the element type. */
int ctm_kernel_permute(int dt_in, const void *in, int nd, const int64_t *dims, const int *perm,
                       int dt_out, void *out, double scale, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTM_KERNELS_H */

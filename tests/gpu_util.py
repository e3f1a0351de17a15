"""Helpers for GPU tests: device buffers through torch, calls through the
C-ABI of libctm.so (kernel-level entry points of include/ctm_kernels.h)."""

import ctypes
import sys

import numpy as np


def torch():
    import torch as _t
    return _t


def lib():
    import paper_2306_08212_amd as P
    return P.load()


def dev(x, dtype=None):
    t = torch()
    a = np.ascontiguousarray(x)
    tt = t.from_numpy(a)
    if dtype is not None:
        tt = tt.to(dtype)
    return tt.to("cuda")


def stream_ptr():
    return torch().cuda.current_stream().cuda_stream


def gemm(dtype, A, B, ta=False, tb=False, alpha=1.0, beta=0.0, C=None):
    """A, B: torch cuda tensors (2-D, contiguous) of the kernel's input type."""
    t = torch()
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    out_dt = t.float64 if dtype == 0 else t.float32
    if C is None:
        C = t.empty((m, n), dtype=out_dt, device="cuda")
    st = lib().ctm_kernel_gemm(dtype, m, n, k, alpha, A.data_ptr(), A.shape[1], int(ta),
                               B.data_ptr(), B.shape[1], int(tb), beta, C.data_ptr(), n,
                               stream_ptr())
    assert st == 0, st
    t.cuda.synchronize()
    return C


def tsvd(M, k, tau=1e-14, expect=0):
    """M: numpy float64 (m x n); returns (U, S) numpy via the device kernel
    (the call's status must equal `expect`)."""
    t = torch()
    m, n = M.shape
    kk = min(k, m, n)
    dM = dev(M)
    U = t.empty((m, kk), dtype=t.float64, device="cuda")
    S = t.empty((kk,), dtype=t.float64, device="cuda")
    nb = lib().ctm_kernel_tsvd_workspace(m, n, k)
    ws = t.empty(nb, dtype=t.uint8, device="cuda")
    st = lib().ctm_kernel_tsvd(dM.data_ptr(), m, n, k, tau, U.data_ptr(), S.data_ptr(),
                               ws.data_ptr(), nb, stream_ptr())
    assert st == expect, st
    t.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy()


def permute(x, perm, dt_in, dt_out, scale=1.0):
    t = torch()
    dims = (ctypes.c_int64 * x.dim())(*x.shape)
    p = (ctypes.c_int * x.dim())(*perm)
    tmap = {0: t.float64, 1: t.float32, 2: t.bfloat16}
    out = t.empty([x.shape[i] for i in perm], dtype=tmap[dt_out], device="cuda")
    st = lib().ctm_kernel_permute(dt_in, x.data_ptr(), x.dim(), dims, p, dt_out,
                                  out.data_ptr(), scale, stream_ptr())
    assert st == 0, st
    t.cuda.synchronize()
    return out


def log(*a):
    """Print a test's measurement; with CTM_TEST_LOG naming a file, also
    append it there, so passing tests leave their numbers behind."""
    print(*a, flush=True)
    sys.stdout.flush()
    import os
    path = os.environ.get("CTM_TEST_LOG")
    if path and os.path.isdir(os.path.dirname(os.path.abspath(path))):
        with open(path, "a") as f:
            f.write(" ".join(str(x) for x in a) + "\n")

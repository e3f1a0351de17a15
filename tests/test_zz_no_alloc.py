"""The allocation-free truncation (ctm_kernel_tsvd_static) against the
workspace one (ctm_kernel_tsvd): same results, bitwise, on two calls in a
row, the second with a smaller input, through the C-ABI."""

import numpy as np
import pytest

from gpu_util import dev, lib, log, stream_ptr, torch, tsvd

pytestmark = pytest.mark.gpu


def _tsvd_static(M, k, tau=1e-14):
    t = torch()
    m, n = M.shape
    kk = min(k, m, n)
    dM = dev(M)
    U = t.empty((m, kk), dtype=t.float64, device="cuda")
    S = t.empty((kk,), dtype=t.float64, device="cuda")
    st = lib().ctm_kernel_tsvd_static(dM.data_ptr(), m, n, k, tau, U.data_ptr(), S.data_ptr(),
                                      stream_ptr())
    assert st == 0, st
    t.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy()


def _graded(m, n, rate, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    Q1, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    s = rate ** np.arange(min(m, n))
    return Q1 @ np.diag(s) @ Q2.T + 1e-3 * A / np.linalg.norm(A)


@pytest.mark.parametrize("first,second", [((2048, 2048, 256), (300, 200, 40)),
                                          ((864, 864, 144), (256, 64, 64))])
def test_static_scratch_matches_workspace_entry(first, second):
    for (m, n, k), seed in ((first, 1), (second, 2)):
        log("tsvd static", m, n, k)
        M = _graded(m, n, 0.97, seed)
        U0, S0 = tsvd(M, k)
        U1, S1 = _tsvd_static(M, k)
        assert np.array_equal(S0, S1)
        assert np.array_equal(U0, U1)


def test_static_scratch_rejects_oversized_problem():
    t = torch()
    cap = lib().ctm_kernel_tsvd_static_max()
    assert cap == 64 << 20
    m = n = 4096
    assert lib().ctm_kernel_tsvd_workspace(m, n, 1024) > cap
    dM = t.zeros((8,), dtype=t.float64, device="cuda")    # never read: size check first
    st = lib().ctm_kernel_tsvd_static(dM.data_ptr(), m, n, 1024, 1e-14, dM.data_ptr(),
                                      dM.data_ptr(), stream_ptr())
    assert st == 2    # CTM_ENOMEM

"""Kernel-level parity of the HIP library against plain references.

GEMM and permute are checked against float64 products on the CPU; the
truncated SVD against the oracle's LAPACK-based truncate (same cutoff and
sign rule)."""

import numpy as np
import pytest

import oracle as O
from gpu_util import dev, gemm, log, permute, torch, tsvd
from synth import random_orthogonal

pytestmark = pytest.mark.gpu


GEMM_SHAPES = [(1, 1, 1), (16, 16, 4), (77, 130, 45), (128, 128, 16), (200, 3, 513),
               (513, 257, 64), (64, 2048, 256), (1000, 64, 8)]


@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_fp64(m, n, k, ta, tb):
    log("gemm f64", m, n, k, ta, tb)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    ref = (A.T if ta else A) @ (B.T if tb else B)
    C = gemm(0, dev(A), dev(B), ta, tb).cpu().numpy()
    np.testing.assert_allclose(C, ref, rtol=0, atol=1e-12 * np.sqrt(k) * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_gemm_fp32_and_bf16(m, n, k, ta, tb):
    log("gemm f32/bf16", m, n, k, ta, tb)
    t = torch()
    rng = np.random.default_rng(m + n + k)
    A = rng.standard_normal((k, m) if ta else (m, k)).astype(np.float32)
    B = rng.standard_normal((n, k) if tb else (k, n)).astype(np.float32)
    ref = (A.T.astype(np.float64) if ta else A.astype(np.float64)) @ \
        (B.T.astype(np.float64) if tb else B.astype(np.float64))
    C = gemm(1, dev(A), dev(B), ta, tb).cpu().numpy()
    scale = np.sqrt(k) * max(1.0, np.abs(ref).max())
    np.testing.assert_allclose(C, ref, rtol=0, atol=2e-6 * scale)
    Ab = dev(A, t.bfloat16)
    Bb = dev(B, t.bfloat16)
    refb = (Ab.double().cpu().numpy().T if ta else Ab.double().cpu().numpy()) @ \
        (Bb.double().cpu().numpy().T if tb else Bb.double().cpu().numpy())
    Cb = gemm(2, Ab, Bb, ta, tb).cpu().numpy()
    np.testing.assert_allclose(Cb, refb, rtol=0, atol=2e-6 * scale)


def test_gemm_beta_accumulates():
    rng = np.random.default_rng(1)
    A, B, C0 = rng.standard_normal((33, 17)), rng.standard_normal((17, 65)), rng.standard_normal((33, 65))
    C = dev(C0)
    gemm(0, dev(A), dev(B), alpha=2.0, beta=-0.5, C=C)
    np.testing.assert_allclose(C.cpu().numpy(), 2.0 * A @ B - 0.5 * C0, atol=1e-12)


@pytest.mark.parametrize("shape,perm", [((3, 5, 7), (2, 0, 1)), ((64, 64), (1, 0)),
                                         ((2, 8, 8, 8, 8), (0, 2, 1, 4, 3)),
                                         ((33, 2, 40, 9), (3, 1, 0, 2)),
                                         ((4, 5, 6, 7, 8, 3), (5, 4, 3, 2, 1, 0)),
                                         ((100, 1, 37), (2, 1, 0)), ((1000,), (0,)),
                                         ((70, 3, 130), (2, 1, 0)),
                                         ((3, 96, 2, 130), (0, 3, 2, 1)),
                                         ((6, 5, 7, 3), (0, 2, 1, 3)),
                                         ((3, 70, 40, 33), (0, 2, 1, 3)),
                                         ((5, 40, 96, 2, 8), (0, 2, 3, 1, 4)),
                                         ((16, 70, 2, 8), (2, 1, 0, 3))])
def test_permute_and_cast(shape, perm):
    log("permute", shape, perm)
    t = torch()
    rng = np.random.default_rng(len(shape))
    x = rng.standard_normal(shape)
    ref = np.transpose(x, perm)
    y = permute(dev(x), perm, 0, 0).cpu().numpy()
    assert np.array_equal(y, ref)
    y32 = permute(dev(x), perm, 0, 1, scale=0.5).cpu().numpy()
    np.testing.assert_allclose(y32, 0.5 * ref.astype(np.float32), rtol=1e-7)
    yb = permute(dev(x.astype(np.float32)), perm, 1, 2).float().cpu().numpy()
    refb = t.from_numpy(ref.astype(np.float32)).to(t.bfloat16).float().numpy()
    assert np.array_equal(yb, refb)


@pytest.mark.parametrize("shape,perm", [((256, 8, 256, 8, 8), (0, 1, 3, 2, 4)),
                                        ((8, 256, 256, 2, 8, 8), (0, 2, 3, 4, 1, 5)),
                                        ((8, 2, 8, 256, 8, 256), (5, 4, 0, 1, 2, 3)),
                                        ((256, 8, 8, 2, 8, 256), (0, 4, 5, 3, 2, 1))])
def test_permute_move_shapes_f32(shape, perm):
    """Full-size permutes of the FP32 absorption chains at D=8, chi=256 (the
    D-leg payload tile and the composite tile), bitwise against a CPU
    transpose."""
    log("permute f32", shape, perm)
    t = torch()
    g = t.Generator().manual_seed(7)
    x = t.randn(shape, generator=g, dtype=t.float32)
    ref = x.permute(perm).contiguous()
    y = permute(x.to("cuda"), perm, 1, 1).cpu()
    assert t.equal(y, ref)


def _graded(m, n, decay, seed):
    k = min(m, n)
    U = random_orthogonal(m, seed)[:, :k]
    V = random_orthogonal(n, seed + 1)[:, :k]
    return U @ np.diag(decay ** np.arange(k)) @ V.T


def _zero_cols(m, n, rank, nzero, seed):
    """Rank-deficient with many exactly zero columns (the shape of the
    truncated matrices of the reduced move at the cut): exercises the
    dependent-column handling of the QR preconditioner."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((m, rank)) @ (rng.standard_normal((rank, n)) * np.exp(-0.2 * np.arange(rank))[:, None])
    M[:, rng.permutation(n)[:nzero]] = 0.0
    return M


SVD_CASES = [("square16", lambda: np.random.default_rng(0).standard_normal((16, 16)), 8),
             ("tall", lambda: np.random.default_rng(1).standard_normal((300, 40)), 12),
             ("wide", lambda: np.random.default_rng(2).standard_normal((40, 300)), 12),
             ("graded", lambda: _graded(96, 96, 0.8, 3), 64),
             ("rankdef", lambda: np.random.default_rng(4).standard_normal((64, 5))
              @ np.random.default_rng(5).standard_normal((5, 70)), 10),
             ("k>rank", lambda: np.random.default_rng(6).standard_normal((24, 24)), 64),
             ("tall256", lambda: _graded(512, 256, 0.97, 7), 256),
             ("zerocols", lambda: _zero_cols(256, 256, 60, 150, 8), 64),
             # rank 30 over 96 columns of 1024 rows: dependent columns in
             # every block of the QR, whose Gram-Schmidt fallback then spans
             # four chunks of rows and a second level
             ("tallrankdef", lambda: np.random.default_rng(9).standard_normal((1024, 30))
              @ np.random.default_rng(10).standard_normal((30, 96)), 40),
             # 4096 rows: four chunks at the tree's second level, whose last
             # workgroup to finish runs the third level and the products down
             ("tallrankdef4096", lambda: np.random.default_rng(11).standard_normal((4096, 30))
              @ np.random.default_rng(12).standard_normal((30, 96)), 40)]


@pytest.mark.parametrize("name,make,k", SVD_CASES)
def test_tsvd_matches_oracle_truncate(name, make, k):
    log("tsvd", name)
    M = make()
    U, S = tsvd(M, k)
    Uo, So = O.truncate(M, k)
    assert U.shape == Uo.shape
    np.testing.assert_allclose(S, So, rtol=0, atol=1e-12 * So[0])
    keep = So > 0
    assert np.array_equal(S > 0, keep)
    # vectors: compare where the singular value is separated from its neighbours
    s = np.concatenate([[np.inf], So, [0.0]])
    for c in np.nonzero(keep)[0]:
        gap = min(s[c] - s[c + 1], s[c + 1] - s[c + 2]) / So[0]
        if gap > 1e-6:
            np.testing.assert_allclose(U[:, c], Uo[:, c], rtol=0, atol=2e-12 / gap + 1e-11)
    # properties that hold regardless: orthonormal kept columns, Eckart-Young
    np.testing.assert_allclose(U[:, keep].T @ U[:, keep], np.eye(int(keep.sum())), atol=1e-12)
    R = M - U @ (U.T @ M)
    lam = np.sort(np.linalg.eigvalsh(M @ M.T))[::-1]
    assert abs(np.sum(R * R) - np.clip(lam[int(keep.sum()):], 0, None).sum()) < 1e-10 * lam[0]


def _move_spectrum(D, chi, col):
    """Singular values of a truncation input of the move (column 0: the side
    product L = C1 T1, column 1: the row M'), written by the oracle into
    tests/golden/spectra_D<D>_chi<chi>.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"spectra_D{D}_chi{chi}.txt")
    return np.loadtxt(path)[:, col]


@pytest.mark.parametrize("D,chi,col", [(6, 144, 0), (6, 144, 1), (8, 256, 0), (8, 256, 1)])
def test_tsvd_full_size_move_spectra(D, chi, col):
    """The large truncations of the move ((chi D) x (D chi) to chi: 864 x 864
    to 144 and 2048 x 2048 to 256) go through the randomised range finder.
    On matrices with the singular values of the move's own inputs (side
    product L and row M', from the oracle) and random singular vectors, the
    result is the exact truncation to rounding, compared with the oracle's
    LAPACK-based truncate: every kept singular value to 1e-13 sigma_0, every
    singular vector whose value is separated from its neighbours by more
    than 1e-6 sigma_0 element-wise, the kept projector applied to M to
    1e-11 ||M||, the Eckart-Young residual at its optimum to 1e-10
    (relative), and U orthonormal."""
    s = _move_spectrum(D, chi, col)
    n = s.size
    log("tsvd full size", D, chi, "L" if col == 0 else "M'", n)
    M = (random_orthogonal(n, 40 + col) * s) @ random_orthogonal(n, 50 + col).T
    U, S = tsvd(M, chi)
    Uo, So = O.truncate(M, chi)
    s0 = So[0]
    keep = So > 0
    # a value within rounding of the cutoff tau sigma_0 may be kept on one side only
    near_cut = np.abs(So - 1e-14 * s0) < 1e-15 * s0
    assert np.array_equal((S > 0)[~near_cut], keep[~near_cut])
    np.testing.assert_allclose(S, So, rtol=0, atol=1e-13 * s0)
    sp = np.concatenate([[np.inf], So, [0.0]])
    checked = 0
    for c in np.nonzero(keep)[0]:
        gap = min(sp[c] - sp[c + 1], sp[c + 1] - sp[c + 2]) / s0
        if gap > 1e-6:
            np.testing.assert_allclose(U[:, c], Uo[:, c], rtol=0, atol=2e-12 / gap + 1e-11)
            checked += 1
    assert checked >= 5
    kk = keep & (S > 0)
    Pd = U[:, kk] @ (U[:, kk].T @ M) - Uo[:, kk] @ (Uo[:, kk].T @ M)
    assert np.linalg.norm(Pd) <= 1e-11 * np.linalg.norm(M)
    R = M - U @ (U.T @ M)
    opt = np.sum(np.linalg.svd(M, compute_uv=False)[int(keep.sum()):] ** 2)
    assert np.sum(R * R) <= opt * (1.0 + 1e-10) + (1e-13 * s0) ** 2
    np.testing.assert_allclose(U[:, kk].T @ U[:, kk], np.eye(int(kk.sum())), atol=1e-12)


def test_tsvd_tall_compressed_matches_oracle():
    """m >= 4 n goes through the exact QR compression."""
    M = _graded(1024, 200, 0.95, 13)
    U, S = tsvd(M, 200)
    Uo, So = O.truncate(M, 200)
    np.testing.assert_allclose(S, So, rtol=0, atol=1e-12 * So[0])
    np.testing.assert_allclose(U.T @ U, np.eye(200), atol=1e-12)
    np.testing.assert_allclose(np.abs(U[:, :20]), np.abs(Uo[:, :20]), atol=1e-10)


def test_tsvd_reports_nonconvergence(monkeypatch):
    """A Jacobi solve still rotating after its last allowed sweep is reported
    as CTM_ENUMERIC (here with the sweep cap lowered to one through the
    CTM_DEBUG_MAX_SWEEPS knob; a 200 x 200 Gaussian matrix needs several);
    with the normal cap the same call succeeds and matches the oracle."""
    rng = np.random.default_rng(21)
    M = rng.standard_normal((200, 200))
    monkeypatch.setenv("CTM_DEBUG_MAX_SWEEPS", "1")
    tsvd(M, 50, expect=4)
    monkeypatch.delenv("CTM_DEBUG_MAX_SWEEPS")
    U, S = tsvd(M, 50)
    So = np.linalg.svd(M, compute_uv=False)[:50]
    np.testing.assert_allclose(S, So, rtol=0, atol=1e-12 * So[0])


@pytest.mark.parametrize("name", ["graded", "tall256", "zerocols", "tallrankdef"])
def test_tsvd_late_sweeps_in_one_launch(name, monkeypatch):
    """The Jacobi sweeps after the first eight run in one launch of one
    workgroup, block pair after block pair.  With the split moved to after
    the first sweep (CTM_DEBUG_PAR_SWEEPS=1) every later sweep runs there;
    the pairs of a round touch disjoint columns, so the result is bitwise the
    one of the launch-per-round sweeps, and it still matches the oracle."""
    make, k = {n: (mk, kk) for n, mk, kk in SVD_CASES}[name]
    M = make()
    log("tsvd late sweeps", name)
    U0, S0 = tsvd(M, k)
    monkeypatch.setenv("CTM_DEBUG_PAR_SWEEPS", "1")
    U1, S1 = tsvd(M, k)
    monkeypatch.delenv("CTM_DEBUG_PAR_SWEEPS")
    assert np.array_equal(S0, S1)
    assert np.array_equal(U0, U1)
    So = O.truncate(M, k)[1]
    np.testing.assert_allclose(S1, So, rtol=0, atol=1e-12 * So[0])

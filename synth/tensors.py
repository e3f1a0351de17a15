"""Seeded generators for site tensors and request streams.

Site tensors follow the layout of the two-site unit cell of Sec. II: A and B
are real arrays indexed ``[s, l, u, r, d]`` (physical index first, then the
left, up, right and down virtual legs), shape ``(d, D, D, D, D)``.

The recipe stands in for the imaginary-time-optimised Heisenberg states of
Sec. V, which are not available: a Neel product state on virtual index 0
(A carries spin up, B spin down, the antiferromagnetic order of the
Heisenberg ground state) plus Gaussian noise whose amplitude decays along
every virtual leg as exp(-k) for bond index k, mimicking the decaying bond
spectrum of a gauge-fixed iPEPS.  Noise amplitude is 1, exactly as the
recipe states.
"""

from __future__ import annotations

import numpy as np


def _bond_weights(D: int) -> np.ndarray:
    return np.exp(-np.arange(D, dtype=np.float64))


def site_tensors(d: int, D: int, seed: int):
    """Return (A, B), float64 arrays of shape (d, D, D, D, D).

    ``numpy.random.default_rng(seed)`` draws the noise of A first, then
    that of B, each with ``standard_normal((d, D, D, D, D))``.
    """
    if d < 2 or D < 1:
        raise ValueError("need d >= 2 and D >= 1")
    rng = np.random.default_rng(seed)
    lam = _bond_weights(D)
    w = (lam[:, None, None, None] * lam[None, :, None, None]
         * lam[None, None, :, None] * lam[None, None, None, :])
    A = rng.standard_normal((d, D, D, D, D)) * w[None]
    B = rng.standard_normal((d, D, D, D, D)) * w[None]
    A[0, 0, 0, 0, 0] += 1.0
    B[1, 0, 0, 0, 0] += 1.0
    return A, B


def product_state_tensors(d: int, seed: int):
    """D = 1 tensors of two random real product states: (A, B, psi_a, psi_b).

    A[s,0,0,0,0] = psi_a[s] with psi_a a standard-normal vector (not
    normalised), likewise B.
    """
    rng = np.random.default_rng(seed)
    pa = rng.standard_normal(d)
    pb = rng.standard_normal(d)
    return pa.reshape(d, 1, 1, 1, 1).copy(), pb.reshape(d, 1, 1, 1, 1).copy(), pa, pb


def random_orthogonal(n: int, seed: int) -> np.ndarray:
    """A Haar-like real orthogonal n x n matrix (QR of a Gaussian matrix)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


def random_rotation2(seed: int) -> np.ndarray:
    """A real 2 x 2 rotation by a uniformly drawn angle."""
    th = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi)
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s], [s, c]])


def serving_stream(n: int, seed: int, rate: float, d: int = 2,
                   D_min: int = 3, D_max: int = 8, chi_cap: int = 256):
    """A stream of n independent environment-solve requests.

    Request i has D uniform in {D_min..D_max}, chi uniform in
    [D^2, min(4 D^2, chi_cap)], site-tensor seed i and an arrival time from
    seeded exponential gaps of mean 1/rate (rate <= 0: all arrive at t = 0).
    Returns a list of dicts with keys id, d, D, chi, seed, t_arrival.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n):
        D = int(rng.integers(D_min, D_max + 1))
        lo = D * D
        hi = max(lo, min(4 * D * D, chi_cap))
        chi = int(rng.integers(lo, hi + 1))
        if rate > 0:
            t += float(rng.exponential(1.0 / rate))
        out.append({"id": i, "d": d, "D": D, "chi": chi, "seed": i,
                    "t_arrival": t if rate > 0 else 0.0})
    return out

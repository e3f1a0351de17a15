"""Observables of a converged environment on the GPU against the oracle:
one-site expectation values (staggered magnetisation, order parameter,
transverse-field term) and the connected correlation along a row (Sec. V),
FP64, through the C-ABI (ctm_expect1, ctm_row_correlation)."""

import numpy as np
import pytest

import oracle as O
import paper_2306_08212_amd as P
from gpu_util import log
from synth import site_tensors

pytestmark = pytest.mark.gpu

SX = np.array([[0.0, 0.5], [0.5, 0.0]])
SZ = np.array([[0.5, 0.0], [0.0, -0.5]])


def _pair(D, chi, seed, method, iters):
    A, B = site_tensors(2, D, seed)
    om = {P.STANDARD: O.STANDARD, P.REDUCED: O.REDUCED, P.REDUCED_ENV: O.REDUCED_ENV}[method]
    env = O.solve(A, B, chi, om, max_iters=iters)["env"]
    s = P.Solver(P.Config(d=2, D=D, chi=chi, method=method, precision=P.FP64), A, B)
    s.iterate(iters)
    return A, B, env, s


@pytest.mark.parametrize("method", [P.REDUCED, P.STANDARD])
def test_one_site_expectations_match_oracle(method):
    """d=2, D=2, chi=8, 20 iterations: <S^z>, <S^x> on both sublattices and
    the staggered magnetisation to 1e-10 (relative to the largest)."""
    A, B, env, s = _pair(2, 8, 0, method, 20)
    for op in (SZ, SX):
        g = s.expect1(op)
        o = O.expect1(env, A, B, op)
        log("expect1", method, g, o)
        scale = max(abs(o[0]), abs(o[1]), 1e-3)
        np.testing.assert_allclose(g, o, rtol=0, atol=1e-10 * scale)
    ms, mo = s.staggered_magnetisation(), O.staggered_magnetisation(env, A, B)
    log("m_s", ms, mo)
    assert abs(ms - mo) <= 1e-10 * mo
    s.close()


@pytest.mark.parametrize("method", [P.REDUCED, P.STANDARD])
def test_row_correlation_matches_oracle(method):
    """S_zz(x) for x = 1..6 at d=2, D=2, chi=8 after 20 iterations, to 1e-10
    of |C(1)|; C(1) also equals <S^z S^z> - <S^z>_a <S^z>_b with all three
    taken from the (separately coded) bond energy network."""
    A, B, env, s = _pair(2, 8, 1, method, 20)
    g = s.row_correlation(SZ, 6)
    o = O.row_correlation(env, A, B, SZ, 6)
    log("S_zz", method, g, o)
    np.testing.assert_allclose(g, o, rtol=0, atol=1e-10 * abs(o[0]))
    one = np.eye(2)
    _, eb = s.energy(np.kron(SZ, SZ))
    _, ea = s.energy(np.kron(SZ, one))
    _, ebb = s.energy(np.kron(one, SZ))
    assert abs(g[0] - (eb[0] - ea[0] * ebb[0])) <= 1e-10 * abs(o[0])
    s.close()


def test_observables_at_config2_size():
    """d=2, D=4, chi=64, standard move, 4 iterations: <S^z> on both
    sublattices and S_zz(x), x = 1..4, against the oracle's stored values
    (tests/golden/config_D4_chi64_oracle.json) within ten times the
    oracle's own spread between its gesdd and gesvd runs (never below
    1e-10 of the largest value): the truncations keep directions that any
    SVD fixes only to eps / gap."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "config_D4_chi64_oracle.json")
    g = json.load(open(path))["results"]
    ref = np.array(g["gesdd"]["standard"]["sz"] + g["gesdd"]["standard"]["szz"])
    alt = np.array(g["gesvd"]["standard"]["sz"] + g["gesvd"]["standard"]["szz"])
    scale = np.abs(ref).max()
    spread = np.abs(ref - alt).max() / scale
    bar = max(1e-10, 10.0 * spread)
    A, B = site_tensors(2, 4, 0)
    s = P.Solver(P.Config(d=2, D=4, chi=64, method=P.STANDARD, precision=P.FP64), A, B)
    s.iterate(g["gesdd"]["standard"]["iterations"])
    got = np.array(s.expect1(SZ) + s.row_correlation(SZ, 4))
    err = np.abs(got - ref).max() / scale
    log(f"observables D=4: gpu {got} oracle {ref} err {err:.2e} spread {spread:.2e}")
    assert err <= bar
    s.close()

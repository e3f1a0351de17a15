"""FP64 parity of the HIP corner-transfer path with the oracle, through the
C-ABI (ctm_init / ctm_move / ctm_iterate / ctm_energy / ctm_get_env).

Tolerances: energies 1e-10 relative (the FP64 bar).  Environment tensors
element by element (up to the sign of each boundary-bond basis vector, which
the truncation's sign rule cannot fix for ill-determined vectors), and the
corner spectra, are held to the oracle's own conditioning: directions kept
near the cut have
tiny singular values and gaps, so they are fixed by any backward-stable SVD
only to about eps / gap, and the reduced move amplifies such differences
from move to move.  The bar is 100 times what eps-level noise added to the
oracle's truncated matrices does to its own environment after the same
moves (measured in the test; 2.6e-10 to 2.8e-7 at D = 2, chi = 8 over 20
iterations), and never below 1e-8 (1e-10 of sigma_0 for the spectra).
"""

import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2306_08212_amd as P
from gpu_util import log
from synth import site_tensors

pytestmark = pytest.mark.gpu


OMETHOD = {P.STANDARD: O.STANDARD, P.REDUCED: O.REDUCED, P.REDUCED_ENV: O.REDUCED_ENV}


def _solver(A, B, D, chi, method, prec=P.FP64, boot=0):
    cfg = P.Config(d=A.shape[0], D=D, chi=chi, method=method, precision=prec, boot_iters=boot)
    return P.Solver(cfg, A, B)


def _align_bond_signs(g, o):
    """g with a sign per value of each boundary (chi) bond, axes 0 and -1,
    chosen to match o.  The truncation fixes each kept singular vector's sign
    by its largest entry; for an ill-determined vector (tiny singular value
    next to a near-degenerate partner) that choice can go either way within
    rounding, which flips one slice of every tensor on that bond and leaves
    every physical quantity unchanged."""
    g = g.copy()
    for _ in range(3):
        for ax in (0, g.ndim - 1):
            gm = np.moveaxis(g, ax, 0).reshape(g.shape[ax], -1)
            om = np.moveaxis(o, ax, 0).reshape(o.shape[ax], -1)
            sg = np.where(np.sum(gm * om, axis=1) < 0, -1.0, 1.0)
            shape = [1] * g.ndim
            shape[ax] = -1
            g = g * sg.reshape(shape)
    return g


def _compare_env(sol, env, tol):
    for name in O.ENV_KEYS:
        g = sol.get_env(P.env_index(name))
        o = env[name]
        assert g.shape == o.shape, (name, g.shape, o.shape)
        err = np.abs(_align_bond_signs(g, o) - o).max() / np.abs(o).max()
        assert err < tol, (name, err)


def _spectra(env):
    return {k: np.linalg.svd(env[k], compute_uv=False) for k in O.ENV_KEYS if k[0] == "C"}


def _spectra_err(a, b):
    """Largest change of a corner singular value, relative to sigma_0."""
    return max(np.abs(a[k] - b[k]).max() / b[k][0] for k in b)


def _compare_spectra(sol, env, tol):
    """Singular values of every corner (gauge-invariant) to tol * sigma_0."""
    g = _spectra({k: sol.get_env(P.env_index(k)) for k in O.ENV_KEYS if k[0] == "C"})
    err = _spectra_err(g, _spectra(env))
    assert err < tol, err


def _oracle_env_sensitivity(run, trials=2):
    """Largest element-wise change (relative to each tensor's largest entry)
    of the oracle's environment, and largest change of a corner singular
    value (relative to sigma_0), when every matrix it truncates gets Gaussian
    noise of Frobenius norm eps ||M||_F (a backward error of one ulp)."""
    ref = run()
    ref_spec = _spectra(ref)
    orig = O.ctm.truncate
    worst = 0.0
    worst_spec = 0.0
    for t in range(trials):
        rng = np.random.default_rng(1000 + t)

        def noisy(M, k, tau=None):
            Mp = M + rng.standard_normal(M.shape) * (2.2e-16 * np.linalg.norm(M) / np.sqrt(M.size))
            return orig(Mp, k) if tau is None else orig(Mp, k, tau)

        O.ctm.truncate = noisy
        try:
            env = run()
        finally:
            O.ctm.truncate = orig
        worst = max(worst, max(np.abs(env[k] - ref[k]).max() / np.abs(ref[k]).max()
                               for k in O.ENV_KEYS))
        worst_spec = max(worst_spec, _spectra_err(_spectra(env), ref_spec))
    return ref, worst, worst_spec


def test_neel_d1():
    log("neel")
    A = np.zeros((2, 1, 1, 1, 1)); A[0] = 1.0
    B = np.zeros((2, 1, 1, 1, 1)); B[1] = 1.0
    for method in (P.STANDARD, P.REDUCED):
        s = _solver(A, B, 1, 4, method)
        s.iterate(3)
        e, eb = s.energy()
        assert abs(e + 0.5) < 1e-14
        s.close()


def test_init_env_and_energy_match_oracle():
    log("init")
    A, B = site_tensors(2, 2, 0)
    s = _solver(A, B, 2, 8, P.REDUCED)
    env = O.init_env(A, B)
    _compare_env(s, env, 1e-13)
    e, eb = s.energy()
    eo, ebo = O.energy(env, A, B)
    np.testing.assert_allclose(eb, ebo, rtol=1e-12)
    s.close()


@pytest.mark.parametrize("method", [P.STANDARD, P.REDUCED, P.REDUCED_ENV])
def test_single_moves_match_oracle(method):
    """Each direction once from the initial environment (frames, rotation
    relabel and every anchor kind)."""
    A, B = site_tensors(2, 2, 1)
    om = OMETHOD[method]
    for r in range(4):
        log("move", method, r)
        s = _solver(A, B, 2, 8, method)
        s.move(r)
        env, sens, ssens = _oracle_env_sensitivity(
            lambda: O.move(O.init_env(A, B), A, B, r, 8, om))
        log(f"  oracle sensitivity: env {sens:.1e} spectra {ssens:.1e}")
        _compare_env(s, env, max(1e-8, 100 * sens))
        _compare_spectra(s, env, max(1e-10, 100 * ssens))
        e, eb = s.energy()
        np.testing.assert_allclose(eb, O.energy(env, A, B)[1], rtol=1e-10)
        s.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("method", [P.REDUCED, P.STANDARD, P.REDUCED_ENV])
def test_config1_twenty_iterations(seed, method):
    """d=2, D=2, chi=8, 20 iterations (the small configuration): energies to
    1e-10 relative, corner spectra to 1e-10, environment tensors to the
    oracle's own conditioning (module docstring).  The reduced-env move does
    not converge for seeds 0 and 2 at this size (its corner spectra keep
    moving by ~3e-3 per iteration, in the oracle alone) and amplifies
    rounding differences from iteration to iteration, so those two are
    compared after 4 iterations."""
    iters = 4 if (method == P.REDUCED_ENV and seed != 1) else 20
    log("config1", seed, method, iters)
    A, B = site_tensors(2, 2, seed)
    om = OMETHOD[method]
    r = O.solve(A, B, 8, om, max_iters=iters)
    _, sens, ssens = _oracle_env_sensitivity(lambda: O.solve(A, B, 8, om, max_iters=iters)["env"])
    s = _solver(A, B, 2, 8, method)
    s.iterate(iters)
    e, eb = s.energy()
    np.testing.assert_allclose(eb, r["e_bond"], rtol=1e-10)
    assert abs(e - r["e_site"]) < 1e-10 * abs(r["e_site"])
    log(f"  oracle sensitivity: env {sens:.1e} spectra {ssens:.1e}")
    _compare_env(s, r["env"], max(1e-8, 100 * sens))
    _compare_spectra(s, r["env"], max(1e-10, 100 * ssens))
    s.close()


def test_converge_reports_delta():
    A, B = site_tensors(2, 2, 0)
    s = _solver(A, B, 2, 8, P.REDUCED)
    it, delta, ok = s.converge(40, 1e-10)
    r = O.solve(A, B, 8, O.REDUCED, max_iters=40, tol=1e-10)
    assert ok == (r["delta"] < 1e-10)
    assert it == r["iters"]
    s.close()


# At d=2, D=4, chi=64 the synthetic state's anchor spectra have decayed to
# ~1e-10 sigma_0 at the cut, with neighbouring gaps ~1e-12 sigma_0.  The kept
# directions there are fixed by any SVD only to an angle of about
# (backward error) / gap, and the one-sided projector keeps them at full weight
# in the absorbed tensors, and the reduced moves amplify differences from
# move to move.  The bar is therefore derived from the oracle itself: the
# larger of ten times the difference between its runs with the gesdd and
# gesvd drivers and a hundred times the change one ulp of noise on every
# truncated matrix causes (a backward-error budget of 100 ulps, as for the
# environment tensors above), never below 1e-10; all three runs are stored
# by tests/golden/make_config2.py.  With a
# cutoff that zeroes the ill-determined directions every kept direction is
# well defined and the plain FP64 bar applies
# (test_config2_well_determined_cutoff).
CONFIG2 = os.path.join(os.path.dirname(__file__), "golden", "config_D4_chi64_oracle.json")


def _config2(name):
    """The stored gesdd result and the bar: the larger of ten times the
    gesdd/gesvd spread and a hundred times the spread under one ulp of
    noise on every truncated matrix, never below 1e-10."""
    g = json.load(open(CONFIG2))["results"]
    a = g["gesdd"][name]

    def spread(b):
        return max(abs(x - y) for x, y in zip([a["e_site"]] + a["e_bond"],
                                              [b["e_site"]] + b["e_bond"])) / abs(a["e_site"])
    sd, sn = spread(g["gesvd"][name]), spread(g["noise"][name])
    return a, sd, sn, max(1e-10, 10.0 * sd, 100.0 * sn)


@pytest.mark.parametrize("method,name", [(P.STANDARD, "standard"), (P.REDUCED, "reduced"),
                                         (P.REDUCED_ENV, "reduced_env")])
def test_config2_energy(method, name):
    """d=2, D=4, chi=64: energies after the stored number of iterations (4
    standard, 2 of each reduced method) to the plain FP64 bar, 1e-10
    relative.  The oracle's own spreads (_config2: gesdd vs gesvd, and one
    ulp of noise on every truncated matrix) are logged beside it; they are
    below 2e-12 here, so the result is determined well inside the bar."""
    r, spread, nspread, _ = _config2(name)
    bar = 1e-10
    iters = r["iterations"]
    log("config2", name, iters)
    A, B = site_tensors(2, 4, 0)
    s = _solver(A, B, 4, 64, method)
    s.iterate(iters)
    e, eb = s.energy()
    err = max(abs(x - y) for x, y in zip([e] + eb, [r["e_site"]] + r["e_bond"])) / abs(r["e_site"])
    log(f"config2 {name}: rel err {err:.2e}, oracle driver spread {spread:.2e}, one-ulp spread "
        f"{nspread:.2e}, bar {bar:.2e}")
    assert err <= bar
    s.close()


@pytest.mark.parametrize("method", [P.STANDARD, P.REDUCED, P.REDUCED_ENV])
def test_config2_well_determined_cutoff(method):
    """Same size with cutoff tau = 1e-7: directions below 1e-7 sigma_0 are
    zeroed on both sides, every kept direction is well determined, and the
    FP64 bar (1e-10 relative) holds after 2 iterations."""
    log("config2 tau", method)
    A, B = site_tensors(2, 4, 0)
    om = OMETHOD[method]
    import oracle.ctm as OC
    saved = OC.TAU
    OC.TAU = 1e-7
    try:
        r = O.solve(A, B, 64, om, max_iters=2)
    finally:
        OC.TAU = saved
    cfg = P.Config(d=2, D=4, chi=64, method=method, precision=P.FP64, svd_cutoff=1e-7)
    s = P.Solver(cfg, A, B)
    s.iterate(2)
    e, eb = s.energy()
    log("config2 tau rel err", np.max(np.abs(np.array(eb) - r["e_bond"]) / np.abs(r["e_bond"])))
    np.testing.assert_allclose(eb, r["e_bond"], rtol=1e-10)
    s.close()



@pytest.mark.parametrize("D,chi,chi_p,chi_pp,iters", [(2, 8, 12, 16, 6), (3, 9, 18, 12, 3)])
def test_independent_chi_p_chi_pp(D, chi, chi_p, chi_pp, iters):
    """chi' (anchor first stage) and chi'' (helper first stage) set apart
    from chi: energies to 1e-10 relative and corner spectra to the oracle's
    conditioning after a few iterations."""
    log("chi_p", D, chi, chi_p, chi_pp)
    A, B = site_tensors(2, D, 2)
    r = O.solve(A, B, chi, O.REDUCED, max_iters=iters, chi_p=chi_p, chi_pp=chi_pp)
    _, _, ssens = _oracle_env_sensitivity(
        lambda: O.solve(A, B, chi, O.REDUCED, max_iters=iters, chi_p=chi_p, chi_pp=chi_pp)["env"])
    cfg = P.Config(d=2, D=D, chi=chi, method=P.REDUCED, precision=P.FP64, chi_p=chi_p,
                   chi_pp=chi_pp)
    s = P.Solver(cfg, A, B)
    s.iterate(iters)
    e, eb = s.energy()
    log(f"  gpu {e!r} oracle {r['e_site']!r}")
    np.testing.assert_allclose(eb, r["e_bond"], rtol=1e-10)
    _compare_spectra(s, r["env"], max(1e-10, 100 * ssens))
    s.close()

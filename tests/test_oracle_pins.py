"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, a brute-force
contraction, a library routine used in a different way, or an invariant of
the mathematics, chosen so that a dropped term, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""

import os

import numpy as np
import pytest
from scipy.special import ellipk

import oracle as O
import oracle.ctm as OC
from bruteforce import patch_bond_energy
from synth import product_state_tensors, random_orthogonal, random_rotation2, site_tensors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("method", [O.STANDARD, O.REDUCED, O.REDUCED_ENV])
@pytest.mark.parametrize("chi", [1, 4])
def test_neel_product_state_energy(method, chi):
    """D = 1 Neel state: <S.S> = -1/4 on every bond, -1/2 per site."""
    A = np.zeros((2, 1, 1, 1, 1)); A[0] = 1.0
    B = np.zeros((2, 1, 1, 1, 1)); B[1] = 1.0
    r = O.solve(A, B, chi, method, max_iters=3)
    assert abs(r["e_site"] + 0.5) < 1e-14
    for e in r["e_bond"]:
        assert abs(e + 0.25) < 1e-14


def _spin_expectation(psi):
    sx = np.array([[0.0, 1.0], [1.0, 0.0]]) / 2
    sz = np.array([[1.0, 0.0], [0.0, -1.0]]) / 2
    n = psi @ psi
    return np.array([psi @ sx @ psi / n, 0.0, psi @ sz @ psi / n])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_product_state_energy(seed):
    """D = 1 product states: <S_i.S_j> = <S>_i . <S>_j (S^y vanishes for
    real states)."""
    A, B, pa, pb = product_state_tensors(2, seed)
    exact = _spin_expectation(pa) @ _spin_expectation(pb)
    for method in (O.STANDARD, O.REDUCED, O.REDUCED_ENV):
        r = O.solve(A, B, 3, method, max_iters=2)
        for e in r["e_bond"]:
            assert abs(e - exact) < 1e-13
        assert abs(r["e_site"] - 2 * exact) < 1e-13


# ------------------------------------------------------------ operators

def _spin_ops():
    """Spin-1/2 operators S = sigma / 2 as complex matrices, written from
    the Pauli matrices (not from the oracle's real form of S.S)."""
    sx = np.array([[0, 1], [1, 0]], dtype=complex) / 2
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex) / 2
    sz = np.array([[1, 0], [0, -1]], dtype=complex) / 2
    return sx, sy, sz


def test_heisenberg_h2_spectrum():
    """S.S on two spins 1/2: singlet -3/4, triplet +1/4 (three times), from
    S_tot^2 = s(s+1) with S_1.S_2 = (S_tot^2 - 3/2) / 2.  A wrong sign on
    any of the three terms moves an eigenvalue (e.g. -S^yS^y gives
    {-1/4, -1/4, -1/4, 3/4})."""
    h = O.heisenberg_h2()
    assert h.shape == (4, 4)
    np.testing.assert_allclose(h, h.T, atol=0)
    np.testing.assert_allclose(np.linalg.eigvalsh(h), [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


def test_heisenberg_h2_singlet_and_triplet_states():
    """<h> on the two-site singlet (|ud> - |du>)/sqrt2 is -3/4, on the
    triplet states |uu>, (|ud> + |du>)/sqrt2 and |dd> it is +1/4 (basis
    order (s1 s2) with s = 0 up, 1 down)."""
    h = O.heisenberg_h2()
    r2 = np.sqrt(0.5)
    singlet = np.array([0.0, r2, -r2, 0.0])
    t0 = np.array([0.0, r2, r2, 0.0])
    assert abs(singlet @ h @ singlet + 0.75) < 1e-15
    assert abs(t0 @ h @ t0 - 0.25) < 1e-15
    for i in (0, 3):
        e = np.zeros(4); e[i] = 1.0
        assert abs(e @ h @ e - 0.25) < 1e-15


def test_heisenberg_h2_equals_spin_dot_product_and_is_su2_invariant():
    """h equals S_1.S_2 built from the complex Pauli matrices, and commutes
    with every component of the total spin (SU(2) invariance)."""
    sx, sy, sz = _spin_ops()
    ref = sum(np.kron(a, a) for a in (sx, sy, sz))
    assert np.abs(ref.imag).max() == 0.0
    h = O.heisenberg_h2()
    np.testing.assert_allclose(h, ref.real, atol=1e-16)
    one = np.eye(2)
    for a in (sx, sy, sz):
        tot = np.kron(a, one) + np.kron(one, a)
        assert np.abs(h @ tot - tot @ h).max() < 1e-15


# ------------------------------------------------------------ convergence measure

def _env_with_corner_spectra(chi, spectra, seed=0):
    """An environment whose 8 corners have the given singular values (in a
    random orthogonal basis on each side); edges are unused."""
    env = {}
    for i, key in enumerate(OC.CORNERS):
        s = np.asarray(spectra[i], dtype=float)
        n = s.size
        U = random_orthogonal(n, seed + 2 * i)
        V = random_orthogonal(n, seed + 2 * i + 1)
        env[key] = U @ np.diag(s) @ V.T
    return env


def test_corner_spectra_known_values():
    """Normalised by the largest singular value and zero padded to chi:
    singular values (3, 2, 1) at chi = 5 give (1, 2/3, 1/3, 0, 0)."""
    spectra = [[3.0, 2.0, 1.0]] * 8
    sp = O.corner_spectra(_env_with_corner_spectra(5, spectra), 5)
    for key in OC.CORNERS:
        np.testing.assert_allclose(sp[key], [1.0, 2.0 / 3.0, 1.0 / 3.0, 0.0, 0.0], atol=1e-15)


def test_corner_spectra_scale_invariant_and_truncated_to_chi():
    """Each corner's spectrum is divided by its own sigma_0 (scaling one
    corner changes nothing) and cut to chi entries when the corner is
    larger."""
    spectra = [[4.0, 1.0, 0.5, 0.25]] * 4 + [[8.0, 2.0, 1.0, 0.5]] * 4
    env = _env_with_corner_spectra(3, spectra, seed=5)
    sp = O.corner_spectra(env, 3)
    for key in OC.CORNERS:
        np.testing.assert_allclose(sp[key], [1.0, 0.25, 0.125], atol=1e-15)
    env2 = dict(env)
    env2["C3b"] = 17.0 * env["C3b"]
    sp2 = O.corner_spectra(env2, 3)
    np.testing.assert_allclose(sp2["C3b"], sp["C3b"], atol=1e-15)


def test_solve_delta_is_max_change_of_normalised_spectra():
    """solve's delta after an iteration is the largest change of a
    normalised corner singular value, and solve stops at the first
    iteration whose delta is below tol.  The Onsager Ising state converges
    (a fixed point), so delta falls below 1e-11 and stays there."""
    A = _ising_peps(0.3)
    zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    r = O.solve(A, A, 12, O.STANDARD, max_iters=40, tol=1e-11, h2=zz)
    assert r["delta"] < 1e-11 and r["iters"] < 40
    assert all(d >= 1e-11 for d in r["deltas"][:-1])
    # one more iteration from the fixed point: delta recomputed by hand
    env0 = r["env"]
    env1 = O.ctm_iteration(env0, A, A, 12, O.STANDARD)
    dl = 0.0
    for key in OC.CORNERS:
        s0 = np.linalg.svd(env0[key], compute_uv=False)
        s1 = np.linalg.svd(env1[key], compute_uv=False)
        v0 = np.zeros(12); v0[:min(12, s0.size)] = (s0 / s0[0])[:12]
        v1 = np.zeros(12); v1[:min(12, s1.size)] = (s1 / s1[0])[:12]
        dl = max(dl, np.abs(v1 - v0).max())
    assert dl < 1e-11


# ------------------------------------------------------------ brute force

def _bf_all(A, B, h2, nL, nR, nU, nD):
    ext = dict(left=1 + 2 * nL, right=1 + 2 * nR, up=1 + 2 * nU, down=1 + 2 * nD)
    return [patch_bond_energy(A, B, h2, True, "h", **ext),
            patch_bond_energy(A, B, h2, False, "h", **ext),
            patch_bond_energy(A, B, h2, True, "v", **ext),
            patch_bond_energy(A, B, h2, False, "v", **ext)]


def _ctm_all(env, A, B, h2):
    return [O.bond_energy(env, A, B, "a", h2, 0), O.bond_energy(env, A, B, "b", h2, 0),
            O.bond_energy(env, A, B, "a", h2, 1), O.bond_energy(env, A, B, "b", h2, 1)]


@pytest.mark.parametrize("method", [O.STANDARD, O.REDUCED, O.REDUCED_ENV])
def test_untruncated_ctm_equals_bruteforce_patch(method):
    """With identity isometries every move is an exact contraction: after
    moves L / L,R,U,D the environment is the traced boundary of a finite
    patch grown by two sites per move, contracted here column by column with
    no environment tensors at all (init, rotation, absorption topology and
    the energy networks are all pinned)."""
    h2 = O.heisenberg_h2()
    A, B = site_tensors(2, 2, 3)
    env = O.init_env(A, B)
    np.testing.assert_allclose(_ctm_all(env, A, B, h2), _bf_all(A, B, h2, 0, 0, 0, 0),
                               rtol=0, atol=1e-12)
    e1 = O.move(env, A, B, 0, 8, method, untruncated=True)
    np.testing.assert_allclose(_ctm_all(e1, A, B, h2), _bf_all(A, B, h2, 1, 0, 0, 0),
                               rtol=0, atol=1e-12)
    e2 = O.move(env, A, B, 1, 8, method, untruncated=True)
    np.testing.assert_allclose(_ctm_all(e2, A, B, h2), _bf_all(A, B, h2, 0, 0, 1, 0),
                               rtol=0, atol=1e-12)
    e4 = O.ctm_iteration(env, A, B, 8, method, untruncated=True)
    np.testing.assert_allclose(_ctm_all(e4, A, B, h2), _bf_all(A, B, h2, 1, 1, 1, 1),
                               rtol=0, atol=1e-12)


def test_untruncated_bruteforce_D3():
    h2 = O.heisenberg_h2()
    A, B = site_tensors(2, 3, 4)
    env = O.init_env(A, B)
    np.testing.assert_allclose(_ctm_all(env, A, B, h2), _bf_all(A, B, h2, 0, 0, 0, 0),
                               rtol=0, atol=1e-12)
    for method in (O.STANDARD, O.REDUCED):
        e1 = O.move(env, A, B, 2, 9, method, untruncated=True)
        np.testing.assert_allclose(_ctm_all(e1, A, B, h2), _bf_all(A, B, h2, 0, 1, 0, 0),
                                   rtol=0, atol=1e-12)


# ------------------------------------------------------------ Onsager

def _onsager_nn(beta):
    k = 2 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    return 0.5 / np.tanh(2 * beta) * (1 + (2 / np.pi) * (2 * np.tanh(2 * beta) ** 2 - 1)
                                      * ellipk(k * k))


_ISING_CACHE = {}


def _ising_solve(beta, method, boot):
    """Converged CTMRG of the classical Ising PEPS at beta (chi = 24, delta
    < 1e-11), with the nearest-neighbour sigma^z sigma^z as bond operator;
    cached, since several pins use the same solve."""
    key = (beta, method, boot)
    if key not in _ISING_CACHE:
        A = _ising_peps(beta)
        zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
        _ISING_CACHE[key] = O.solve(A, A, 24, method, max_iters=60, tol=1e-11, h2=zz,
                                    boot_iters=boot)
    return _ISING_CACHE[key]


def _ising_peps(beta):
    """A[s,l,u,r,d] = Q[s,l]Q[s,u]Q[s,r]Q[s,d], Q Q^T = exp(beta/2 s s'):
    then <psi|psi> is the classical Ising partition function at beta and
    <sz sz> on a bond is the nearest-neighbour correlation."""
    W = np.array([[np.exp(beta / 2), np.exp(-beta / 2)], [np.exp(-beta / 2), np.exp(beta / 2)]])
    w, U = np.linalg.eigh(W)
    Q = U @ np.diag(np.sqrt(w)) @ U.T
    return np.einsum("sl,su,sr,sd->slurd", Q, Q, Q, Q)


def _golden_onsager():
    vals = {}
    with open(os.path.join(GOLDEN, "onsager_nn.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                b, v = line.split()
                vals[float(b)] = float(v)
    return vals


def test_onsager_golden_values():
    for beta, v in _golden_onsager().items():
        assert abs(_onsager_nn(beta) - v) < 1e-11


@pytest.mark.parametrize("beta,method,boot", [(0.3, O.STANDARD, 1), (0.3, O.REDUCED, 3),
                                              (0.3, O.REDUCED_ENV, 3), (0.4, O.STANDARD, 1)])
def test_onsager_nearest_neighbour(beta, method, boot):
    """Converged truncated CTMRG (projectors and SVDs included) reproduces
    Onsager's exact nearest-neighbour correlation.  The Ising legs span a
    2-dim subspace of each D^2 bond, so the reduced move needs a few
    standard iterations to reach full numerical rank before it takes over."""
    r = _ising_solve(beta, method, boot)
    exact = _golden_onsager()[beta]
    for e in r["e_bond"]:
        assert abs(e - exact) < 1e-9


# ------------------------------------------------------------ truncation

def _mats():
    rng = np.random.default_rng(7)
    out = [rng.standard_normal((12, 12)), rng.standard_normal((20, 9)),
           rng.standard_normal((7, 15))]
    lo = rng.standard_normal((16, 3)) @ rng.standard_normal((3, 10))   # rank 3
    out.append(lo)
    # graded spectrum
    Q1 = random_orthogonal(10, 1); Q2 = random_orthogonal(10, 2)
    out.append(Q1 @ np.diag(10.0 ** -np.arange(10)) @ Q2)
    return out


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_truncate_eckart_young(k):
    """||M - U U^T M||_F^2 = sum of discarded sigma^2 (eigenvalues of M M^T
    from the symmetric eigensolver, not the SVD); U^T U = I on kept
    columns; sign rule; zeroed columns below the cutoff."""
    for M in _mats():
        m, n = M.shape
        U, S = O.truncate(M, k)
        kk = min(k, m, n)
        assert U.shape == (m, kk) and S.shape == (kk,)
        lam = np.sort(np.clip(np.linalg.eigvalsh(M @ M.T), 0, None))[::-1]
        keep = S > 0
        R = M - U @ (U.T @ M)
        discarded = lam[int(keep.sum()):].sum()
        assert abs(np.sum(R * R) - discarded) <= 1e-10 * lam[0]
        np.testing.assert_allclose(S[keep] ** 2, lam[:int(keep.sum())], rtol=1e-9, atol=1e-12 * lam[0])
        G = U.T @ U
        np.testing.assert_allclose(G, np.diag(keep.astype(float)), atol=1e-12)
        for c in np.nonzero(keep)[0]:
            a = np.abs(U[:, c])
            i = np.nonzero(a >= (1 - OC.SIGN_TIE) * a.max())[0][0]
            assert U[i, c] > 0
        assert np.all(U[:, ~keep] == 0)


def test_truncate_rank_deficient_cutoff():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((16, 2)) @ rng.standard_normal((2, 16))
    U, S = O.truncate(M, 6)
    assert np.count_nonzero(S) == 2
    assert np.all(U[:, 2:] == 0)
    U0, S0 = O.truncate(np.zeros((4, 5)), 3)
    assert U0.shape == (4, 3) and not U0.any() and not S0.any()


def test_truncate_sign_tie_is_stable():
    """Mirrored entries (the ket <-> bra symmetry of the standard move)
    produce exact ties; the lowest tied row decides, whatever the rounding."""
    v = np.array([0.0, 0.6, 0.2, -0.6, 0.1])
    M = np.outer(v, [1.0, 2.0])
    for eps in (0.0, 1e-15, -1e-15):
        Mp = M.copy(); Mp[3, 0] *= (1 + eps)
        U, _ = O.truncate(Mp, 1)
        assert U[1, 0] > 0


# ------------------------------------------------------------ invariances

def _gauge(A, B, seed):
    D = A.shape[1]
    O1, O2, O3, O4 = [random_orthogonal(D, seed + i) for i in range(4)]
    A2 = np.einsum("slurd,lL,uU,rR,dD->sLURD", A, O2, O3, O1, O4)
    B2 = np.einsum("slurd,lL,uU,rR,dD->sLURD", B, O1, O4, O2, O3)
    return A2, B2


@pytest.mark.parametrize("method", [O.STANDARD, O.REDUCED, O.REDUCED_ENV])
@pytest.mark.parametrize("D,chi,its", [(2, 8, 20), (3, 18, 3)])
def test_bond_gauge_invariance(method, D, chi, its):
    """An independent real orthogonal change of basis on each of the four
    bond types leaves the state, hence every bond energy, unchanged; any
    projector applied to the wrong bond or leg would break this."""
    A, B = site_tensors(2, D, 1)
    A2, B2 = _gauge(A, B, 10)
    r1 = O.solve(A, B, chi, method, max_iters=its)
    r2 = O.solve(A2, B2, chi, method, max_iters=its)
    np.testing.assert_allclose(r1["e_bond"], r2["e_bond"], rtol=0, atol=1e-12)


def test_broken_gauge_changes_energy():
    A, B = site_tensors(2, 2, 1)
    Q = random_orthogonal(2, 3)
    A3 = np.einsum("slurd,rR->sluRd", A, Q)
    e1 = O.solve(A, B, 8, O.REDUCED, max_iters=3)["e_site"]
    e2 = O.solve(A3, B, 8, O.REDUCED, max_iters=3)["e_site"]
    assert abs(e1 - e2) > 1e-3


@pytest.mark.parametrize("method", [O.STANDARD, O.REDUCED, O.REDUCED_ENV])
def test_spin_rotation_invariance(method):
    """A real rotation of the physical index of A and B is a global SU(2)
    rotation: S.S energies and the norm network (corner spectra) are
    unchanged."""
    A, B = site_tensors(2, 2, 2)
    R = random_rotation2(9)
    A2 = np.einsum("st,tlurd->slurd", R, A)
    B2 = np.einsum("st,tlurd->slurd", R, B)
    r1 = O.solve(A, B, 8, method, max_iters=6)
    r2 = O.solve(A2, B2, 8, method, max_iters=6)
    np.testing.assert_allclose(r1["e_bond"], r2["e_bond"], rtol=0, atol=1e-12)
    s1, s2 = O.corner_spectra(r1["env"], 8), O.corner_spectra(r2["env"], 8)
    for k in O.CORNERS:
        np.testing.assert_allclose(s1[k], s2[k], rtol=0, atol=1e-9)


def test_swap_sublattices():
    """Exchanging A and B exchanges the a and b environments."""
    A, B = site_tensors(2, 2, 5)
    for method in (O.STANDARD, O.REDUCED):
        r1 = O.solve(A, B, 8, method, max_iters=4)
        r2 = O.solve(B, A, 8, method, max_iters=4)
        e1, e2 = r1["e_bond"], r2["e_bond"]
        np.testing.assert_allclose([e1[0], e1[1], e1[2], e1[3]], [e2[1], e2[0], e2[3], e2[2]],
                                   rtol=0, atol=1e-12)
        for key in O.ENV_KEYS:
            other = key[:2] + ("b" if key[2] == "a" else "a")
            np.testing.assert_allclose(r1["env"][key], r2["env"][other], rtol=0, atol=1e-9)


def test_c4v_symmetric_state_has_equal_directions():
    """A = B invariant under the 8 symmetries of the square: once converged
    the four corners have the same spectrum (the rotation relabel and the
    site transposes of every frame are pinned together)."""
    A, _ = site_tensors(2, 2, 6)
    perms = []
    for r in range(4):
        X = O.rotate_site(A, r)
        perms.append(X)
        perms.append(X.transpose(0, 3, 2, 1, 4))     # mirror l <-> r
    S = sum(perms) / len(perms)
    r = O.solve(S, S, 8, O.STANDARD, max_iters=60, tol=1e-12)
    sp = O.corner_spectra(r["env"], 8)
    for k in ("C2a", "C3a", "C4a", "C1b"):
        np.testing.assert_allclose(sp[k], sp["C1a"], rtol=0, atol=1e-8)


# ------------------------------------------------------------ reduced anchor

def test_reduced_row_is_exact_without_truncation():
    """If chi' is large enough that v_l, v_r truncate nothing, the
    approximated row C'1 T'2 C'2 equals the reduced half-network
    [C1 T2 C2; T1 z T3] contracted in one go (Appendix, Fig. A)."""
    A, B = site_tensors(2, 2, 8)
    env = O.solve(A, B, 8, O.STANDARD, max_iters=2)["env"]
    sites = {"a": A, "b": B}
    for z in "ab":
        _, _, parts = OC.anchor_reduced(env, sites, z, 64, return_parts=True)
        X = sites[z]
        # one network, contracted by numpy's path optimiser in one call:
        # C1[m,i] T1[j,k,l,m] T2[i,u,v,q] A[s,k,u,r,d] A[s,l,v,R,D] C2[q,n] T3[n,r,R,o]
        exact = np.einsum("mi,jklm,iuvq,skurd,slvRD,qn,nrRo->jdDo",
                          env[f"C1{z}"], env[f"T1{z}"], env[f"T2{z}"], X, X,
                          env[f"C2{z}"], env[f"T3{z}"], optimize=True)
        np.testing.assert_allclose(parts["Mp"], exact, rtol=0, atol=1e-12 * np.abs(exact).max())


def test_reduced_env_network_and_rank():
    """The reduced-env sub-network (Sec. III) is [C1 T2 C2; T1 z T3]
    contracted as one network (written out independently here, ket and bra
    sites instead of the double layer), and its isometry spans that
    network's column space: rank at most the far bond T3.q, and v v^T M = M
    when chi covers the rank."""
    A, B = site_tensors(2, 2, 8)
    env = O.solve(A, B, 8, O.STANDARD, max_iters=2)["env"]
    sites = {"a": A, "b": B}
    for z in "ab":
        X = sites[z]
        exact = np.einsum("mi,jklm,iuvq,skurd,slvRD,qn,nrRo->jdDo",
                          env[f"C1{z}"], env[f"T1{z}"], env[f"T2{z}"], X, X,
                          env[f"C2{z}"], env[f"T3{z}"], optimize=True)
        M = OC.reduced_half_network(env, sites, z)
        np.testing.assert_allclose(M, exact, rtol=0, atol=1e-13 * np.abs(exact).max())
        nj, D, _, nj2 = M.shape
        v = OC.anchor_reduced_env(env, sites, z, 8)
        assert v.shape == (nj, D, D, min(8, nj2))
        V = v.reshape(nj * D * D, -1)
        Mm = M.reshape(nj * D * D, nj2)
        np.testing.assert_allclose(V @ (V.T @ Mm), Mm, rtol=0, atol=1e-12 * np.abs(Mm).max())


def test_reduced_env_and_sequential_projectors_agree_without_first_stage_cut():
    """With nothing cut before the last stage (v_l, v_r and v^1 keep their
    full range, as from the traced-boundary start at D=2, chi=16), the
    sequential-order isometry v = (v^1 x 1) v^2 spans the same subspace as
    the reduced-env one: both are the column space of the same reduced
    half-network (Secs. III-IV)."""
    A, B = site_tensors(2, 2, 5)
    env = O.init_env(A, B)
    sites = {"a": A, "b": B}
    for z in "ab":
        v1, v2 = OC.anchor_reduced(env, sites, z, 16)
        nj, D, c1 = v1.shape
        assert c1 == nj * D
        vs = np.einsum("jdm,mbn->jdbn", v1, v2).reshape(nj * D * D, -1)
        ve = OC.anchor_reduced_env(env, sites, z, 16).reshape(nj * D * D, -1)
        assert vs.shape == ve.shape
        np.testing.assert_allclose(vs @ vs.T, ve @ ve.T, rtol=0, atol=1e-12)


def test_sequential_isometries_reproduce_first_stage():
    """With chi'' >= rank N, v2 spans range(N), so the composite
    v = v1 v2 projects M' exactly as v1 alone does (Sec. IV)."""
    A, B = site_tensors(2, 2, 9)
    env = O.solve(A, B, 8, O.REDUCED, max_iters=3)["env"]
    sites = {"a": A, "b": B}
    for z in "ab":
        v1, v2, parts = OC.anchor_reduced(env, sites, z, 8, return_parts=True)
        Mp = parts["Mp"]
        nj, D = Mp.shape[0], Mp.shape[1]
        Mmat = Mp.reshape(nj * D * D, -1)
        v = np.einsum("jdm,mDn->jdDn", v1, v2).reshape(nj * D * D, -1)
        P1 = np.einsum("jdm,kem->jdke", v1, v1).reshape(nj * D, nj * D)
        lhs = v @ (v.T @ Mmat)
        rhs = np.einsum("ab,bDo->aDo", P1, Mp.reshape(nj * D, D, -1)).reshape(nj * D * D, -1)
        np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(Mmat).max())
        np.testing.assert_allclose(v.T @ v, np.diag((np.abs(v).sum(0) > 0).astype(float)), atol=1e-12)


@pytest.mark.parametrize("method", [O.REDUCED, O.REDUCED_ENV])
def test_reduced_approaches_standard_as_chi_grows(method):
    """Trend only (Sec. V: the methods agree for large chi); the finite-chi
    gap itself is not pinned.  D=2, chi = 4 and 16 (the largest bond the
    traced boundary can reach at D=2 is D^4 = 16)."""
    A, B = site_tensors(2, 2, 0)
    gaps = []
    for chi in (4, 16):
        es = O.solve(A, B, chi, O.STANDARD, max_iters=20, tol=1e-10)["e_site"]
        er = O.solve(A, B, chi, method, max_iters=20, tol=1e-10)["e_site"]
        gaps.append(abs(es - er))
    assert gaps[1] < gaps[0] / 10


def test_side_second_stage_enters_only_through_its_range():
    """The side isometries' second stage v_l^2 (and v_r^2) is summed over
    between C'^1 = v_l^2T L' and the v_l^2 of the absorption chain, so M'
    depends on it only through v_l^2 v_l^2T (Appendix, Sec. IV).  When that
    stage keeps every column, any orthonormal basis of range(L') gives the
    same M'; the GPU path takes the QR basis there.  A basis of a smaller
    subspace changes M' (the check is sensitive)."""
    A, B = site_tensors(2, 2, 11)
    env = O.solve(A, B, 8, O.REDUCED, max_iters=3)["env"]
    sites = {"a": A, "b": B}
    for z in "ab":
        _, _, parts = OC.anchor_reduced(env, sites, z, 8, return_parts=True)
        vl1, vr1, vl2, vr2 = parts["vl1"], parts["vr1"], parts["vl2"], parts["vr2"]
        Lp = np.einsum("ikm,iklj->mlj", vl1, parts["L"])
        Rp = np.einsum("ikm,iklj->mlj", vr1, parts["R"])
        c1, D, nj = Lp.shape
        assert vl2.shape[2] == nj and vr2.shape[2] == Rp.shape[2]   # every column kept

        def mprime(wl2, wr2):
            Cp1 = np.einsum("mln,mlj->nj", wl2, Lp)
            Cp2 = np.einsum("mln,mlj->nj", wr2, Rp)
            Tp2 = OC.absorb_chain(env[f"T2{z}"], OC._site_in_T2(sites[z]), vl1, wl2, vr1, wr2)
            Mp = np.einsum("nj,ndDo->jdDo", Cp1, Tp2)
            return np.einsum("jdDo,ok->jdDk", Mp, Cp2)

        ref = mprime(vl2, vr2)
        np.testing.assert_allclose(ref, parts["Mp"], rtol=0, atol=1e-13 * np.abs(ref).max())
        ql = np.linalg.qr(Lp.reshape(c1 * D, nj))[0].reshape(c1, D, nj)
        qr = np.linalg.qr(Rp.reshape(Rp.shape[0] * D, -1))[0].reshape(Rp.shape[0], D, -1)
        np.testing.assert_allclose(mprime(ql, qr), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        rot = random_orthogonal(nj, 5)
        rl = np.einsum("mln,nk->mlk", vl2, rot)
        np.testing.assert_allclose(mprime(rl, vr2), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.abs(mprime(vl2[:, :, :-1], vr2) - ref).max() > 1e-6 * np.abs(ref).max()


def test_left_move_changes_only_the_left_column():
    """A left move (two insertions) rewrites C1, T1 and C4 of both
    sublattices and nothing else (Sec. II), so the right-side isometries
    built from C2 and T3 are the same for both insertions of a move; the GPU
    path computes them once per move."""
    A, B = site_tensors(2, 2, 12)
    env = O.solve(A, B, 8, O.REDUCED, max_iters=2)["env"]
    for r in range(4):
        new = OC.move(env, A, B, r, 8, O.REDUCED)
        changed = {k for k in O.ENV_KEYS if not np.array_equal(new[k], env[k])}
        left = {f"{kind}{(i - 1 + r) % 4 + 1}{z}" for kind, i in (("C", 1), ("T", 1), ("C", 4))
                for z in "ab"}
        assert changed <= left and changed, (r, sorted(changed))
        env = new


# ------------------------------------------------------------ observables

SX = np.array([[0.0, 0.5], [0.5, 0.0]])
SZ = np.array([[0.5, 0.0], [0.0, -0.5]])


@pytest.mark.parametrize("seed", [0, 3])
def test_product_state_one_site_values_and_no_correlation(seed):
    """D = 1 product states: <O>_z = psi^T O psi / psi^T psi exactly, and
    every connected correlation along a row vanishes."""
    A, B, pa, pb = product_state_tensors(2, seed)
    env = O.solve(A, B, 3, O.REDUCED, max_iters=2)["env"]
    for op in (SX, SZ):
        got = O.expect1(env, A, B, op)
        assert abs(got[0] - pa @ op @ pa / (pa @ pa)) < 1e-14
        assert abs(got[1] - pb @ op @ pb / (pb @ pb)) < 1e-14
    c = O.row_correlation(env, A, B, SZ, 5)
    assert np.abs(c).max() < 1e-14


def test_neel_staggered_magnetisation():
    A = np.zeros((2, 1, 1, 1, 1)); A[0] = 1.0
    B = np.zeros((2, 1, 1, 1, 1)); B[1] = 1.0
    env = O.solve(A, B, 2, O.STANDARD, max_iters=2)["env"]
    assert abs(O.staggered_magnetisation(env, A, B) - 0.5) < 1e-15


def test_nearest_correlation_equals_bond_network():
    """C(1) from the row contraction equals <O O> from the (independently
    written) bond energy network minus <O>_a <O>_b, on a generic state."""
    A, B = site_tensors(2, 2, 6)
    env = O.solve(A, B, 8, O.REDUCED, max_iters=6)["env"]
    c1 = O.row_correlation(env, A, B, SZ, 1)[0]
    one = np.eye(2)
    za = O.bond_energy(env, A, B, "a", np.kron(SZ, one), 0)
    zb = O.bond_energy(env, A, B, "a", np.kron(one, SZ), 0)
    zz = O.bond_energy(env, A, B, "a", np.kron(SZ, SZ), 0)
    assert abs(c1 - (zz - za * zb)) < 1e-13


def test_ising_row_correlation_onsager_and_decay():
    """Classical Ising PEPS at beta = 0.3 (disordered, <sigma^z> = 0): the
    row correlation of sigma^z at distance 1 is Onsager's nearest-neighbour
    value, and it decays with distance (finite correlation length)."""
    A = _ising_peps(0.3)
    sz = np.diag([1.0, -1.0])
    env = _ising_solve(0.3, O.STANDARD, 1)["env"]
    m = O.expect1(env, A, A, sz)
    assert abs(m[0]) < 1e-10 and abs(m[1]) < 1e-10
    c = O.row_correlation(env, A, A, sz, 8)
    assert abs(c[0] - _golden_onsager()[0.3]) < 1e-9
    assert all(c[i + 1] < c[i] for i in range(7)) and c[7] > 0
    # geometric decay: the ratio of successive values settles
    ratios = [c[i + 1] / c[i] for i in range(3, 7)]
    assert max(ratios) - min(ratios) < 0.05


# ------------------------------------------------------------ chi' and chi''

def test_chi_p_and_chi_pp_reach_the_right_stages():
    """chi' bounds the anchors' first stage v^1 (Sec. IV) and chi'' the
    helper isometries' first stage (App.).  With both large enough that no
    first stage cuts (here 16 = chi D at D=2, chi=8), the sequential-order
    isometry spans the column space of the exact reduced half-network M,
    like the reduced-env one: P M = M to rounding (the directions of M with
    singular values near 1e-12 are themselves fixed only to eps / gap, so
    the projectors are compared on M).  With chi' = chi (the default) v^1
    cuts and P M misses M by far more.  Shapes follow chi', chi''."""
    A, B = site_tensors(2, 2, 4)
    env = O.solve(A, B, 8, O.STANDARD, max_iters=2)["env"]
    sites = {"a": A, "b": B}
    for z in "ab":
        M = OC.reduced_half_network(env, sites, z)
        nj, D, _, nj2 = M.shape
        Mm = M.reshape(nj * D * D, nj2)
        nrm = np.linalg.norm(Mm)
        v1, v2, parts = OC.anchor_reduced(env, sites, z, 8, chi_p=16, chi_pp=16, return_parts=True)
        assert v1.shape == (nj, D, 16) and parts["vl1"].shape[2] == 16
        vs = np.einsum("jdm,mbn->jdbn", v1, v2).reshape(nj * D * D, -1)
        assert np.linalg.norm(vs @ (vs.T @ Mm) - Mm) < 1e-13 * nrm
        ve = OC.anchor_reduced_env(env, sites, z, 8).reshape(nj * D * D, -1)
        assert np.linalg.norm(ve @ (ve.T @ Mm) - Mm) < 1e-13 * nrm
        v1d, v2d = OC.anchor_reduced(env, sites, z, 8)
        assert v1d.shape == (nj, D, 8)
        vd = np.einsum("jdm,mbn->jdbn", v1d, v2d).reshape(nj * D * D, -1)
        assert np.linalg.norm(vd @ (vd.T @ Mm) - Mm) > 1e-9 * nrm
    # a whole solve with chi' = chi'' = chi is the default one
    r0 = O.solve(A, B, 8, O.REDUCED, max_iters=3)
    r1 = O.solve(A, B, 8, O.REDUCED, max_iters=3, chi_p=8, chi_pp=8)
    assert r0["e_site"] == r1["e_site"]

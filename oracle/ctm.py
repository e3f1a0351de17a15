"""Plain FP64 NumPy corner-transfer oracle (test infrastructure only).

What it computes, and where each part comes from in the paper
(Lan & Evenbly, arXiv:2306.08212):

* two-site unit cell {A, B} of 5-index tensors (d, D, D, D, D); double-layer
  transfer tensor a = sum_s A A*                     -- Sec. II, Fig. 1(a,b)
* environment {C^i, T^i} with boundary dimension chi -- Sec. II, Fig. 1(d)
* CTM iteration of left, right, up, down moves; the left move inserts a
  column twice and truncates enlarged bonds with isometries
                                                     -- Sec. II, Fig. 2(a,b)
* standard isometry: top-chi left singular vectors of the half-plaquette
  sub-network, cost chi^3 D^6                        -- Sec. II, Fig. 2(c)
* reduced (sequential-order) move: split isometries v^1 (boundary + ket)
  and v^2 (chi' + bra) from a (chi D) x (chi D) SVD and a (chi D) x chi SVD
  of an approximated row {C'^1, T'^2, C'^2}; ket-then-bra absorption
                                                     -- Sec. III-IV, Figs. 3-4
* the row {C'^1, T'^2, C'^2} built with helper isometries {v_l, v_r}
  computed from {C^1, T^1} and {C^2, T^3} alone     -- Appendix, Fig. A
* reduced-env move: one 4-index isometry from the reduced half-network
  [C1 T2 C2; T1 z T3] reshaped (chi D^2) x chi, absorbed like the
  standard one                                       -- Sec. III, Fig. 3(a,b)
* Heisenberg bond energy                             -- Sec. V, Eq. (1)

Conventions where the paper is silent (its figures are missing), fixed here
and shared by the GPU library only through this description:

Lattice.  Checkerboard; every neighbour of an a-site is a b-site.  For each
sublattice z in {a, b} the state holds 16 tensors C1..C4, T1..T4 (per z):
C1 up-left, C2 up-right, C3 down-right, C4 down-left corner of a z-site;
T1, T2, T3, T4 the edges left of, above, right of and below a z-site.

Index order is clockwise around the boundary (C4 T1 C1 T2 C2 T3 C3 T4):
C^i[p, q]: p bonds to T^i, q bonds to T^{i+1}; T^i[p, k, b, q]: p toward
C^{i-1}, q toward C^i, (k, b) the ket and bra legs into the site.
Site tensors are A[s, l, u, r, d].

Rotation.  A quarter turn counter-clockwise (top edge becomes left edge) is
a pure relabel: role C^i <- stored C^{i+r}, role T^i <- stored T^{i+r}, and
every site tensor is transposed (s,l,u,r,d) -> (s,u,r,d,l) per quarter
turn.  Every move is the left move in frame r (left 0, up 1, right 2,
down 3).  The iteration order is left, right, up, down.

Init.  Each environment tensor is the single boundary site it stands for
with its outward legs traced (ket index = bra index, summed); fused
(k, b) bonds have dimension D^2; each tensor is normalised.

Bond dimensions are decided by shapes only: a truncation of an m x n
matrix to k keeps min(k, m, n) columns.  Columns whose singular value is
<= TAU * sigma_0 are set to zero; every kept column is sign-fixed: among
the rows whose magnitude is within a relative SIGN_TIE of the column's
largest, the lowest one is made positive (exact ties are common: the
standard move is symmetric under ket <-> bra, so its singular vectors come
in mirrored pairs of entries).

Bootstrap.  The reduced sub-network has rank at most the dimension of the
far-side boundary bond (T^3.q), so it cannot grow a bond.  An insertion of
the reduced method therefore uses the standard isometries whenever the
reduced rule would leave a new bond smaller (by shape) than the standard
rule would; optionally the first boot_iters iterations (default 0) use the
standard move throughout.

THIS MODULE IS TEST INFRASTRUCTURE; see the package docstring.
"""

from __future__ import annotations

import numpy as np

TAU = 1e-14
SIGN_TIE = 1e-8
# LAPACK driver of the SVD in truncate: "gesdd" (divide and conquer, numpy's
# default) or "gesvd" (QR iteration).  Both are backward-stable SVDs; running
# the oracle with each measures how far rounding alone moves its results.
SVD_DRIVER = "gesdd"
STANDARD = "standard"
REDUCED = "reduced"
REDUCED_ENV = "reduced_env"

CORNERS = [f"C{i}{z}" for z in "ab" for i in range(1, 5)]
ENV_KEYS = [f"{k}{i}{z}" for z in "ab" for k in "CT" for i in range(1, 5)]


def _c(spec, *ops):
    """One pairwise (or small) tensor contraction, einsum notation."""
    return np.einsum(spec, *ops, optimize=True)


def _other(z):
    return "b" if z == "a" else "a"


# ---------------------------------------------------------------- operators

def heisenberg_h2(d=2):
    """Two-site S.S with S = sigma / 2 (antiferromagnetic sign), as a
    (d*d) x (d*d) matrix h[(s1 s2), (s1' s2')].  Sec. V, Eq. (1): the
    printed minus sign and the word 'Pauli' are read as the spin-1/2
    antiferromagnet in S = sigma/2 units, the model whose QMC energy the
    paper quotes (-0.669437 per site)."""
    if d != 2:
        raise ValueError("Heisenberg operator defined for d = 2")
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    sz = np.array([[1.0, 0.0], [0.0, -1.0]])
    # sigma^y (x) sigma^y is real: -(i sigma^y) (x) (i sigma^y)
    isy = np.array([[0.0, 1.0], [-1.0, 0.0]])
    return 0.25 * (np.kron(sx, sx) - np.kron(isy, isy) + np.kron(sz, sz))


def double_layer(A):
    """Transfer tensor a[kl,bl,ku,bu,kr,br,kd,bd] = sum_s A[s,k..] A[s,b..]
    (Sec. II, Fig. 1(b)); real tensors so A* = A."""
    return _c("slurd,sLURD->lLuUrRdD", A, A)


def rotate_site(A, r):
    """Site tensor in frame r: (s,l,u,r,d) -> (s,u,r,d,l) per quarter turn."""
    for _ in range(r % 4):
        A = A.transpose(0, 2, 3, 4, 1)
    return np.ascontiguousarray(A)


def frame_env(env, r):
    """Relabel the stored environment into frame r (role X^i = stored X^{i+r})."""
    out = {}
    for k in "CT":
        for i in range(1, 5):
            j = (i - 1 + r) % 4 + 1
            for z in "ab":
                out[f"{k}{i}{z}"] = env[f"{k}{j}{z}"]
    return out


def unframe_env(fenv, r):
    """Inverse of frame_env."""
    out = {}
    for k in "CT":
        for i in range(1, 5):
            j = (i - 1 + r) % 4 + 1
            for z in "ab":
                out[f"{k}{j}{z}"] = fenv[f"{k}{i}{z}"]
    return out


# ---------------------------------------------------------------- truncation

def truncate(M, k, tau=None):
    """Top-k left singular vectors of the matrix M (Sec. II: the isometry is
    the truncated unitary of an SVD of a sub-network; Sec. IV: the same for
    v^1 and v^2).  Returns (U, S) with min(k, m, n) columns; columns with
    sigma <= tau * sigma_0 are zeroed (tau defaults to the module's TAU,
    read at call time); each kept column is sign-fixed (the lowest row within
    SIGN_TIE of the largest magnitude is positive)."""
    if tau is None:
        tau = TAU
    m, n = M.shape
    kk = min(k, m, n)
    if SVD_DRIVER == "gesdd":
        U, S, _ = np.linalg.svd(M, full_matrices=False)
    else:
        import scipy.linalg
        U, S, _ = scipy.linalg.svd(M, full_matrices=False, lapack_driver=SVD_DRIVER)
    U = np.array(U[:, :kk], dtype=np.float64)
    S = np.array(S[:kk], dtype=np.float64)
    if kk == 0 or not S[0] > 0.0:
        return np.zeros((m, kk)), np.zeros(kk)
    drop = S <= tau * S[0]
    U[:, drop] = 0.0
    S[drop] = 0.0
    for c in range(kk):
        if drop[c]:
            continue
        a = np.abs(U[:, c])
        # lowest row whose magnitude is within SIGN_TIE of the largest
        i = int(np.nonzero(a >= (1.0 - SIGN_TIE) * a.max())[0][0])
        if U[i, c] < 0.0:
            U[:, c] = -U[:, c]
    return U, S


def _iso(M, k, untruncated):
    if untruncated:
        return np.eye(M.shape[0])
    return truncate(M, k)[0]


# ---------------------------------------------------------------- init

def init_env(A, B):
    """Traced-boundary environment (one boundary site per tensor, outward
    legs traced, fused (k,b) -> k*D+b bonds), each normalised."""
    D = A.shape[1]
    D2 = D * D
    sites = {"a": A, "b": B}
    env = {}
    for z in "ab":
        X = sites[z]             # corners are diagonal neighbours: same sublattice
        Y = sites[_other(z)]     # edges are nearest neighbours: other sublattice
        # C1[(kd,bd),(kr,br)]: l, u traced
        env[f"C1{z}"] = _c("slurd,sluRD->dDrR", X, X).reshape(D2, D2)
        # C2[(kl,bl),(kd,bd)]: u, r traced
        env[f"C2{z}"] = _c("slurd,sLurD->lLdD", X, X).reshape(D2, D2)
        # C3[(ku,bu),(kl,bl)]: r, d traced
        env[f"C3{z}"] = _c("slurd,sLUrd->uUlL", X, X).reshape(D2, D2)
        # C4[(kr,br),(ku,bu)]: l, d traced
        env[f"C4{z}"] = _c("slurd,slURd->rRuU", X, X).reshape(D2, D2)
        # T1[(kd,bd), kr, br, (ku,bu)]: l traced
        env[f"T1{z}"] = _c("slurd,slURD->dDrRuU", Y, Y).reshape(D2, D, D, D2)
        # T2[(kl,bl), kd, bd, (kr,br)]: u traced
        env[f"T2{z}"] = _c("slurd,sLuRD->lLdDrR", Y, Y).reshape(D2, D, D, D2)
        # T3[(ku,bu), kl, bl, (kd,bd)]: r traced
        env[f"T3{z}"] = _c("slurd,sLUrD->uUlLdD", Y, Y).reshape(D2, D, D, D2)
        # T4[(kr,br), ku, bu, (kl,bl)]: d traced
        env[f"T4{z}"] = _c("slurd,sLURd->rRuUlL", Y, Y).reshape(D2, D, D, D2)
    return {k: v / np.linalg.norm(v) for k, v in env.items()}


# ---------------------------------------------------------------- anchors

def anchor_standard(fenv, sites, z, chi, untruncated=False):
    """4-index isometry v_z[j, kd, bd, nu] for the bond below a z-site in
    the left column (Sec. II, Fig. 2(c)): top-chi left singular vectors of
    M = Q1 Q2, Q1 = {C1_z, T2_z, T1_z, a_z}, Q2 = {T2_w, C2_w, T3_w, a_w}
    with w the right neighbour of z, reshaped (chi D^2) x (D^2 chi)."""
    w = _other(z)
    D = sites[z].shape[1]
    C1, T1, T2 = fenv[f"C1{z}"], fenv[f"T1{z}"], fenv[f"T2{z}"]
    T2w, C2w, T3w = fenv[f"T2{w}"], fenv[f"C2{w}"], fenv[f"T3{w}"]
    nj = T1.shape[0]
    if untruncated:
        return np.eye(nj * D * D).reshape(nj, D, D, nj * D * D)
    az, aw = double_layer(sites[z]), double_layer(sites[w])
    X = _c("mn,nuvq->muvq", C1, T2)
    Y = _c("jklm,muvq->jkluvq", T1, X)
    Q1 = _c("jkluvq,kluvrRdD->jdDqrR", Y, az)
    X2 = _c("quvn,nm->quvm", T2w, C2w)
    Y2 = _c("quvm,mrRj->quvrRj", X2, T3w)
    Q2 = _c("quvrRj,lLuvrRdD->qlLdDj", Y2, aw)
    nq, nj2 = T2.shape[3], T3w.shape[3]
    M = Q1.reshape(nj * D * D, nq * D * D) @ Q2.reshape(nq * D * D, D * D * nj2)
    U = truncate(M, chi)[0]
    return U.reshape(nj, D, D, U.shape[1])


def _split_iso(X, chi, untruncated, chi1=None):
    """Two-stage isometry of a 4-index X[i, k, b, j] bonded on (i, k, b):
    v1 from X as [(i,k),(b,j)] (top chi1, default chi), then v2 from
    X' = v1^T X as [(mu,b), j] (top chi); returns (v1[i,k,mu], v2[mu,b,nu],
    X''[nu, j]) (Appendix, Fig. A(c) for {C^1,T^1} and {C^2,T^3}; Sec. IV for
    the row {C'^1,T'^2,C'^2})."""
    ni, D, _, nj = X.shape
    v1 = _iso(X.reshape(ni * D, D * nj), chi if chi1 is None else chi1, untruncated)
    c1 = v1.shape[1]
    v1 = v1.reshape(ni, D, c1)
    Xp = _c("ikm,iklj->mlj", v1, X)
    v2 = _iso(Xp.reshape(c1 * D, nj), chi, untruncated)
    c2 = v2.shape[1]
    v2 = v2.reshape(c1, D, c2)
    Xpp = _c("mln,mlj->nj", v2, Xp)
    return v1, v2, Xpp


def absorb_chain(T, S, vp1, vp2, vq1, vq2):
    """Sequential ket-then-bra absorption of one site into an edge tensor
    (Sec. IV, Fig. 4(b)): T[p,k,b,q] with site S[s, in, p-side, open,
    q-side]; the p-side bond is truncated by (vp1, vp2), the q-side bond by
    (vq1, vq2); v^1 acts on (boundary, ket), v^2 on (chi', bra).  Order:
    T.vp1, .A (ket), .vq1, vp2., .A* (bra), .vq2.  Returns out[nu_p, ko,
    bo, nu_q]."""
    X1 = _c("pkbq,pim->kbqim", T, vp1)
    X2 = _c("kbqim,skioj->bqmsoj", X1, S)
    X3 = _c("bqmsoj,qjn->bmson", X2, vq1)
    X4 = _c("bmson,mIv->vIbson", X3, vp2)
    X5 = _c("vIbson,sbIOJ->vonOJ", X4, S)
    return _c("vonOJ,nJw->voOw", X5, vq2)


def _site_in_T1(A):
    """A[s,l,u,r,d] -> S[s, in=l, p-side=d, open=r, q-side=u] (T1 chain)."""
    return np.ascontiguousarray(A.transpose(0, 1, 4, 3, 2))


def _site_in_T2(A):
    """A[s,l,u,r,d] -> S[s, in=u, p-side=l, open=d, q-side=r] (T2 chain)."""
    return np.ascontiguousarray(A.transpose(0, 2, 1, 4, 3))


def anchor_reduced(fenv, sites, z, chi, untruncated=False, return_parts=False, chi_p=None,
                   chi_pp=None):
    """Split isometries (v^1_z[j,kd,mu], v^2_z[mu,bd,nu]) for the bond below
    a z-site in the left column, from the reduced half-network
    [C1 T2 C2; T1 z T3] of z alone (Sec. III: the right half is replaced by
    {C^2, T^3}; Fig. 3(c): further approximated by the row {C'^1, T'^2,
    C'^2}; Appendix: that row is built with {v_l, v_r} from {C^1, T^1} and
    {C^2, T^3}).  M' is reshaped (chi D) x (D chi) with the ket leg paired
    with the left boundary bond (Sec. IV), then N = v1^T M' as (chi' D) x chi.
    chi_p (chi', Sec. IV) bounds v^1 and chi_pp (chi'', Sec. V) the first
    stage of the helper isometries; both default to chi (the paper's runs).
    """
    chi_p = chi if chi_p is None else chi_p
    chi_pp = chi if chi_pp is None else chi_pp
    C1, T1, T2 = fenv[f"C1{z}"], fenv[f"T1{z}"], fenv[f"T2{z}"]
    C2, T3 = fenv[f"C2{z}"], fenv[f"T3{z}"]
    D = sites[z].shape[1]
    nj, nj2 = T1.shape[0], T3.shape[3]
    if untruncated:
        v1 = np.eye(nj * D).reshape(nj, D, nj * D)
        v2 = np.eye(nj * D * D).reshape(nj * D, D, nj * D * D)
        return v1, v2
    # left part: L[i,kl,bl,j] = C1[m,i] T1[j,kl,bl,m]
    L = _c("mi,jklm->iklj", C1, T1)
    vl1, vl2, Cp1 = _split_iso(L, chi, False, chi_pp)
    # right part: R[i,kr,br,j] = C2[i,m] T3[m,kr,br,j]
    R = _c("im,mklj->iklj", C2, T3)
    vr1, vr2, Cp2 = _split_iso(R, chi, False, chi_pp)
    Tp2 = absorb_chain(T2, _site_in_T2(sites[z]), vl1, vl2, vr1, vr2)
    Mp = _c("nj,ndDo->jdDo", Cp1, Tp2)
    Mp = _c("jdDo,ok->jdDk", Mp, Cp2)
    v1 = truncate(Mp.reshape(nj * D, D * nj2), chi_p)[0]
    c1 = v1.shape[1]
    v1 = v1.reshape(nj, D, c1)
    N = _c("jdm,jdDk->mDk", v1, Mp)
    v2 = truncate(N.reshape(c1 * D, nj2), chi)[0]
    v2 = v2.reshape(c1, D, v2.shape[1])
    if return_parts:
        return v1, v2, {"L": L, "R": R, "vl1": vl1, "vl2": vl2, "vr1": vr1,
                        "vr2": vr2, "Cp1": Cp1, "Cp2": Cp2, "Tp2": Tp2,
                        "Mp": Mp, "N": N}
    return v1, v2


def reduced_half_network(fenv, sites, z):
    """The reduced half-network [C1 T2 C2; T1 z T3] of a z-site, open on the
    bond below it: M[j, kd, bd, j'] (Sec. III: the right half {w, T2_w,
    C2_w, T3_w} of the half-plaquette is stood in for by {C2_z, T3_z}; the
    right move's isometry is dropped, since multiplying by a co-isometry
    from the right leaves the left singular vectors unchanged)."""
    C1, T1, T2 = fenv[f"C1{z}"], fenv[f"T1{z}"], fenv[f"T2{z}"]
    C2, T3 = fenv[f"C2{z}"], fenv[f"T3{z}"]
    a = double_layer(sites[z])
    L = _c("mi,jklm->iklj", C1, T1)              # L[i, kl, bl, j]
    R = _c("im,mklj->iklj", C2, T3)              # R[i', kr, br, j']
    X = _c("iklj,iuvn->kljuvn", L, T2)
    X = _c("kljuvn,kluvrRdD->jnrRdD", X, a)
    return _c("jnrRdD,nrRk->jdDk", X, R)


def anchor_reduced_env(fenv, sites, z, chi, untruncated=False):
    """Reduced-env 4-index isometry v_z[j, kd, bd, nu] (Sec. III, Fig.
    3(a,b)): the top-chi left singular vectors of the reduced half-network
    reshaped (chi D^2) x chi."""
    D = sites[z].shape[1]
    nj = fenv[f"T1{z}"].shape[0]
    if untruncated:
        return np.eye(nj * D * D).reshape(nj, D, D, nj * D * D)
    M = reduced_half_network(fenv, sites, z)
    nj2 = M.shape[3]
    U = truncate(M.reshape(nj * D * D, nj2), chi)[0]
    return U.reshape(nj, D, D, U.shape[1])


# ---------------------------------------------------------------- moves

def _new_dims(fenv, z, D, chi, method=REDUCED, chi_p=None):
    """Bond dimension below a z-site after (standard, reduced) truncation."""
    chi_p = chi if chi_p is None else chi_p
    nj = fenv[f"T1{z}"].shape[0]
    nj2 = fenv[f"T3{z}"].shape[3]
    std = min(chi, nj * D * D, D * D * nj2)
    if method == REDUCED_ENV:
        return std, min(chi, nj * D * D, nj2)
    c1 = min(chi_p, nj * D, D * nj2)
    red = min(chi, c1 * D, nj2)
    return std, red


def insertion_is_standard(fenv, sites, x, method, chi, untruncated=False, chi_p=None):
    if method == STANDARD:
        return True
    if untruncated:
        return False
    D = sites[x].shape[1]
    for z in (x, _other(x)):
        std, red = _new_dims(fenv, z, D, chi, method, chi_p)
        if red < std:
            return True
    return False


def _insert(fenv, sites, chi, method, untruncated, chi_p=None, chi_pp=None):
    """Insert one column into the left environment and truncate the enlarged
    bonds (Sec. II, Fig. 2(a,b)).  Reading: the column is {T2, site, site,
    T4} with both sublattices in turn down the column; every tensor of the
    left column (C1, T1, C4 of both sublattices) moves one site to the right
    so that all of them sit at the same column.  V_z truncates the bond below
    a z-site (equivalently above the other sublattice)."""
    std = insertion_is_standard(fenv, sites, "a", method, chi, untruncated, chi_p)
    four = std or method == REDUCED_ENV      # 4-index isometries
    V = {}
    for z in "ab":
        if std:
            V[z] = anchor_standard(fenv, sites, z, chi, untruncated)
        elif method == REDUCED_ENV:
            V[z] = anchor_reduced_env(fenv, sites, z, chi, untruncated)
        else:
            V[z] = anchor_reduced(fenv, sites, z, chi, untruncated, chi_p=chi_p, chi_pp=chi_pp)
    new = {}
    for x in "ab":
        y = _other(x)
        X = sites[x]
        C1x, T2x, T1x = fenv[f"C1{x}"], fenv[f"T2{x}"], fenv[f"T1{x}"]
        C4x, T4x = fenv[f"C4{x}"], fenv[f"T4{x}"]
        # corner up-left of the y-site right of x: C1_x T2_x, bond above x (V_y)
        G = _c("jm,mubq->jubq", C1x, T2x)
        # edge left of that y-site: T1_x + site x; top bond V_y, bottom bond V_x
        # corner down-left of that y-site: C4_x T4_x, bond below x (V_x)
        G4 = _c("mj,pkbm->jkbp", C4x, T4x)
        if four:
            vy, vx = V[y], V[x]
            C1n = _c("jubq,jubn->nq", G, vy)
            Z = _c("pklq,quvn->pkluvn", T1x, vy)
            Z = _c("pkluvn,kluvrRdD->pnrRdD", Z, double_layer(X))
            T1n = _c("pnrRdD,pdDm->mrRn", Z, vx)
            C4n = _c("jkbp,jkbn->pn", G4, vx)
        else:
            (vy1, vy2), (vx1, vx2) = V[y], V[x]
            G = _c("jubq,jum->mbq", G, vy1)
            C1n = _c("mbq,mbn->nq", G, vy2)
            T1n = absorb_chain(T1x, _site_in_T1(X), vx1, vx2, vy1, vy2)
            G4 = _c("jkbp,jkm->mbp", G4, vx1)
            C4n = _c("mbp,mbn->pn", G4, vx2)
        new[f"C1{y}"], new[f"T1{y}"], new[f"C4{y}"] = C1n, T1n, C4n
    out = dict(fenv)
    for key, val in new.items():
        nrm = np.linalg.norm(val)
        if not np.isfinite(nrm) or nrm == 0.0:
            raise FloatingPointError(f"degenerate tensor {key} in insertion")
        out[key] = val / nrm
    return out


def move(env, A, B, r, chi, method=REDUCED, untruncated=False, chi_p=None, chi_pp=None):
    """One directional move = the left move in frame r: two column
    insertions (Sec. II), so the left environment advances by one unit cell.
    method=STANDARD forces the standard isometries (used for bootstrap
    iterations); REDUCED (sequential order) and REDUCED_ENV follow the shape
    rule of the module docstring."""
    fenv = frame_env(env, r)
    sites = {"a": rotate_site(A, r), "b": rotate_site(B, r)}
    fenv = _insert(fenv, sites, chi, method, untruncated, chi_p, chi_pp)
    fenv = _insert(fenv, sites, chi, method, untruncated, chi_p, chi_pp)
    return unframe_env(fenv, r)


MOVE_ORDER = (0, 2, 1, 3)   # left, right, up, down (Sec. II)


def ctm_iteration(env, A, B, chi, method=REDUCED, untruncated=False, chi_p=None, chi_pp=None):
    for r in MOVE_ORDER:
        env = move(env, A, B, r, chi, method, untruncated, chi_p, chi_pp)
    return env


def corner_spectra(env, chi):
    """Singular values of the 8 corners, normalised by sigma_0 and
    zero-padded to chi: dict corner -> array(chi)."""
    out = {}
    for k in CORNERS:
        s = np.linalg.svd(env[k], compute_uv=False)
        v = np.zeros(chi)
        n = min(chi, s.size)
        if s[0] > 0:
            v[:n] = s[:n] / s[0]
        out[k] = v
    return out


# ---------------------------------------------------------------- energy

def bond_energy(env, A, B, x, h2, r=0):
    """<h> on the bond between an x-site and its right neighbour y, in
    frame r (r = 0 horizontal; r = 1 is the vertical bond with x on top).
    Network: C1_x T2_x T2_y C2_y / T1_x x y T3_y / C4_x T4_x T4_y C3_y."""
    y = _other(x)
    f = frame_env(env, r)
    sites = {"a": rotate_site(A, r), "b": rotate_site(B, r)}
    Ax, Ay = sites[x], sites[y]
    d = Ax.shape[0]
    # left half -> HL[c, s1, r1, i, S1, R1]; ket absorbed before T4 so no
    # intermediate carries more than chi^2 D^4 d entries
    P = _c("ab,fkla->bfkl", f[f"C1{x}"], f[f"T1{x}"])
    P = _c("bfkl,hf->bklh", P, f[f"C4{x}"])
    P = _c("bklh,buUc->kluUch", P, f[f"T2{x}"])
    P = _c("kluUch,skurd->lhUcsrd", P, Ax)
    P = _c("lhUcsrd,idDh->lUcsriD", P, f[f"T4{x}"])
    HL = _c("lUcsriD,SlURD->csriSR", P, Ax)
    # right half -> HR[c, t, r1, i, T, R1]
    Q = _c("eg,gkKj->ekKj", f[f"C2{y}"], f[f"T3{y}"])
    Q = _c("ekKj,jn->ekKn", Q, f[f"C3{y}"])
    Q = _c("ekKn,cuUe->kKncuU", Q, f[f"T2{y}"])
    Q = _c("kKncuU,trukd->KncUtrd", Q, Ay)
    Q = _c("KncUtrd,ndDi->KcUtriD", Q, f[f"T4{y}"])
    HR = _c("KcUtriD,TRUKD->ctriTR", Q, Ay)
    rho = _c("csriSR,ctriTR->stST", HL, HR)      # [s1, s2, s1', s2']
    h4 = np.asarray(h2, dtype=np.float64).reshape(d, d, d, d)
    num = _c("stST,STst->", rho, h4)
    den = _c("stst->", rho)
    return float(num / den)


def energy(env, A, B, h2=None):
    """(e_site, [e_h(a,b), e_h(b,a), e_v(a,b), e_v(b,a)]); two bonds per site."""
    if h2 is None:
        h2 = heisenberg_h2(A.shape[0])
    eb = [bond_energy(env, A, B, "a", h2, 0), bond_energy(env, A, B, "b", h2, 0),
          bond_energy(env, A, B, "a", h2, 1), bond_energy(env, A, B, "b", h2, 1)]
    return 0.5 * sum(eb), eb


# ---------------------------------------------------------------- observables

def site_rdm(env, A, B, z):
    """One-site reduced density matrix rho[s, S] of a z-site (ket index s,
    bra index S), unnormalised: the site between its four corners and four
    edges (3 x 3 network, frame 0).  <O>_z = sum rho[s, S] O[S, s] / tr rho
    gives the order parameters of Sec. V (staggered magnetisation, m_z) and
    the transverse-field term of the Ising model."""
    X = A if z == "a" else B
    e = {k: env[f"{k}{z}"] for k in ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")}
    # left column C1 T1 C4 with the top and bottom edges, then the site
    # (ket, bra) and the right column C2 T3 C3, one pair at a time
    L = _c("ha,ilLh->ailL", e["C1"], e["T1"])
    L = _c("ailL,gi->algL", L, e["C4"])
    L = _c("algL,auUb->lgLuUb", L, e["T2"])
    L = _c("lgLuUb,fdDg->lLuUbfdD", L, e["T4"])
    L = _c("lLuUbfdD,slurd->LUbfDsr", L, X)
    L = _c("LUbfDsr,SLURD->bfsrSR", L, X)
    R = _c("bc,crRe->brRe", e["C2"], e["T3"])
    R = _c("brRe,ef->brRf", R, e["C3"])
    return _c("bfsrSR,brRf->sS", L, R)


def expect1(env, A, B, op):
    """(<op>_a, <op>_b) for a d x d one-site operator op[s', s]."""
    out = []
    for z in "ab":
        rho = site_rdm(env, A, B, z)
        out.append(float(_c("sS,Ss->", rho, op) / np.trace(rho)))
    return out


def staggered_magnetisation(env, A, B):
    """m_s = |<S>_a - <S>_b| / 2 with S = sigma / 2 (Sec. V); for real
    tensors <S^y> = 0, so only S^x and S^z enter."""
    sx = np.array([[0.0, 0.5], [0.5, 0.0]])
    sz = np.array([[0.5, 0.0], [0.0, -0.5]])
    xa, xb = expect1(env, A, B, sx)
    za, zb = expect1(env, A, B, sz)
    return 0.5 * float(np.hypot(xa - xb, za - zb))


def row_correlation(env, A, B, op, L):
    """C(x) = <op_0 op_x> - <op_0><op_x> for x = 1..L along a row (frame 0),
    site 0 on sublattice a (Sec. V, Fig. 8(b): S_zz(x)).  The row between
    the edges above (T2) and below (T4) is contracted column by column from
    the left boundary {C1, T1, C4} of site 0 to the right boundary
    {C2, T3, C3} of site x."""
    sites = {"a": A, "b": B}

    def left(z, o):
        # left boundary + site z with o on its physical legs -> V[c, r, R, f]
        X = sites[z]
        L = _c("ha,ilLh->ailL", env[f"C1{z}"], env[f"T1{z}"])
        L = _c("ailL,gi->algL", L, env[f"C4{z}"])
        L = _c("algL,auUc->lgLuUc", L, env[f"T2{z}"])
        L = _c("lgLuUc,fdDg->lLuUcfdD", L, env[f"T4{z}"])
        L = _c("lLuUcfdD,slurd->LUcfDsr", L, X)
        L = _c("LUcfDsr,Ss->LUcfDSr", L, o)
        return _c("LUcfDSr,SLURD->crRf", L, X)

    def column(V, z, o):
        # absorb the column {T2_z, z, T4_z} with o on the site: V[c, r, R, f]
        X = sites[z]
        W = _c("crRf,cuUb->rRfuUb", V, env[f"T2{z}"])
        W = _c("rRfuUb,srutd->RfUbstd", W, X)
        W = _c("RfUbstd,Ss->RfUbStd", W, o)
        W = _c("RfUbStd,SRUTD->fbtdTD", W, X)
        return _c("fbtdTD,gdDf->btTg", W, env[f"T4{z}"])

    def right(V, z, o):
        # close with site z (op o) and its right boundary {C2, T3, C3}
        W = column(V, z, o)                                  # [b, t, T, g]
        R = _c("bn,ntTe->btTe", env[f"C2{z}"], env[f"T3{z}"])
        R = _c("btTe,eg->btTg", R, env[f"C3{z}"])
        return float(_c("btTg,btTg->", W, R))

    d = A.shape[0]
    one = np.eye(d)
    VO, VI = left("a", op), left("a", one)
    out = []
    for x in range(1, L + 1):
        z = "a" if x % 2 == 0 else "b"
        oo, io = right(VO, z, op), right(VI, z, op)
        oi, ii = right(VO, z, one), right(VI, z, one)
        out.append(oo / ii - (oi / ii) * (io / ii))
        VO, VI = column(VO, z, one), column(VI, z, one)
        nrm = np.linalg.norm(VI)
        VO, VI = VO / nrm, VI / nrm
    return out


# ---------------------------------------------------------------- driver

def solve(A, B, chi, method=REDUCED, max_iters=20, tol=0.0, h2=None, env=None,
          boot_iters=0, callback=None, chi_p=None, chi_pp=None):
    """Iterate CTM until the corner-spectrum change delta < tol (or
    max_iters).  The first boot_iters iterations use the standard move
    whatever the method.  Returns dict(env, iters, delta, e_site, e_bond,
    deltas)."""
    if env is None:
        env = init_env(A, B)
    prev = corner_spectra(env, chi)
    deltas = []
    it = 0
    delta = np.inf
    while it < max_iters:
        m = STANDARD if it < boot_iters else method
        env = ctm_iteration(env, A, B, chi, m, chi_p=chi_p, chi_pp=chi_pp)
        it += 1
        cur = corner_spectra(env, chi)
        delta = max(float(np.max(np.abs(cur[k] - prev[k]))) for k in CORNERS)
        deltas.append(delta)
        prev = cur
        if callback is not None:
            callback(it, env, delta)
        if delta < tol:
            break
    e_site, e_bond = energy(env, A, B, h2)
    return {"env": env, "iters": it, "delta": delta, "e_site": e_site,
            "e_bond": e_bond, "deltas": deltas}

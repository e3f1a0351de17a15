"""Exact contraction of small finite PEPS patches (test pin, CPU only).

A patch is a W x H block of sites on the checkerboard.  Its norm network is
<psi|psi> with every dangling virtual leg on the patch border traced (ket
index = bra index, summed); two chosen sites keep their physical ket/bra
indices open so a two-site operator can be measured.  The contraction sweeps
the columns left to right, carrying one fused (ket, bra) index per row, so it
shares nothing with the corner-transfer code: no environment tensors, no
projectors, no rotations.
"""

from __future__ import annotations

import numpy as np


def _double(A, open_phys):
    """Fused double layer e[l,u,r,d] (each index k*D+b), or with open
    physical legs e[s,s',l,u,r,d]."""
    d, D = A.shape[0], A.shape[1]
    D2 = D * D
    if open_phys:
        t = np.einsum("slurd,tLURD->stlLuUrRdD", A, A)
        return t.reshape(d, d, D2, D2, D2, D2)
    t = np.einsum("slurd,sLURD->lLuUrRdD", A, A)
    return t.reshape(D2, D2, D2, D2)


def patch_rdm(sites_grid, open_sites):
    """sites_grid[r][c] is a site tensor A[s,l,u,r,d]; open_sites is a list
    of two (r, c) positions whose physical legs stay open.  Returns
    rho[s1, s2, s1', s2'] (ket indices first) for the two open sites, in
    the order given."""
    H = len(sites_grid)
    W = len(sites_grid[0])
    D = sites_grid[0][0].shape[1]
    d = sites_grid[0][0].shape[0]
    D2 = D * D
    tr = np.eye(D).reshape(D2)            # traced dangling leg
    # state: horizontal bonds h_0..h_{H-1}, then open physical pairs
    v = tr
    for _ in range(H - 1):
        v = np.multiply.outer(v, tr)
    v = v.reshape((D2,) * H)
    n_open = 0
    for c in range(W):
        # append the vertical bond as the last axis: top leg traced
        v = np.multiply.outer(v, tr)      # axes: h_0..h_{H-1}, [phys...], vert
        for r in range(H):
            A = sites_grid[r][c]
            is_open = (r, c) in open_sites
            e = _double(A, is_open)
            nd = v.ndim
            # axis of h_r is r; vertical bond is the last axis
            if is_open:
                # e[s,s',l,u,r,d]: contract l with h_r, u with vert
                v = np.tensordot(v, e, axes=([r, nd - 1], [2, 3]))
                # new axes appended: s, s', r_out, d_out
                # move r_out to position r, keep s, s' before vert
                v = np.moveaxis(v, nd - 2 + 2, r)   # r_out
                # now the tail is ..., s, s', d_out
                n_open += 1
            else:
                v = np.tensordot(v, e, axes=([r, nd - 1], [0, 1]))
                # appended: r_out, d_out
                v = np.moveaxis(v, nd - 2, r)
        # bottom leg traced
        v = np.tensordot(v, tr, axes=([v.ndim - 1], [0]))
    # right dangling legs traced
    for _ in range(H):
        v = np.tensordot(v, tr, axes=([0], [0]))
    # v axes: physical pairs in the order the open sites were met
    # (column-major sweep); reorder to the requested order
    met = sorted(open_sites, key=lambda rc: (rc[1], rc[0]))
    v = v.reshape((d, d) * len(met))
    if met[0] != open_sites[0]:
        v = v.transpose(2, 3, 0, 1)
    # v[s1, s1', s2, s2'] -> rho[s1, s2, s1', s2']
    return v.transpose(0, 2, 1, 3)


def patch_bond_energy(A, B, h2, x_is_a, orient, left, right, up, down):
    """<h> on a bond (x, y) of a finite patch.  orient 'h': y right of x;
    'v': y below x.  left/right/up/down = number of extra columns/rows of
    sites around the two-site core (the traced border included)."""
    sites = {True: A, False: B}
    if orient == "h":
        W, Hh = left + 2 + right, up + 1 + down
        xr, xc = up, left
        yr, yc = up, left + 1
    else:
        W, Hh = left + 1 + right, up + 2 + down
        xr, xc = up, left
        yr, yc = up + 1, left
    grid = []
    for r in range(Hh):
        row = []
        for c in range(W):
            same = ((r - xr) + (c - xc)) % 2 == 0
            row.append(sites[same == x_is_a])
        grid.append(row)
    rho = patch_rdm(grid, [(xr, xc), (yr, yc)])
    d = A.shape[0]
    h4 = np.asarray(h2).reshape(d, d, d, d)
    num = np.einsum("stST,STst->", rho, h4)
    den = np.einsum("stst->", rho)
    return float(num / den)

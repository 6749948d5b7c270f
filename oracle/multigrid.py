"""Multigrid transfer operators and Galerkin coarse matrices (oracle).

Paper §3.2: coarse matrices are Galerkin products J_{l+1} = P_l^T J_l P_l,
P_l is trilinear space-time interpolation and restriction is P_l^T; §3.2.1
semi-coarsens either in space (dx doubles, dt kept) or in time (dt doubles).

Readings (the paper is silent on Dirichlet nodes inside the hierarchy):
  * the prolongation is masked, P_m = N_f P, so no correction reaches a fine
    Dirichlet node;
  * a coarse node whose column of P_m is zero is Dirichlet on the coarse
    level; its row and column of P_m^T J P_m vanish and it gets an identity row.
"""
import numpy as np
import scipy.sparse as sp

from .hierarchy import SPACE, TIME, FULL


def interp_1d(n_coarse_elems):
    """Linear interpolation from n_c+1 coarse vertices to 2 n_c + 1 fine vertices."""
    nc = n_coarse_elems
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for i in range(nf + 1):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [(i - 1) // 2, (i + 1) // 2]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf + 1, nc + 1))


def prolongation(fine, how):
    """Unmasked P from the coarse level (made from `fine` by `how`) to `fine`.
    Node order (t, x2, x1) with x1 fastest, so P = kron(Pt, Py, Px)."""
    It = sp.identity(fine["nt"] + 1, format="csr")
    Iy = sp.identity(fine["ny"] + 1, format="csr")
    Ix = sp.identity(fine["nx"] + 1, format="csr")
    if how == SPACE:
        return sp.kron(It, sp.kron(interp_1d(fine["ny"] // 2), interp_1d(fine["nx"] // 2))).tocsr()
    if how == TIME:
        return sp.kron(interp_1d(fine["nt"] // 2), sp.kron(Iy, Ix)).tocsr()
    if how == FULL:
        return sp.kron(interp_1d(fine["nt"] // 2),
                       sp.kron(interp_1d(fine["ny"] // 2), interp_1d(fine["nx"] // 2))).tocsr()
    raise ValueError(how)


def masked_prolongation(P, fine_mask):
    keep = (~np.asarray(fine_mask, dtype=bool).ravel()).astype(np.float64)
    return (sp.diags(keep) @ P).tocsr()


def coarse_mask_from(Pm):
    """Coarse Dirichlet set: nodes whose column of P_m is identically zero."""
    colnorm = np.asarray(abs(Pm).sum(axis=0)).ravel()
    return colnorm == 0.0


def galerkin(A, Pm, coarse_mask):
    """P_m^T A P_m with identity rows on the coarse Dirichlet set."""
    Ac = (Pm.T @ A @ Pm).tocsr()
    cm = np.asarray(coarse_mask, dtype=bool).ravel()
    Ac = Ac + sp.diags(cm.astype(np.float64))
    return Ac.tocsr()


def build_operators(levels, J0, mask0):
    """Operators, masks and masked prolongations for every level.

    Returns lists A[l], mask[l] (bool, flat) and Pm[l] (prolongation from level
    l+1 to level l)."""
    A = [sp.csr_matrix(J0)]
    masks = [np.asarray(mask0, dtype=bool).ravel()]
    Pms = []
    for l in range(len(levels) - 1):
        P = prolongation(levels[l], levels[l + 1]["how"])
        Pm = masked_prolongation(P, masks[l])
        cm = coarse_mask_from(Pm)
        A.append(galerkin(A[l], Pm, cm))
        masks.append(cm)
        Pms.append(Pm)
    return A, masks, Pms


def stencil_of(A, level):
    """27-point stencil view of a level matrix: array [27, nt+1, ny+1, nx+1]
    where entry d = (dt+1)*9 + (dy+1)*3 + (dx+1) holds A(node, node+offset).
    Entries that would leave the grid are zero.  Raises if A couples nodes
    farther apart than one step in any direction."""
    nx, ny, nt = level["nx"], level["ny"], level["nt"]
    A = sp.coo_matrix(A)
    shp = (nt + 1, ny + 1, nx + 1)
    rn, rj, ri = np.unravel_index(A.row, shp)
    cn, cj, ci = np.unravel_index(A.col, shp)
    dn, dj, di = cn - rn, cj - rj, ci - ri
    if np.any(np.abs(dn) > 1) or np.any(np.abs(dj) > 1) or np.any(np.abs(di) > 1):
        raise ValueError("matrix is not 27-point")
    d = (dn + 1) * 9 + (dj + 1) * 3 + (di + 1)
    st = np.zeros((27,) + shp)
    np.add.at(st, (d, rn, rj, ri), A.data)
    return st

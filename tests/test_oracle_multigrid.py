"""Pins of the oracle's transfers and Galerkin operators."""
import numpy as np
import pytest

from oracle.assemble import assemble_matrix, apply_dirichlet
from oracle.grid import Grid, dirichlet_mask
from oracle.hierarchy import build_hierarchy
from oracle.multigrid import build_operators, prolongation, stencil_of, interp_1d
from oracle.residual import apply_masked

PATCH = [(0, 0.5, 0.05)]


def _setup(n, nt, time_varying, seed=0, patch=PATCH):
    g = Grid(n, n, nt, 1.0 / n, 1.0 / nt)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1e-3, 1, (nt, n, n) if time_varying else (n, n))
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    C = np.ones_like(k)
    mask = dirichlet_mask(g, patch)
    Jm, _ = apply_dirichlet(assemble_matrix(g, k, C), np.zeros(g.n_nodes), mask)
    lv = build_hierarchy(n, n, nt, 1.0 / n, 1.0 / nt, 1.0, 1e-3, 1.0, 1.0, max_coarse_nodes=100)
    A, masks, Pm = build_operators(lv, Jm, mask)
    return g, k, C, mask, lv, A, masks, Pm


def test_interp_1d_reproduces_linears():
    P = interp_1d(5)
    xc = np.linspace(0, 1, 6)
    xf = np.linspace(0, 1, 11)
    assert np.allclose(P @ (3 * xc - 1), 3 * xf - 1, atol=1e-15)


def test_prolongation_reproduces_trilinears():
    lv = dict(nx=4, ny=6, nt=8)
    for how, c in (("space", (2, 3, 8)), ("time", (4, 6, 4))):
        P = prolongation(lv, how)
        cn, cy, cx = [np.linspace(0, 1, d + 1) for d in (c[2], c[1], c[0])]
        fn, fy, fx = [np.linspace(0, 1, d + 1) for d in (8, 6, 4)]
        fc = (cn[:, None, None] * 2 + cy[None, :, None] - 3 * cx[None, None, :]).ravel()
        ff = (fn[:, None, None] * 2 + fy[None, :, None] - 3 * fx[None, None, :]).ravel()
        assert np.allclose(P @ fc, ff, atol=1e-14)


@pytest.mark.parametrize("tv", [False, True])
def test_galerkin_matrix_free_identity(tv):
    """A_{l+1} x = P_m^T (A_l (P_m x)) off the coarse Dirichlet set, with the
    level-0 product taken matrix-free from element matrices."""
    g, k, C, mask, lv, A, masks, Pm = _setup(8, 8, tv)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(A[1].shape[0])
    x[masks[1]] = 0.0
    y_mf = Pm[0].T @ apply_masked(g, k, C, mask, Pm[0] @ x)
    assert np.max(np.abs(A[1] @ x - y_mf)) < 1e-14 * np.max(np.abs(y_mf))


@pytest.mark.parametrize("tv", [False, True])
def test_galerkin_keeps_27_points(tv):
    g, k, C, mask, lv, A, masks, Pm = _setup(16, 16, tv)
    for l in range(len(lv)):
        stencil_of(A[l], lv[l])     # raises if any coupling leaves the 3x3x3 box


def test_coarse_dirichlet_sets():
    """Zero columns of P_m: after a space coarsening exactly the t = 0 plane,
    after a time coarsening exactly the nodes of a patch that survives in
    every time level (the t = 0 plane is not Dirichlet any more)."""
    g, k, C, mask, lv, A, masks, Pm = _setup(32, 32, False)
    shp = lambda L: (L["nt"] + 1, L["ny"] + 1, L["nx"] + 1)
    # level 1 made by space coarsening of a level with t0 plane + patch
    m1 = masks[1].reshape(shp(lv[1]))
    assert lv[1]["how"] == "space" and m1[0].all() and not m1[1:].any()
    # level 2 made by time coarsening of level 1 (no patch left): nothing
    assert lv[2]["how"] == "time" and not masks[2].any()
    # a hierarchy that time-coarsens the fine level keeps the patch only
    g2 = Grid(8, 8, 16, 1 / 8, 1 / 16)
    mk = dirichlet_mask(g2, PATCH + [(2, 0.5, 0.6)])
    Jm, _ = apply_dirichlet(assemble_matrix(g2, np.ones((8, 8)), np.ones((8, 8))), np.zeros(g2.n_nodes), mk)
    lvt = [dict(nx=8, ny=8, nt=16, how=None), dict(nx=8, ny=8, nt=8, how="time")]
    A2, masks2, _ = build_operators(lvt, Jm, mk)
    mc = masks2[1].reshape(9, 9, 9)
    assert not mc[0, 1:, 1:].any()               # t=0 plane interior is free
    assert mc[:, 0, :].all()                     # full-edge patch survives in all levels


def test_time_constant_interior_rows_repeat():
    """Time-constant k: on every level the stencil rows of interior time
    levels (away from the first two and the last) are identical."""
    g, k, C, mask, lv, A, masks, Pm = _setup(16, 16, False)
    for l in range(len(lv)):
        st = stencil_of(A[l], lv[l])
        nt = lv[l]["nt"]
        if nt >= 5:
            ref = st[:, 2]
            for n in range(3, nt - 1):
                assert np.max(np.abs(st[:, n] - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_level_transpose_identity():
    g, k, C, mask, lv, A, masks, Pm = _setup(8, 8, True, seed=3)
    rng = np.random.default_rng(2)
    for l in range(len(lv)):
        v, w = rng.standard_normal((2, A[l].shape[0]))
        assert abs((A[l] @ v) @ w - v @ (A[l].T @ w)) < 1e-13 * np.linalg.norm(A[l] @ v) * np.linalg.norm(w)
    for l in range(len(Pm)):
        v = rng.standard_normal(Pm[l].shape[1])
        w = rng.standard_normal(Pm[l].shape[0])
        assert abs((Pm[l] @ v) @ w - v @ (Pm[l].T @ w)) < 1e-13 * np.linalg.norm(v) * np.linalg.norm(w) * 4


@pytest.mark.parametrize("tv,full", [(False, False), (True, False), (True, True)])
def test_time_offset_blocks_are_symmetric_in_space(tv, full):
    """Every time-offset block of every Galerkin level is symmetric in space:
    A(p, p + (dn, dj, di)) = A(q, q + (dn, -dj, -di)) with q = p + (0, dj, di)
    (each slab's element matrices are k A~ + C B~ with spatial factors M, S
    that are symmetric, the prolongation is a tensor product and the Dirichlet
    set of a level is the same at every time level but the first, which is
    all identity rows).  The GPU's FP32 and BF16 stencils store 15 of the 27
    entries of a row on this basis; the mirror of a lower entry (dj < 0, or
    dj = 0 and di < 0) is its neighbour's upper one.  Also on a 16 x 12 x 16
    grid with an extra patch on another edge."""
    for (n, ny, nt, patch) in [(16, 16, 16, PATCH), (16, 12, 16, PATCH + [(3, 0.3, 0.2)])]:
        g = Grid(n, ny, nt, 1.0 / max(n, ny), 1.0 / nt)
        rng = np.random.default_rng(3)
        rho = rng.uniform(1e-3, 1, (nt, ny, n) if tv else (ny, n))
        k = 1e-3 + (1 - 1e-3) * rho ** 3
        C = 0.5 + rho
        mask = dirichlet_mask(g, patch)
        Jm, _ = apply_dirichlet(assemble_matrix(g, k, C), np.zeros(g.n_nodes), mask)
        lv = build_hierarchy(n, ny, nt, g.dx, g.dt, 1.0, 1e-3, 1.5, 0.5, max_coarse_nodes=100,
                             full=full)
        A, masks, Pm = build_operators(lv, Jm, mask)
        assert len(lv) >= 3
        for l in range(len(lv)):
            st = stencil_of(A[l], lv[l])          # [27, nt+1, ny+1, nx+1]
            L = lv[l]
            scale = np.max(np.abs(st))
            checked = 0
            for dn in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        d = (dn + 1) * 9 + (dj + 1) * 3 + (di + 1)
                        dm = (dn + 1) * 9 + (-dj + 1) * 3 + (-di + 1)
                        # rows p whose neighbour q = p + (0, dj, di) exists
                        j0, j1 = max(0, -dj), L["ny"] + 1 - max(0, dj)
                        i0, i1 = max(0, -di), L["nx"] + 1 - max(0, di)
                        a = st[d][:, j0:j1, i0:i1]
                        b = st[dm][:, j0 + dj:j1 + dj, i0 + di:i1 + di]
                        assert np.max(np.abs(a - b)) <= 1e-14 * scale, (l, dn, dj, di)
                        checked += a.size
            assert checked > 0

"""GPU parity of the single operators against the FP64 oracle (element by
element): fine matrix-free apply and transpose, diagonal, Galerkin stencils of
every level, masks, transfers, coarse applies, FP32 variants, one smoothing and
one V-cycle."""
import numpy as np
import pytest

from oracle.krylov import gmres_jacobi, VCycle
from oracle.multigrid import stencil_of
from tests._cases import Case, rel, maxrel

pytestmark = pytest.mark.gpu

# (64 q + 1 node columns -- nx = 64, 128 -- take the 65-wide last tile column)
SHAPES = [(3, 2, 2, False), (3, 2, 2, True), (8, 6, 5, True), (12, 12, 8, False),
          (32, 32, 32, False), (16, 16, 16, True), (64, 20, 6, True), (128, 9, 5, False)]


def _t(x):
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def torch_cuda(require_gpu):
    import torch
    return torch


@pytest.mark.parametrize("nx,ny,nt,tv", SHAPES)
def test_fine_apply_and_transpose(torch_cuda, nx, ny, nt, tv):
    c = Case(nx, ny, nt, tv=tv, seed=nx + nt, patches=((0, 0.5 * ny / max(nx, ny), 0.3),))
    p = c.problem(max_coarse_nodes=10 ** 9)
    rng = np.random.default_rng(1)
    shp = (nt + 1, ny + 1, nx + 1)
    for trans in (False, True):
        x = rng.standard_normal(shp)
        y = p.debug_apply(0, _t(x), transpose=trans).cpu().numpy()
        ref = (c.Jm.T if trans else c.Jm) @ x.ravel()
        assert maxrel(y, ref) < 1e-13, (trans, maxrel(y, ref))
    p.close()
    # the FP32 apply of the V-cycle (same tiling)
    p = c.problem(max_coarse_nodes=10 ** 9, precision="mixed")
    for trans in (False, True):
        x = rng.standard_normal(shp)
        y = p.debug_apply(0, _t(x), transpose=trans, mixed=True).cpu().numpy()
        ref = (c.Jm.T if trans else c.Jm) @ x.ravel()
        assert rel(y, ref) < 1e-5, (trans, rel(y, ref))
    p.close()


@pytest.mark.parametrize("nx,ny,nt,tv", SHAPES)
def test_fine_diagonal_mask_and_stencil(torch_cuda, nx, ny, nt, tv):
    c = Case(nx, ny, nt, tv=tv, seed=3, patches=((0, 0.5 * ny / max(nx, ny), 0.3), (3, 0.4, 0.2)))
    p = c.problem(max_coarse_nodes=10 ** 9)
    invd, m = p.debug_diag(0)
    assert np.array_equal(m.cpu().numpy().astype(bool).ravel(), c.mask.ravel())
    assert maxrel(invd.cpu().numpy(), 1.0 / c.Jm.diagonal()) < 1e-14
    st = p.debug_stencil(0).cpu().numpy()
    ref = stencil_of(c.Jm, c.levels[0])
    assert maxrel(st, ref) < 1e-13
    p.close()


@pytest.mark.parametrize("nx,ny,nt,tv,full", [(16, 16, 16, False, False), (16, 16, 16, True, False),
                                              (16, 12, 8, True, False), (32, 32, 32, False, False),
                                              (16, 16, 16, True, True), (16, 12, 8, False, True),
                                              (24, 20, 12, True, True)])
def test_galerkin_hierarchy(torch_cuda, nx, ny, nt, tv, full):
    """Every coarse level: mask, stencil (P_m^T A P_m with identity rows),
    inverse diagonal; and the transfers on every level pair (semi-coarsening
    by Algorithm 1, or full space-time coarsening)."""
    c = Case(nx, ny, nt, tv=tv, seed=5, max_coarse_nodes=200, full=full)
    p = c.problem(max_coarse_nodes=200)
    if full:
        assert all(L["how"] == "full" for L in c.levels[1:]) and len(c.levels) > 1
    dims, planes = p.hierarchy()
    assert [(L["nx"], L["ny"], L["nt"]) for L in c.levels] == [tuple(d) for d in dims]
    A, masks, Pm = c.ops
    rng = np.random.default_rng(2)
    for l in range(1, len(dims)):
        invd, m = p.debug_diag(l)
        assert np.array_equal(m.cpu().numpy().astype(bool).ravel(), masks[l]), l
        st = p.debug_stencil(l).cpu().numpy()
        ref = stencil_of(A[l], c.levels[l])
        assert maxrel(st, ref) < 1e-13, (l, maxrel(st, ref))
        assert maxrel(invd.cpu().numpy(), 1.0 / A[l].diagonal()) < 1e-13
        if not tv:
            assert planes[l] <= 8, planes
        # transfers
        xc = rng.standard_normal(A[l].shape[0])
        xf = rng.standard_normal(A[l - 1].shape[0])
        pro = p.debug_transfer(l - 1, _t(xc).reshape(p.level_shape(l)), prolong=True).cpu().numpy()
        res = p.debug_transfer(l - 1, _t(xf).reshape(p.level_shape(l - 1)), prolong=False).cpu().numpy()
        assert maxrel(pro, Pm[l - 1] @ xc) < 1e-15
        assert maxrel(res, Pm[l - 1].T @ xf) < 1e-14
        # coarse apply and transpose
        for trans in (False, True):
            y = p.debug_apply(l, _t(xc).reshape(p.level_shape(l)), transpose=trans).cpu().numpy()
            ref = (A[l].T if trans else A[l]) @ xc
            assert maxrel(y, ref) < 1e-13, (l, trans)
    p.close()


def _bf16_round(a):
    """FP64 -> FP32 -> BF16 (round to nearest even on the upper 16 bits), the
    storage rounding of BF16 coarse stencils, back as FP64."""
    u = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_reference():
    """The test's BF16 rounding: exact for BF16 values, ties to even."""
    # BF16 keeps 8 significant bits: the spacing at 1 is 2^-7
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9,
                     1.0 + 3 * 2.0 ** -9, -2.5, 0.0])
    assert np.array_equal(_bf16_round(vals), [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0, 1.0 + 2.0 ** -7,
                                              -2.5, 0.0])


def _bf16_compensated(A, P, by_column):
    """The BF16 storage model of a coarse operator: every entry rounded to
    BF16 except the in-plane centre of each time offset (the entry coupling a
    node to itself at time offset dn), which instead takes the exact sum of
    its group minus the rounded rest.  The group is a row's entries of one
    time offset (forward apply) or a column's (by_column, transposed apply),
    so those sums survive the rounding exactly.  The GPU stores the
    symmetric half of each time-offset block and reads a lower entry from the
    neighbouring row's upper one: the same numbers, to rounding of the FP64
    Galerkin product, so this model covers that storage too."""
    import scipy.sparse as sp
    C = sp.coo_matrix(A)
    i, j, v = C.row, C.col, C.data
    dn = j // P - i // P
    centre = (j % P) == (i % P)
    key = (j if by_column else i) * 3 + (dn + 1)
    n = A.shape[0]
    exact = np.zeros(3 * n)
    rounded = np.zeros(3 * n)
    np.add.at(exact, key, v)
    np.add.at(rounded, key[~centre], _bf16_round(v[~centre]))
    used = np.zeros(3 * n, dtype=bool)
    used[key] = True
    k = np.nonzero(used)[0]
    node, g = k // 3, k % 3 - 1          # g = time of the column - time of the row
    ci, cj = (node - g * P, node) if by_column else (node, node + g * P)
    keep = ~centre
    rows = np.concatenate([i[keep], ci])
    cols = np.concatenate([j[keep], cj])
    vals = np.concatenate([_bf16_round(v[keep]), exact[k] - rounded[k]])
    return sp.csr_matrix((vals, (rows, cols)), shape=A.shape)


@pytest.mark.parametrize("tv", [False, True])
def test_bf16_stencil_applies(torch_cuda, tv):
    """Levels >= 1 stored in BF16: the apply equals the oracle operator under
    the BF16 storage model (off-centre entries rounded, compensated FP32
    centres), to FP32 accuracy (1e-5), forward and transposed; and the
    compensation keeps the action on fields constant in space exact to FP32
    rounding, where plain BF16 rounding is off by about 1e-3."""
    import scipy.sparse as sp
    c = Case(16, 16, 16, tv=tv, seed=17, max_coarse_nodes=200)
    p = c.problem(max_coarse_nodes=200, precision="mixed", bf16_from_level=1)
    A, masks, Pm = c.ops
    rng = np.random.default_rng(6)
    for l in range(1, len(c.levels)):
        Al = sp.csr_matrix(A[l])
        P = (c.levels[l]["nx"] + 1) * (c.levels[l]["ny"] + 1)
        nt1 = Al.shape[0] // P
        x = rng.standard_normal(Al.shape[0])
        xt = np.repeat(rng.standard_normal(nt1), P)          # constant in space
        for trans in (False, True):
            Ab = _bf16_compensated(Al, P, by_column=trans)
            for v in (x, xt):
                y = p.debug_apply(l, _t(v).reshape(p.level_shape(l)), transpose=trans, mixed=True)
                ref = (Ab.T if trans else Ab) @ v
                assert rel(y.cpu().numpy(), ref) < 1e-5, (l, trans, rel(y.cpu().numpy(), ref))
            exact = (Al.T if trans else Al) @ xt
            y = p.debug_apply(l, _t(xt).reshape(p.level_shape(l)), transpose=trans, mixed=True)
            assert np.max(np.abs(y.cpu().numpy().ravel() - exact)) <= 1e-5 * np.max(np.abs(Al.data)) * \
                np.max(np.abs(xt))
            # distance of the BF16 operator from the exact FP64 one on a random
            # vector: the stated bound for BF16 coarse levels is 1e-2 (2-norm)
            y = p.debug_apply(l, _t(x).reshape(p.level_shape(l)), transpose=trans, mixed=True)
            d = rel(y.cpu().numpy(), (Al.T if trans else Al) @ x)
            print(f"level {l} trans={trans}: BF16 apply vs exact {d:.2e}", flush=True)
            assert d <= 1e-2, (l, trans, d)
    p.close()


@pytest.mark.parametrize("tv", [False, True])
def test_mixed_precision_applies(torch_cuda, tv):
    """FP32 level operators (mixed precision) against the FP64 oracle: 1e-5."""
    c = Case(16, 16, 16, tv=tv, seed=7, max_coarse_nodes=200)
    p = c.problem(max_coarse_nodes=200, precision="mixed")
    A, masks, Pm = c.ops
    rng = np.random.default_rng(3)
    for l in range(len(c.levels)):
        x = rng.standard_normal(A[l].shape[0])
        for trans in (False, True):
            y = p.debug_apply(l, _t(x).reshape(p.level_shape(l)), transpose=trans, mixed=True)
            ref = (A[l].T if trans else A[l]) @ x
            assert rel(y.cpu().numpy(), ref) < 1e-5, (l, trans, rel(y.cpu().numpy(), ref))
    p.close()


@pytest.mark.parametrize("tv,prec", [(False, "fp32"), (True, "fp32"), (True, "bf16"), (False, "fp64"),
                                     (True, "fp64")])
def test_stencil_apply_wide_planes(torch_cuda, tv, prec):
    """Coarse applies on planes that span several 64-lane waves (a node's
    in-plane neighbours come from the lanes beside it, 62 outputs per wave):
    planes of 713 and 192 nodes (11 full waves and a ragged one; rows 31 and
    16 nodes wide, so waves cross row ends), 71 and 36 time levels (chunks of
    four with a ragged last one).  Forward and transposed against the oracle
    operator -- under the BF16 storage model for BF16 -- to 1e-5 in FP32 and
    BF16 storage and 1e-13 in FP64, on a random field and on a field that is
    non-zero on one node only (every neighbour coefficient of that column in
    place).  The same with ST_FLAG_ROW_MARCH, the row-march kernel that the
    library takes for levels past 2 GiB."""
    import scipy.sparse as sp
    from paper_2508_09589_amd import _lib as Lb
    c = Case(60, 44, 70, tv=tv, seed=21)
    fp64 = prec == "fp64"
    p = c.problem(precision="fp64" if fp64 else "mixed", bf16_from_level=1 if prec == "bf16" else 0)
    A, masks, Pm = c.ops
    rng = np.random.default_rng(8)
    assert len(c.levels) >= 4
    flags0 = p.opts.flags
    for march, l in [(m, l) for m in (False, True) for l in range(1, len(c.levels))]:
        p.set_flags(flags0 | (Lb.ST_FLAG_ROW_MARCH if march else 0))
        Al = sp.csr_matrix(A[l])
        P = (c.levels[l]["nx"] + 1) * (c.levels[l]["ny"] + 1)
        x = rng.standard_normal(Al.shape[0])
        e = np.zeros(Al.shape[0])
        e[(c.levels[l]["nt"] // 2) * P + P // 2 + 7] = 1.0
        for trans in (False, True):
            Ab = _bf16_compensated(Al, P, by_column=trans) if prec == "bf16" else Al
            for v in (x, e):
                y = p.debug_apply(l, _t(v).reshape(p.level_shape(l)), transpose=trans,
                                  mixed=not fp64).cpu().numpy()
                ref = (Ab.T if trans else Ab) @ v
                if fp64:
                    assert maxrel(y, ref) < 1e-13, (l, march, trans, maxrel(y, ref))
                else:
                    assert rel(y, ref) < 1e-5, (l, march, trans, rel(y, ref))
    p.close()


@pytest.mark.parametrize("level", [0, 1, 2])
def test_smoother_matches_oracle_gmres(torch_cuda, level):
    """One Jacobi-GMRES smoothing (10 iterations, CGS, left Jacobi) on a level,
    from zero and from a given x0, forward and transposed."""
    c = Case(16, 16, 16, tv=True, seed=9, max_coarse_nodes=200)
    p = c.problem(max_coarse_nodes=200)
    A, masks, Pm = c.ops
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A[level].shape[0])
    b[masks[level]] = 0.0
    x0 = rng.standard_normal(A[level].shape[0]) * 0.1
    shp = p.level_shape(level)
    for trans in (False, True):
        Al = A[level].T.tocsr() if trans else A[level]
        xg = p.debug_smooth(level, _t(b).reshape(shp), None, 10, 1e-6, trans).cpu().numpy()
        xo, _, _ = gmres_jacobi(Al, b, None, 10, 1e-6)
        assert rel(xg, xo) < 1e-10, (trans, rel(xg, xo))
        xg = p.debug_smooth(level, _t(b).reshape(shp), _t(x0).reshape(shp), 10, 1e-6, trans).cpu().numpy()
        xo, _, _ = gmres_jacobi(Al, b, x0, 10, 1e-6)
        assert rel(xg, xo) < 1e-10, (trans, rel(xg, xo))
    p.close()


@pytest.mark.parametrize("level", [0, 1, 2])
def test_sstep_smoother_matches_oracle(torch_cuda, level):
    """One smoothing in s-step form (10 monomial Krylov vectors, Gram matrix,
    scaled normal equations) on a level, from zero and from x0, forward and
    transposed: the preconditioned residual it reaches is the minimum that
    Arnoldi GMRES reaches over the same space (1e-7 relative: the minimum is
    a well-conditioned quantity), while x itself agrees with the oracle's
    s-step smoother only as far as the conditioning of the monomial Gram
    matrix allows (about 2e-5 measured here; bound 1e-3)."""
    from oracle.krylov import gmres_jacobi_sstep
    c = Case(16, 16, 16, tv=True, seed=9, max_coarse_nodes=200)
    p = c.problem(max_coarse_nodes=200, smoother="sstep")
    A, masks, Pm = c.ops
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A[level].shape[0])
    b[masks[level]] = 0.0
    x0 = rng.standard_normal(A[level].shape[0]) * 0.1
    shp = p.level_shape(level)
    for trans in (False, True):
        Al = A[level].T.tocsr() if trans else A[level]
        dinv = 1.0 / Al.diagonal()
        for start in (None, x0):
            xg = p.debug_smooth(level, _t(b).reshape(shp),
                                None if start is None else _t(start).reshape(shp), 10, 1e-6,
                                trans).cpu().numpy().ravel()
            xa, _, _ = gmres_jacobi(Al, b, start, 10, 1e-6)
            xs, _, _ = gmres_jacobi_sstep(Al, b, start, 10, 1e-6)
            ra = np.linalg.norm(dinv * (b - Al @ xa))
            rg = np.linalg.norm(dinv * (b - Al @ xg))
            assert abs(rg - ra) <= 1e-7 * ra, (trans, rg, ra)
            assert rel(xg, xs) < 1e-3, (trans, rel(xg, xs))
    p.close()


@pytest.mark.parametrize("its,tol", [(1, 1e-12), (2, 1e-11), (10, 1e-7), (15, 1e-10)])
def test_sstep_smoother_basis_sizes(torch_cuda, its, tol):
    """The smallest and largest s-step bases (2 and 11 vectors): the residual
    reached is Arnoldi GMRES's minimum; 15 iterations are beyond the monomial
    basis and take the Arnoldi form (so match Arnoldi to rounding); a zero
    right-hand side from a zero start gives exactly zero."""
    c = Case(12, 12, 8, tv=True, seed=13, max_coarse_nodes=200)
    p = c.problem(max_coarse_nodes=200, smoother="sstep")
    A, masks, Pm = c.ops
    rng = np.random.default_rng(3)
    level = 1
    b = rng.standard_normal(A[level].shape[0])
    b[masks[level]] = 0.0
    shp = p.level_shape(level)
    Al = A[level]
    dinv = 1.0 / Al.diagonal()
    xg = p.debug_smooth(level, _t(b).reshape(shp), None, its, 0.0).cpu().numpy().ravel()
    xa, ia, _ = gmres_jacobi(Al, b, None, its, 0.0)
    assert ia == its
    ra = np.linalg.norm(dinv * (b - Al @ xa))
    rg = np.linalg.norm(dinv * (b - Al @ xg))
    assert abs(rg - ra) <= tol * ra, (its, rg, ra)
    z = p.debug_smooth(level, _t(np.zeros_like(b)).reshape(shp), None, its, 1e-6).cpu().numpy()
    assert np.all(z == 0.0)
    p.close()


@pytest.mark.parametrize("tv", [False, True])
@pytest.mark.parametrize("coarse,full", [("gmres", False), ("direct", False), ("direct", True)])
def test_vcycle_matches_oracle(torch_cuda, tv, coarse, full):
    c = Case(16, 16, 16, tv=tv, seed=11, max_coarse_nodes=200, full=full)
    p = c.problem(max_coarse_nodes=200, coarse=coarse)
    A, masks, Pm = c.ops
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A[0].shape[0])
    b[masks[0]] = 0.0
    for trans in (False, True):
        At = [a.T.tocsr() for a in A] if trans else A
        xo = VCycle(At, Pm, coarse=coarse)(b)
        xg = p.debug_vcycle(_t(b).reshape(p.level_shape(0)), transpose=trans).cpu().numpy()
        assert rel(xg, xo) < 1e-9, (trans, rel(xg, xo))
    p.close()


@pytest.mark.parametrize("nx,ny,nt,tv", [(8, 8, 16, True), (5, 7, 3, False), (12, 12, 4, True),
                                         (1, 1, 1, False), (3, 2, 9, True), (16, 16, 8, False),
                                         (17, 16, 5, True), (24, 20, 6, True), (32, 32, 3, False),
                                         (8, 8, 40, True)])
def test_direct_coarse_solve_is_exact(torch_cuda, nx, ny, nt, tv):
    """A one-level hierarchy makes the V-cycle the coarsest-level solve: the
    block-tridiagonal factorisation must reproduce the oracle's direct solve,
    forward and transposed.  Planes of at most 128 nodes with at most 3072
    nodes in all take the one-workgroup factorisation and the LDS-resident
    solve; the others (169, 289, 306, 525 and 1089-node planes, and 81-node
    planes over 41 levels) the wide factorisation (blocked Gauss-Jordan, the
    panel in LDS up to 481 nodes, in global memory above; panels of 16
    columns with a short last one) and the multi-workgroup sweeps."""
    from oracle.solve import solve_direct, solve_adjoint_direct
    c = Case(nx, ny, nt, tv=tv, seed=nx + 3 * ny + 7 * nt,
             patches=((0, 0.5 * ny / max(nx, ny), 0.2), (3, 0.4, 0.3)))
    p = c.problem(max_levels=1)
    assert p.hierarchy()[0] == [(nx, ny, nt)]
    rng = np.random.default_rng(8)
    b = rng.standard_normal(c.Jm.shape[0])
    shp = p.level_shape(0)
    xg = p.debug_vcycle(_t(b).reshape(shp), transpose=False).cpu().numpy()
    assert rel(xg, solve_direct(c.Jm, b)) < 1e-11
    xg = p.debug_vcycle(_t(b).reshape(shp), transpose=True).cpu().numpy()
    import scipy.sparse as sp
    assert rel(xg, solve_direct(sp.csr_matrix(c.Jm.T), b)) < 1e-11
    p.close()


@pytest.mark.parametrize("n,nt,design", [(32, 128, "random"), (32, 256, "sink"), (16, 512, "random")])
def test_wide_coarse_solve_is_exact_at_size(torch_cuda, n, nt, design):
    """The wide factorisation and sweeps at the sizes the 8-level hierarchies
    reach (33^2-node planes over 129 and 257 time levels, 17^2 over 513): on a
    one-level hierarchy the V-cycle is the exact solve, so its residual under
    the matrix-free fine operator (itself checked against the oracle) is at
    rounding level, forward and transposed."""
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import heat_sink_density
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.001, 1, (nt, n, n)) if design == "random" else heat_sink_density(n)
    p = Problem(n, n, nt, torch.tensor(rho), max_levels=1)
    shp = p.level_shape(0)
    for trans in (False, True):
        b = torch.tensor(rng.standard_normal(shp), device="cuda")
        x = p.debug_vcycle(b, transpose=trans)
        r = b - p.debug_apply(0, x, transpose=trans)
        assert float(r.norm() / b.norm()) < 1e-13, (trans, float(r.norm() / b.norm()))
    p.close()

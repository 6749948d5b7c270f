"""Pins of the oracle's Krylov solvers, filter and adjoint gradient."""
import numpy as np
import pytest

from oracle.assemble import Material, assemble_matrix, apply_dirichlet, load_vector
from oracle.design import filter_apply, filter_operators, objective_and_gradient
from oracle.grid import Grid, dirichlet_mask
from oracle.hierarchy import build_hierarchy
from oracle.krylov import gmres_jacobi, fgmres, VCycle
from oracle.multigrid import build_operators
from oracle.solve import solve_direct

PATCH = [(0, 0.5, 0.05)]
MAT = Material()


def _system(n, nt, seed=0, tv=False):
    g = Grid(n, n, nt, 1.0 / n, 1.0 / nt)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1e-3, 1, (nt, n, n) if tv else (n, n))
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    mask = dirichlet_mask(g, PATCH)
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0), mask)
    return g, Jm, fm, mask


@pytest.mark.parametrize("kit", [1, 3, 6])
def test_gmres_minimises_over_krylov_space(kit):
    """k steps of left-Jacobi GMRES from x0 give the minimiser of
    ||D^-1 (b - A x)|| over x0 + span{r, (D^-1 A) r, ...} (explicit basis)."""
    g, A, b, _ = _system(4, 4, seed=1)
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(b.size) * 0.01
    dinv = 1.0 / A.diagonal()
    x, its, _ = gmres_jacobi(A, b, x0, maxit=kit, rtol=0.0, dinv=dinv)
    assert its == kit
    B = dinv[:, None] * A.toarray()
    r = dinv * (b - A @ x0)
    K = [r]
    for _ in range(kit - 1):
        K.append(B @ K[-1])
    Q, _ = np.linalg.qr(np.array(K).T)
    y, *_ = np.linalg.lstsq(B @ Q, r, rcond=None)
    x_ls = x0 + Q @ y
    assert np.linalg.norm(x - x_ls) <= 1e-10 * np.linalg.norm(x_ls)


def test_gmres_restarted_reaches_exact_solution():
    g, A, b, _ = _system(4, 4, seed=3)
    x, its, est = gmres_jacobi(A, b, None, maxit=400, rtol=1e-13, restart=30)
    xs = solve_direct(A, b)
    assert est <= 1e-13 and its < 400
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_fgmres_exact_preconditioner_one_step():
    g, A, b, _ = _system(4, 4, seed=4)
    import scipy.sparse.linalg as spla
    lu = spla.splu(A.tocsc())
    x, its, rel = fgmres(A, b, lu.solve, m=5, rtol=1e-12)
    assert its == 1 and rel < 1e-12


def test_fgmres_vcycle_matches_direct_small_workload():
    """FGMRES(30) + V-cycle on the small workload converges to the direct
    solution; the iteration count stays in a small band (sanity, not a gate)."""
    from paper_2508_09589_amd.inputs import uniform_density
    rho = uniform_density(32, seed=0)
    g = Grid(32, 32, 32, 1 / 32, 1 / 32)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    mask = dirichlet_mask(g, PATCH)
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0), mask)
    lv = build_hierarchy(32, 32, 32, 1 / 32, 1 / 32, 1.0, 1e-3, 1.0, 1.0)
    A, masks, Pm = build_operators(lv, Jm, mask)
    x, its, rel = fgmres(Jm, fm, VCycle(A, Pm), m=30, rtol=1e-10)
    xs = solve_direct(Jm, fm)
    assert rel <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert 2 <= its <= 25


def test_filter_preserves_constants_and_is_symmetric():
    for shape in [(3, 4, 5), (4, 5)]:
        one = np.ones(shape)
        assert np.max(np.abs(filter_apply(one, 0.2, 0.3, 0.3, 0.45) - 1.0)) < 1e-13
    shape = (3, 3, 4)
    n = int(np.prod(shape))
    F = np.zeros((n, n))
    for e in range(n):
        u = np.zeros(n); u[e] = 1.0
        F[:, e] = filter_apply(u.reshape(shape), 0.25, 0.5, 0.375, 0.75).ravel()
    assert np.max(np.abs(F - F.T)) < 1e-14


def test_time_constant_filter_equals_filter_of_extrusion():
    rng = np.random.default_rng(5)
    g2 = rng.uniform(0, 1, (5, 6))
    f2 = filter_apply(g2, 0.2, 0.1, 0.3, 0.15)
    f3 = filter_apply(np.broadcast_to(g2, (4, 5, 6)).copy(), 0.2, 0.1, 0.3, 0.15)
    assert np.max(np.abs(f3 - f2[None])) < 1e-13


@pytest.mark.parametrize("tv,filt", [(True, 1.5), (False, None), (False, 1.5)])
def test_adjoint_gradient_matches_central_differences(tv, filt):
    """dJ/drho from the adjoint chain equals the central difference (h = 1e-6)
    of J = f^T s on a 6x6x5 grid to 1e-7 relative (difference-system form),
    and the naive two-solve central difference at h = 1e-4 to 1e-4."""
    from oracle.design import central_difference
    nx, nt = 6, 5
    g = Grid(nx, nx, nt, 1 / 6, 0.2)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.1, 0.9, (nt, nx, nx) if tv else (nx, nx))
    out = objective_and_gradient(g, MAT, rho, PATCH, 1.0, filt)
    idx = rng.choice(rho.size, 5, replace=False)
    for e in idx:
        ad = out["grad"].ravel()[e]
        fd = central_difference(g, MAT, rho, PATCH, e, 1e-6, 1.0, filt)
        assert abs(fd - ad) <= 1e-7 * abs(ad), (e, fd, ad)
        h = 1e-4
        rp = rho.copy().ravel(); rp[e] += h
        rm = rho.copy().ravel(); rm[e] -= h
        Jp = objective_and_gradient(g, MAT, rp.reshape(rho.shape), PATCH, 1.0, filt, False)["J"]
        Jn = objective_and_gradient(g, MAT, rm.reshape(rho.shape), PATCH, 1.0, filt, False)["J"]
        assert abs((Jp - Jn) / (2 * h) - ad) <= 1e-4 * abs(ad)


def test_filter_cg_route_equals_lu():
    rng = np.random.default_rng(9)
    g = rng.uniform(0, 1, (6, 9, 8))
    a = filter_apply(g, 0.125, 0.1, 0.19, 0.15, method="lu")
    b = filter_apply(g, 0.125, 0.1, 0.19, 0.15, method="cg")
    assert np.max(np.abs(a - b)) < 1e-12


def test_block_gradient_route_equals_direct():
    """The block-in-time gradient chain used for large fixtures equals the
    global-LU chain."""
    from oracle.blockgrad import objective_and_gradient_blocks
    nx, nt = 8, 6
    g = Grid(nx, nx, nt, 1 / 8, 1 / 6)
    rng = np.random.default_rng(10)
    rho = rng.uniform(0.1, 0.9, (nt, nx, nx))
    a = objective_and_gradient(g, MAT, rho, PATCH, 1.0, 1.5)
    b = objective_and_gradient_blocks(g, MAT, rho, PATCH, 1.0, 1.5)
    assert abs(a["J"] - b["J"]) < 1e-13 * abs(a["J"])
    assert np.max(np.abs(a["grad"] - b["grad"])) < 1e-11 * np.max(np.abs(a["grad"]))


@pytest.mark.parametrize("trans", [False, True])
def test_direct_coarse_vcycle_one_level_is_exact(trans):
    """With one level the V-cycle is the coarsest-level solve: the exact
    variant leaves no residual."""
    g, A, b, mask = _system(6, 5, seed=7, tv=True)
    At = A.T.tocsr() if trans else A
    x = VCycle([At], [], coarse="direct")(b)
    assert np.linalg.norm(b - At @ x) <= 1e-13 * np.linalg.norm(b)


def test_direct_coarse_two_grid_galerkin_orthogonality():
    """Without smoothing, a two-level cycle with an exact coarse solve is the
    Galerkin correction x = P A_c^-1 P^T b, whose residual is orthogonal to
    range(P): P^T (b - A x) = 0."""
    g, A, b, mask = _system(8, 8, seed=3, tv=True)
    lv = build_hierarchy(8, 8, 8, 1 / 8, 1 / 8, 1.0, 1e-3, 1.0, 1.0, n_levels=2)
    As, masks, Pm = build_operators(lv, A, mask)
    x = VCycle(As, Pm, smooth_its=0, coarse="direct")(b)
    assert np.linalg.norm(Pm[0].T @ (b - A @ x)) <= 1e-13 * np.linalg.norm(Pm[0].T @ b)
    assert np.linalg.norm(x) > 0


def _two_level(n=8, nt=8, seed=3):
    g, A, b, mask = _system(n, nt, seed=seed, tv=True)
    lv = build_hierarchy(n, n, nt, 1 / n, 1 / nt, 1.0, 1e-3, 1.0, 1.0, n_levels=2)
    As, masks, Pm = build_operators(lv, A, mask)
    return A, b, As, Pm


@pytest.mark.parametrize("smoother", ["gmres", "sstep"])
def test_vcycle_restricts_the_residual_of_the_presmoothed_iterate(smoother):
    """Pre-smoothing only, exact coarse solve: the coarse correction makes the
    residual of the returned iterate orthogonal to range(P_m),
    P_m^T (b - A x) = 0.  Restricting b instead of b - A x_pre, or dropping
    x_pre from the corrected iterate, leaves P_m^T A x_pre != 0 there."""
    A, b, As, Pm = _two_level()
    x = VCycle(As, Pm, coarse="direct", smoother=smoother, pre_its=3, post_its=0)(b)
    nb = np.linalg.norm(Pm[0].T @ b)
    assert np.linalg.norm(Pm[0].T @ (b - A @ x)) <= 1e-12 * nb
    # the pre-smoothed part is really there: the cycle differs from the bare
    # Galerkin correction
    import scipy.sparse.linalg as spla
    x_gal = Pm[0] @ spla.spsolve(As[1].tocsc(), Pm[0].T @ b)
    assert np.linalg.norm(x - x_gal) > 1e-3 * np.linalg.norm(x_gal)


def test_vcycle_with_converged_presmoothing_returns_the_solution():
    """Pre-smoothing run to convergence (rtol 1e-14, as many iterations as
    unknowns) and no post-smoothing: the residual restricted to the coarse
    level is zero, the correction vanishes and the cycle returns A^-1 b."""
    A, b, As, Pm = _two_level(n=4, nt=4, seed=5)
    x = VCycle(As, Pm, smooth_rtol=1e-14, coarse="direct", pre_its=A.shape[0], post_its=0)(b)
    xs = solve_direct(A, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("trans", [False, True])
def test_vcycle_post_smooths_from_the_corrected_iterate(trans):
    """No pre-smoothing, exact coarse solve, one post-smoothing iteration:
    the cycle returns x_cc + alpha D^-1 (b - A x_cc) with x_cc = P_m A_c^-1
    P_m^T b the Galerkin correction (one GMRES step from x_cc searches the
    direction of the preconditioned residual).  A post-smoothing from zero
    would move along D^-1 b instead."""
    import scipy.sparse.linalg as spla
    A, b, As, Pm = _two_level(seed=4)
    if trans:
        As = [a.T.tocsr() for a in As]
        A = As[0]
    x = VCycle(As, Pm, coarse="direct", pre_its=0, post_its=1)(b)
    x_cc = Pm[0] @ spla.spsolve(As[1].tocsc(), Pm[0].T @ b)
    v = (b - A @ x_cc) / A.diagonal()
    u = x - x_cc
    cos = abs(u @ v) / (np.linalg.norm(u) * np.linalg.norm(v))
    assert np.linalg.norm(u) > 0 and abs(1.0 - cos) <= 1e-12


def test_vcycle_recursion_without_smoothing_is_nested_galerkin():
    """Three levels, no smoothing, exact coarsest solve: the cycle is
    P_0 P_1 A_2^-1 P_1^T P_0^T b (each level passes its restricted residual
    down and adds the prolonged correction to its own iterate)."""
    import scipy.sparse.linalg as spla
    g, A, b, mask = _system(8, 8, seed=6, tv=True)
    lv = build_hierarchy(8, 8, 8, 1 / 8, 1 / 8, 1.0, 1e-3, 1.0, 1.0, n_levels=3)
    As, masks, Pm = build_operators(lv, A, mask)
    x = VCycle(As, Pm, coarse="direct", pre_its=0, post_its=0)(b)
    ref = Pm[0] @ (Pm[1] @ spla.spsolve(As[2].tocsc(), Pm[1].T @ (Pm[0].T @ b)))
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_fgmres_direct_coarse_matches_direct_solution():
    """The exact coarse solve changes neither the converged solution nor (on
    the small workload) the outer iteration count by more than one."""
    from paper_2508_09589_amd.inputs import uniform_density
    rho = uniform_density(32, seed=0)
    g = Grid(32, 32, 32, 1 / 32, 1 / 32)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    mask = dirichlet_mask(g, PATCH)
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0), mask)
    lv = build_hierarchy(32, 32, 32, 1 / 32, 1 / 32, 1.0, 1e-3, 1.0, 1.0)
    A, masks, Pm = build_operators(lv, Jm, mask)
    x1, its1, rel1 = fgmres(Jm, fm, VCycle(A, Pm), m=30, rtol=1e-10)
    x2, its2, rel2 = fgmres(Jm, fm, VCycle(A, Pm, coarse="direct"), m=30, rtol=1e-10)
    xs = solve_direct(Jm, fm)
    assert rel2 <= 1e-10
    assert np.linalg.norm(x2 - xs) <= 1e-8 * np.linalg.norm(xs)
    assert abs(its1 - its2) <= 1


@pytest.mark.parametrize("kit", [1, 3, 6])
def test_sstep_smoother_minimises_over_krylov_space(kit):
    """The s-step form of the smoother gives the same minimiser as the
    explicit orthonormal-basis least-squares problem (QR of the Krylov
    vectors), and so the same x as Arnoldi GMRES."""
    from oracle.krylov import gmres_jacobi_sstep
    g, A, b, _ = _system(4, 4, seed=1)
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(b.size) * 0.01
    dinv = 1.0 / A.diagonal()
    x, m, _ = gmres_jacobi_sstep(A, b, x0, maxit=kit, rtol=0.0, dinv=dinv)
    assert m == kit
    B = dinv[:, None] * A.toarray()
    r = dinv * (b - A @ x0)
    K = [r]
    for _ in range(kit - 1):
        K.append(B @ K[-1])
    Q, _ = np.linalg.qr(np.array(K).T)
    y, *_ = np.linalg.lstsq(B @ Q, r, rcond=None)
    x_ls = x0 + Q @ y
    assert np.linalg.norm(x - x_ls) <= 1e-9 * np.linalg.norm(x_ls)
    xg, _, _ = gmres_jacobi(A, b, x0, maxit=kit, rtol=0.0, dinv=dinv)
    assert np.linalg.norm(x - xg) <= 1e-9 * np.linalg.norm(xg)


def test_sstep_smoother_stops_where_gmres_stops():
    """With a tolerance reached before the cap both forms stop after the same
    number of steps; the preconditioned residuals they reach agree (the
    Gram route loses digits of x as the monomial basis grows ill-conditioned,
    about 1e-6 at nine vectors, but not of the residual it minimises)."""
    from oracle.krylov import gmres_jacobi_sstep
    g, A, b, _ = _system(6, 6, seed=5)
    dinv = 1.0 / A.diagonal()
    r0 = np.linalg.norm(dinv * b)
    for rtol, tol_x in ((0.7, 1e-12), (0.5, 1e-12), (0.3, 1e-10), (0.2, 1e-5)):
        xg, ig, eg = gmres_jacobi(A, b, None, maxit=10, rtol=rtol, dinv=dinv)
        xs, ms, es = gmres_jacobi_sstep(A, b, None, maxit=10, rtol=rtol, dinv=dinv)
        assert ig < 10 and ms == ig, (rtol, ig, ms)
        tg = np.linalg.norm(dinv * (b - A @ xg)) / r0
        ts = np.linalg.norm(dinv * (b - A @ xs)) / r0
        assert ts == pytest.approx(tg, rel=1e-8) and tg <= rtol
        assert es == pytest.approx(ts, rel=1e-5)
        assert np.linalg.norm(xs - xg) <= tol_x * np.linalg.norm(xg)


def test_sstep_smoother_vcycle_same_outer_iterations():
    """FGMRES with s-step-smoothed V-cycles converges like the Arnoldi-smoothed
    ones on the small workload (same count) and reaches the direct solution."""
    from paper_2508_09589_amd.inputs import uniform_density
    rho = uniform_density(32, seed=0)
    g = Grid(32, 32, 32, 1 / 32, 1 / 32)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    mask = dirichlet_mask(g, PATCH)
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0), mask)
    lv = build_hierarchy(32, 32, 32, 1 / 32, 1 / 32, 1.0, 1e-3, 1.0, 1.0)
    A, masks, Pm = build_operators(lv, Jm, mask)
    _, its_g, _ = fgmres(Jm, fm, VCycle(A, Pm, coarse="direct"), m=30, rtol=1e-10)
    x, its_s, rel = fgmres(Jm, fm, VCycle(A, Pm, coarse="direct", smoother="sstep"), m=30,
                           rtol=1e-10)
    assert its_s == its_g and rel <= 1e-10
    xs = solve_direct(Jm, fm)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_sstep_smoother_cuts_an_ill_conditioned_basis():
    """Past about ten monomial vectors the scaled Gram pivots reach rounding
    (SSTEP_MIN_PIVOT): the s-step form stops there and returns the minimiser
    over the vectors it kept -- the residual of Arnoldi GMRES with that many
    steps -- instead of amplifying rounding."""
    from oracle.krylov import gmres_jacobi_sstep
    g, A, b, _ = _system(6, 6, seed=5)
    dinv = 1.0 / A.diagonal()
    xs, m, _ = gmres_jacobi_sstep(A, b, None, maxit=15, rtol=0.0, dinv=dinv)
    assert 8 <= m < 15
    xg, _, _ = gmres_jacobi(A, b, None, maxit=m, rtol=0.0, dinv=dinv)
    rs = np.linalg.norm(dinv * (b - A @ xs))
    rg = np.linalg.norm(dinv * (b - A @ xg))
    assert rs == pytest.approx(rg, rel=1e-3)   # the last kept pivot is ~1e-11


@pytest.mark.parametrize("tv,filt", [(True, 1.5), (False, None)])
def test_block_central_difference_matches_adjoint_gradient(tv, filt):
    """The block-in-time difference-system central difference (the route of
    the 128^3 fixture) equals the adjoint gradient of the global-LU chain to
    1e-7 relative at h = 1e-6 on an 8^2 x 6 grid, and the global-LU
    difference system to 1e-9."""
    from oracle.blockgrad import central_difference_blocks
    from oracle.design import central_difference
    nx, nt = 8, 6
    g = Grid(nx, nx, nt, 1 / nx, 1 / nt)
    rng = np.random.default_rng(13)
    rho = rng.uniform(0.1, 0.9, (nt, nx, nx) if tv else (nx, nx))
    out = objective_and_gradient(g, MAT, rho, PATCH, 1.0, filt)
    for e in rng.choice(rho.size, 4, replace=False):
        ad = out["grad"].ravel()[e]
        fdb, sweeps = central_difference_blocks(g, MAT, rho, PATCH, e, 1e-6, 1.0, filt)
        fdg = central_difference(g, MAT, rho, PATCH, e, 1e-6, 1.0, filt)
        assert abs(fdb - ad) <= 1e-7 * abs(ad), (e, fdb, ad)
        assert abs(fdb - fdg) <= 1e-9 * abs(fdg), (e, fdb, fdg)
        assert max(sweeps) < 80

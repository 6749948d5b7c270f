"""Pins of the oracle's solutions: closed forms, invariants and convergence order."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import assemble_matrix, assemble_mass, load_vector, apply_dirichlet
from oracle.element import mass_1d, stiff_1d
from oracle.grid import Grid, dirichlet_mask
from oracle.solve import solve_direct, BlockTimeSystem

PATCH = [(0, 0.5, 0.05)]


def _solve(g, k, C, mask, f, gvals=None):
    J = assemble_matrix(g, k, C)
    Jm, fm = apply_dirichlet(J, f, mask, gvals)
    return solve_direct(Jm, fm), J, Jm, fm


def test_zero_data_gives_zero():
    g = Grid(6, 5, 4, 1 / 6, 0.25)
    rng = np.random.default_rng(0)
    k = rng.uniform(1e-3, 1, (4, 5, 6))
    s, *_ = _solve(g, k, np.ones((4, 5, 6)), dirichlet_mask(g, PATCH), np.zeros(g.n_nodes))
    assert np.max(np.abs(s)) == 0.0


def test_constant_initial_condition_is_preserved():
    """Q = 0, no patch, T(0) = c: T = c everywhere (A 1 = B 1 = 0)."""
    g = Grid(5, 7, 6, 1 / 7, 1 / 6)
    rng = np.random.default_rng(1)
    k = rng.uniform(1e-3, 1, (6, 7, 5))
    gv = np.full(g.n_nodes, 2.75)
    s, *_ = _solve(g, k, np.ones((6, 7, 5)), dirichlet_mask(g), np.zeros(g.n_nodes), gv)
    assert np.max(np.abs(s - 2.75)) < 1e-13


@pytest.mark.parametrize("time_varying", [False, True])
def test_sink_free_closed_form(time_varying):
    """No patch, C = 1, Q = q0: T(i,j,n) = n q0 dt for n < nt and
    (nt - 1/2) q0 dt at n = nt, for ANY conductivity field (§3.1.1: the
    stabilised time term is backward-difference-like, the final row is half
    weighted)."""
    nx, ny, nt = 6, 5, 7
    g = Grid(nx, ny, nt, 1 / 6, 1 / 7)
    rng = np.random.default_rng(2)
    k = rng.uniform(1e-3, 1, (nt, ny, nx) if time_varying else (ny, nx))
    q0 = 1.7
    s, *_ = _solve(g, k, np.ones((ny, nx)), dirichlet_mask(g), load_vector(g, q0))
    T = s.reshape(g.shape_nodes)
    expect = np.arange(nt + 1) * q0 * g.dt
    expect[-1] = (nt - 0.5) * q0 * g.dt
    assert np.max(np.abs(T - expect[:, None, None])) < 1e-13


def test_sink_free_time_dependent_source():
    """Nodal Q = q(t): C (T_n - T_{n-1}) = dt (q_{n-1} + 4 q_n + q_{n+1}) / 6 in
    the interior and dt (q_{nt-1} + 2 q_nt) / 6 at the last level."""
    nx, ny, nt = 4, 4, 9
    g = Grid(nx, ny, nt, 0.25, 1 / 9)
    rng = np.random.default_rng(3)
    k = rng.uniform(1e-3, 1, (ny, nx))
    q = np.cos(5 * np.arange(nt + 1) * g.dt)
    Q = np.broadcast_to(q[:, None, None], g.shape_nodes)
    s, *_ = _solve(g, k, np.ones((ny, nx)), dirichlet_mask(g), load_vector(g, q_nodal=Q))
    T = s.reshape(g.shape_nodes)[:, 0, 0]
    dT = np.diff(T)
    exp = np.empty(nt)
    exp[:-1] = g.dt * (q[:-2] + 4 * q[1:-1] + q[2:]) / 6
    exp[-1] = g.dt * (q[-2] + 2 * q[-1]) / 6
    assert np.max(np.abs(dT - exp)) < 1e-14


def _fe2d(nx, ny, dx, k2):
    """2-D Q1 stiffness and mass (element-wise, square elements)."""
    Mx, Sx = mass_1d(dx), stiff_1d(dx)
    Ke = np.kron(Mx, Sx) + np.kron(Sx, Mx)
    Me = np.kron(Mx, Mx)
    rows, cols, kv, mv = [], [], [], []
    for j in range(ny):
        for i in range(nx):
            loc = [(j + b2) * (nx + 1) + i + b1 for b2 in (0, 1) for b1 in (0, 1)]
            for a in range(4):
                for b in range(4):
                    rows.append(loc[a]); cols.append(loc[b])
                    kv.append(k2[j, i] * Ke[a, b]); mv.append(Me[a, b])
    P = (nx + 1) * (ny + 1)
    return (sp.csr_matrix((kv, (rows, cols)), shape=(P, P)),
            sp.csr_matrix((mv, (rows, cols)), shape=(P, P)))


def test_steady_state_reproduction():
    """Time-constant k, patch, uniform Q; with the initial condition equal to
    the 2-D steady FE solution X, T_n = X at every time level."""
    nx = ny = 8
    nt = 5
    dx = 1 / 8
    g = Grid(nx, ny, nt, dx, 0.2)
    rng = np.random.default_rng(4)
    k2 = rng.uniform(1e-2, 1, (ny, nx))
    K, M = _fe2d(nx, ny, dx, k2)
    m2 = dirichlet_mask(Grid(nx, ny, 0, dx, 1.0), PATCH, ic_dirichlet=False)[0].ravel()
    F = M @ np.ones(K.shape[0])
    Km, Fm = apply_dirichlet(K, F, m2)
    X = solve_direct(Km, Fm)
    mask = dirichlet_mask(g, PATCH)
    gv = np.broadcast_to(X, (nt + 1, X.size)).ravel()
    s, *_ = _solve(g, k2, np.ones((ny, nx)), mask, load_vector(g, 1.0), gv)
    T = s.reshape(nt + 1, -1)
    assert np.max(np.abs(T - X[None])) < 1e-12 * np.max(np.abs(X))


def test_heat_balance():
    """For the unmasked J and f and R = J s - f (zero on free rows):
    1^T J s = 1^T f + sum_D R_D, and 1^T J s telescopes to
    sum_i w_i (T_i(nt) - T_i(0)) with w the lumped capacity-weighted spatial
    mass (C time-constant)."""
    nx, ny, nt = 6, 6, 5
    g = Grid(nx, ny, nt, 1 / 6, 0.2)
    rng = np.random.default_rng(5)
    k = rng.uniform(1e-3, 1, (nt, ny, nx))
    C = rng.uniform(0.5, 2.0, (ny, nx))
    mask = dirichlet_mask(g, PATCH)
    f = load_vector(g, 1.0)
    s, J, _, _ = _solve(g, k, C, mask, f)
    R = J @ s - f
    assert np.max(np.abs(R[~mask.ravel()])) < 1e-14
    lhs = J @ s
    assert abs(lhs.sum() - (f.sum() + R[mask.ravel()].sum())) < 1e-14
    w = np.zeros((ny + 1, nx + 1))
    for a2 in (0, 1):
        for a1 in (0, 1):
            w[a2:a2 + ny, a1:a1 + nx] += C * g.dx ** 2 / 4
    T = s.reshape(g.shape_nodes)
    assert abs(lhs.sum() - (w * (T[-1] - T[0])).sum()) < 1e-14


def test_block_gauss_seidel_matches_global_lu():
    """The block-in-time route and the global LU agree to 1e-13 (small
    workload, time-constant k) and on a time-varying field."""
    from paper_2508_09589_amd.inputs import uniform_density
    rho = uniform_density(32, seed=0)
    g = Grid(32, 32, 32, 1 / 32, 1 / 32)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    C = np.ones_like(k)
    mask = dirichlet_mask(g, PATCH)
    f = load_vector(g, 1.0)
    s, J, Jm, fm = _solve(g, k, C, mask, f)
    bs = BlockTimeSystem(g, k, C, mask)
    sg, sweeps, rel = bs.gauss_seidel(bs.masked_rhs(f), tol=1e-13)
    assert rel <= 1e-13 and sweeps < 40
    assert np.linalg.norm(sg - s) / np.linalg.norm(s) < 1e-13
    # transposed sweep == adjoint LU
    lam_gs, _, _ = bs.gauss_seidel(bs.masked_rhs(f), tol=1e-13, transpose=True)
    from oracle.solve import solve_adjoint_direct
    lam = solve_adjoint_direct(Jm, f, mask)
    assert np.linalg.norm(lam_gs - lam) / np.linalg.norm(lam) < 1e-13


def test_spatial_order_two():
    """Manufactured X = cos(pi x1) cos(pi x2), Neumann, k = 1, Q = 2 pi^2 X,
    T(0) = X: the nodal error is O(dx^2) (§3.1.1: second order in space)."""
    errs = []
    for n in (8, 16, 32):
        nt = 4
        g = Grid(n, n, nt, 1.0 / n, 0.05 / nt)
        c = np.arange(n + 1) / n
        X = np.outer(np.cos(np.pi * c), np.cos(np.pi * c))
        Q = np.broadcast_to(2 * np.pi ** 2 * X, g.shape_nodes)
        f = load_vector(g, q_nodal=Q)
        gv = np.broadcast_to(X, g.shape_nodes).ravel()
        s, *_ = _solve(g, np.ones((n, n)), np.ones((n, n)), dirichlet_mask(g), f, gv)
        errs.append(np.max(np.abs(s.reshape(g.shape_nodes)[-1] - X)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_time_order_one():
    """Sink-free, q(t) = cos 5t: error against T(t) = sin(5t)/5 is first order
    in dt (§3.1.1: stabilisation lowers the time accuracy to first order)."""
    errs = []
    for nt in (16, 32, 64, 128):
        g = Grid(2, 2, nt, 0.5, 1.0 / nt)
        t = np.arange(nt + 1) * g.dt
        Q = np.broadcast_to(np.cos(5 * t)[:, None, None], g.shape_nodes)
        s, *_ = _solve(g, np.ones((2, 2)), np.ones((2, 2)), dirichlet_mask(g), load_vector(g, q_nodal=Q))
        T = s.reshape(g.shape_nodes)[:, 0, 0]
        errs.append(np.max(np.abs(T - np.sin(5 * t) / 5)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((rates > 0.85) & (rates < 1.3)), (errs, rates)


def test_transpose_identity():
    """<J v, w> = <v, J^T w> for the masked matrix and its matrix-free
    transposed application."""
    from oracle.residual import apply_masked
    g = Grid(5, 4, 3, 0.25, 1 / 3)
    rng = np.random.default_rng(6)
    k = rng.uniform(1e-3, 1, (3, 4, 5))
    C = rng.uniform(0.5, 1.5, (3, 4, 5))
    mask = dirichlet_mask(g, PATCH)
    v, w = rng.standard_normal((2, g.n_nodes))
    Jv = apply_masked(g, k, C, mask, v)
    JTw = apply_masked(g, k, C, mask, w, transpose=True)
    assert abs(Jv @ w - v @ JTw) < 1e-14 * np.linalg.norm(Jv) * np.linalg.norm(w)
    Jm, _ = apply_dirichlet(assemble_matrix(g, k, C), np.zeros(g.n_nodes), mask)
    assert np.max(np.abs(Jm @ v - Jv)) < 1e-15
    assert np.max(np.abs(Jm.T @ w - JTw)) < 1e-15


def test_sampled_residual_rows_match_assembled_matrix():
    """The node-by-node residual used for full-size checks reproduces rows of
    the assembled masked matrix (nx != ny, time-varying k and C)."""
    from oracle.residual import apply_masked_at, apply_masked
    g = Grid(7, 5, 4, 0.2, 0.25)
    rng = np.random.default_rng(8)
    k = rng.uniform(1e-3, 1, (4, 5, 7))
    C = rng.uniform(0.5, 1.5, (4, 5, 7))
    mask = dirichlet_mask(g, [(0, 0.5, 0.25), (3, 0.7, 0.3)])
    Jm, _ = apply_dirichlet(assemble_matrix(g, k, C), np.zeros(g.n_nodes), mask)
    x = rng.standard_normal(g.n_nodes)
    nodes = rng.choice(g.n_nodes, 60, replace=False)
    y = Jm @ x
    assert np.max(np.abs(apply_masked_at(g, k, C, mask, x, nodes) - y[nodes])) < 1e-14
    assert np.max(np.abs(apply_masked(g, k, C, mask, x) - y)) < 1e-14


@pytest.mark.parametrize("transpose", [False, True])
def test_residual_by_planes_equals_assembled_residual(transpose):
    """The plane-by-plane residual of the full-size checks equals the
    residual formed with the assembled sparse matrix (norm and maximum)."""
    from oracle.assemble import assemble_matrix, apply_dirichlet, load_vector
    from oracle.grid import Grid, dirichlet_mask
    from oracle.residual import residual_by_planes
    g = Grid(7, 5, 6, 1 / 7, 1 / 6)
    rng = np.random.default_rng(21)
    k = rng.uniform(0.01, 1.0, (6, 5, 7))
    C = rng.uniform(0.5, 2.0, (6, 5, 7))
    mask = dirichlet_mask(g, [(0, 0.5, 0.2)])
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, C), load_vector(g, 1.0), mask)
    x = rng.standard_normal(g.n_nodes)
    r = fm - (Jm.T if transpose else Jm) @ x
    if transpose:
        # the transposed masked system keeps identity rows on the Dirichlet set
        r = np.where(mask.ravel(), fm - x, r)
    nr, mx = residual_by_planes(g, k, C, mask, x, fm, transpose)
    assert abs(nr - np.linalg.norm(r)) <= 1e-13 * np.linalg.norm(r)
    assert abs(mx - np.max(np.abs(r))) <= 1e-13 * np.max(np.abs(r))

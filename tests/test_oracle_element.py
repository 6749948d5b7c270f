"""Pins of the oracle's element matrices and assembly (brute force, closed forms)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.assemble import Material, assemble_matrix, load_vector, apply_dirichlet, simp
from oracle.element import element_matrices, element_matrix_quadrature, mass_1d
from oracle.grid import Grid, dirichlet_mask
from oracle.solve import solve_direct


@pytest.mark.parametrize("dx,dt,k,C", [(0.5, 0.25, 1.0, 1.0), (1 / 3, 0.1, 0.37, 2.5), (0.01, 0.7, 3.0, 0.5)])
def test_kron_equals_quadrature(dx, dt, k, C):
    """The Kronecker element matrix equals 3-point Gauss quadrature of the
    stabilised weak form (§3.1.1) to round-off."""
    A, B = element_matrices(dx, dt)
    Jq = element_matrix_quadrature(dx, dt, k, C)
    Jk = k * A + C * B
    assert np.max(np.abs(Jq - Jk)) <= 1e-15 * max(1.0, np.max(np.abs(Jk))) * 10


def test_capacity_block_is_upwind():
    """With k_ad = C dt / 2 the time term is exactly C * U (x) Mx (x) Mx,
    U = [[0,0],[-1,1]]: the lower node's test row is empty."""
    dx, dt = 0.2, 0.05
    _, B = element_matrices(dx, dt)
    U = np.array([[0.0, 0.0], [-1.0, 1.0]])
    Mx = mass_1d(dx)
    assert np.allclose(B, np.kron(U, np.kron(Mx, Mx)), rtol=0, atol=1e-17)
    assert np.all(B[:4] == 0.0)


def test_element_diagonal_closed_form():
    dx, dt = 0.125, 0.03
    A, B = element_matrices(dx, dt)
    assert np.allclose(np.diag(A), 2 * dt / 9, rtol=1e-14)
    assert np.allclose(np.diag(B)[:4], 0.0)
    assert np.allclose(np.diag(B)[4:], dx * dx / 9, rtol=1e-14)
    # conduction and capacity rows sum to zero (constants are in the kernel)
    assert np.max(np.abs(A.sum(axis=1))) < 1e-16
    assert np.max(np.abs(B.sum(axis=1))) < 1e-16


def test_interior_node_diagonal():
    """An interior node of a uniform-coefficient mesh has 8 elements around it:
    diag = 16 k dt / 9 + 4 C dx^2 / 9."""
    g = Grid(4, 4, 4, 0.25, 0.1)
    k, C = 0.7, 1.3
    J = assemble_matrix(g, np.full((4, 4), k), np.full((4, 4), C))
    a = g.node(2, 2, 2)
    assert abs(J[a, a] - (16 * k * g.dt / 9 + 4 * C * g.dx ** 2 / 9)) < 1e-15


@pytest.mark.parametrize("nx,ny,nt", [(1, 1, 1), (2, 2, 2), (3, 2, 2)])
def test_tiny_assembly_quadrature_and_dense_solve(nx, ny, nt):
    """On tiny grids (nx != ny included) the global matrix assembled from
    quadrature element matrices equals the Kronecker one, and a dense solve
    equals the sparse LU solve."""
    rng = np.random.default_rng(11)
    dx, dt = 1.0 / max(nx, ny), 1.0 / nt
    g = Grid(nx, ny, nt, dx, dt)
    k = rng.uniform(0.1, 2.0, (nt, ny, nx))
    C = rng.uniform(0.5, 1.5, (nt, ny, nx))
    J = assemble_matrix(g, k, C).toarray()
    Jq = np.zeros_like(J)
    conn = g.connectivity()
    for e in range(g.n_elems):
        n, rem = divmod(e, nx * ny)
        j, i = divmod(rem, nx)
        Je = element_matrix_quadrature(dx, dt, k[n, j, i], C[n, j, i])
        Jq[np.ix_(conn[e], conn[e])] += Je
    assert np.max(np.abs(J - Jq)) < 1e-14
    mask = dirichlet_mask(g, patches=[(0, 0.5 * ny * dx, 0.5)])
    f = load_vector(g, q0=1.0)
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, C), f, mask)
    s_sparse = solve_direct(Jm, fm)
    s_dense = np.linalg.solve(Jm.toarray(), fm)
    assert np.max(np.abs(s_sparse - s_dense)) <= 1e-13 * max(1.0, np.max(np.abs(s_dense)))


def test_patch_node_counts():
    """Centred 10% patch on the x1 = 0 edge: 3, 7, 13, 25, 51 nodes per time
    level at 32, 64, 128, 256, 512 elements per side."""
    for n, cnt in [(32, 3), (64, 7), (128, 13), (256, 25), (512, 51)]:
        g = Grid(n, n, 1, 1.0 / n, 1.0)
        m = dirichlet_mask(g, patches=[(0, 0.5, 0.05)], ic_dirichlet=False)
        assert m[1].sum() == cnt


def test_simp_endpoints_and_derivative():
    mat = Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=0.5, c_con=1.0, p_c=2.0)
    k, C, dk, dC = simp(np.array([0.0, 1.0, 0.3]), mat)
    assert np.allclose(k[:2], [1e-3, 1.0]) and np.allclose(C[:2], [0.5, 1.0])
    h = 1e-6
    kp, Cp, _, _ = simp(np.array([0.3 + h]), mat)
    km, Cm, _, _ = simp(np.array([0.3 - h]), mat)
    assert abs((kp - km)[0] / (2 * h) - dk[2]) < 1e-8
    assert abs((Cp - Cm)[0] / (2 * h) - dC[2]) < 1e-8


def test_uniform_load_without_scatter():
    """The separable uniform load equals the scattered one on ragged grids,
    and the loads sum to q0 times the space-time volume."""
    from oracle.assemble import load_vector_uniform
    for nx, ny, nt in [(1, 1, 1), (5, 3, 4), (7, 9, 2)]:
        g = Grid(nx, ny, nt, 0.3, 0.7)
        f = load_vector_uniform(g, 2.5)
        assert np.max(np.abs(f - load_vector(g, 2.5))) < 1e-15
        assert abs(f.sum() - 2.5 * nx * ny * 0.09 * nt * 0.7) < 1e-12

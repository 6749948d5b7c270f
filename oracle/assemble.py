"""Global assembly of the all-at-once space-time system J s = f (oracle).

Paper §3.1.2: J and f are assembled element by element from the left- and
right-hand sides of the space-time heat equation.  Coefficients come from the
modified SIMP interpolation of §2.2 (equations "SIMP c" and "SIMP k"), applied
per element to the physical density (design constant per element, §3.3.1).
"""
import numpy as np
import scipy.sparse as sp

from .element import element_matrices, element_mass


class Material:
    """SIMP endpoints and penalties, §2.2."""

    def __init__(self, k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0):
        self.k_ins, self.k_con, self.p_k = float(k_ins), float(k_con), float(p_k)
        self.c_ins, self.c_con, self.p_c = float(c_ins), float(c_con), float(p_c)


def simp(rho, mat):
    """Return k, C, dk/drho, dC/drho per element (§2.2, modified SIMP)."""
    rho = np.asarray(rho, dtype=np.float64)
    k = mat.k_ins + (mat.k_con - mat.k_ins) * rho ** mat.p_k
    C = mat.c_ins + (mat.c_con - mat.c_ins) * rho ** mat.p_c
    dk = mat.p_k * (mat.k_con - mat.k_ins) * rho ** (mat.p_k - 1.0)
    dC = mat.p_c * (mat.c_con - mat.c_ins) * rho ** (mat.p_c - 1.0)
    return k, C, dk, dC


def broadcast_elements(grid, field):
    """Element field of shape [nt, ny, nx] from a time-constant [ny, nx] (or
    [1, ny, nx]) field -- the extrusion of §3.4.1 -- or pass a full one through."""
    f = np.asarray(field, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    if f.shape[0] == 1 and grid.nt > 1:
        f = np.broadcast_to(f, (grid.nt, grid.ny, grid.nx))
    assert f.shape == grid.shape_elems, (f.shape, grid.shape_elems)
    return np.ascontiguousarray(f)


def assemble_matrix(grid, k_e, C_e):
    """Unmasked global J = sum_e P_e^T (k_e A + C_e B) P_e as CSR."""
    A, B = element_matrices(grid.dx, grid.dt)
    k = broadcast_elements(grid, k_e).ravel()
    C = broadcast_elements(grid, C_e).ravel()
    conn = grid.connectivity()
    vals = k[:, None, None] * A[None] + C[:, None, None] * B[None]   # [E, 8, 8]
    rows = np.repeat(conn[:, :, None], 8, axis=2)
    cols = np.repeat(conn[:, None, :], 8, axis=1)
    N = grid.n_nodes
    J = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N))
    return J.tocsr()


def assemble_mass(grid):
    """Consistent space-time mass matrix M_st (unit capacity)."""
    Me = element_mass(grid.dx, grid.dt)
    conn = grid.connectivity()
    rows = np.repeat(conn[:, :, None], 8, axis=2)
    cols = np.repeat(conn[:, None, :], 8, axis=1)
    vals = np.broadcast_to(Me, (conn.shape[0], 8, 8))
    N = grid.n_nodes
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N)).tocsr()


def load_vector(grid, q0=1.0, q_nodal=None):
    """Consistent load f_a = sum_e int_e Q N_a dV.

    Uniform Q = q0: every element contributes q0*V_e/8 to each of its nodes.
    Nodal Q (trilinear interpolant): f = M_st Q.
    """
    if q_nodal is not None:
        return assemble_mass(grid) @ np.asarray(q_nodal, dtype=np.float64).ravel()
    conn = grid.connectivity()
    f = np.zeros(grid.n_nodes)
    np.add.at(f, conn.ravel(), q0 * grid.dx * grid.dx * grid.dt / 8.0)
    return f


def load_vector_uniform(grid, q0=1.0):
    """The uniform-Q load of load_vector without the connectivity scatter, for
    grids too large for it: node a lies in c_x c_y c_t elements (c = 1 on a
    boundary plane of that axis, 2 inside), so f_a = c_x c_y c_t q0 V_e / 8."""
    def counts(n):
        c = np.full(n + 1, 2.0)
        c[0] = c[-1] = 1.0
        return c
    ve8 = q0 * grid.dx * grid.dx * grid.dt / 8.0
    f = (counts(grid.nt)[:, None, None] * counts(grid.ny)[None, :, None]) * counts(grid.nx)[None, None, :]
    f *= ve8
    return f.ravel()


def apply_dirichlet(J, f, mask, g=None):
    """Symmetric elimination of the Dirichlet set (reading: the paper is silent).

    J_m = N J N + (I - N),  f_m = N (f - J g) + g,  N = diag(1 - mask).
    g holds the prescribed values on Dirichlet nodes (zero elsewhere).
    """
    m = np.asarray(mask, dtype=bool).ravel()
    keep = (~m).astype(np.float64)
    Nd = sp.diags(keep)
    Jm = (Nd @ J @ Nd + sp.diags(1.0 - keep)).tocsr()
    if g is None:
        g = np.zeros(J.shape[0])
    g = np.where(m, np.asarray(g, dtype=np.float64).ravel(), 0.0)
    fm = keep * (f - J @ g) + g
    return Jm, fm

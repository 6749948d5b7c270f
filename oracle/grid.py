"""Structured space-time grid and Dirichlet set (oracle).

Paper §3.1.2: a regular mesh of nx1 x nx2 x nt trilinear elements, square in
space (dx1 = dx2 = dx), dt in time; N_n = (nx1+1)(nx2+1)(nt+1) nodes.

Numbering (the reading used throughout):
  node  g(i, j, n) = (n*(ny+1) + j)*(nx+1) + i     i <= nx, j <= ny, n <= nt
  elem  e(i, j, n) = (n*ny + j)*nx + i
  local node a = a1 + 2*a2 + 4*a3  <->  (i+a1, j+a2, n+a3)
"""
import numpy as np

# Patch edges: which boundary line of the spatial square carries a T=0 patch.
EDGE_X1_LO, EDGE_X1_HI, EDGE_X2_LO, EDGE_X2_HI = 0, 1, 2, 3


class Grid:
    def __init__(self, nx, ny, nt, dx, dt):
        self.nx, self.ny, self.nt = int(nx), int(ny), int(nt)
        self.dx, self.dt = float(dx), float(dt)

    @property
    def shape_nodes(self):
        return (self.nt + 1, self.ny + 1, self.nx + 1)

    @property
    def shape_elems(self):
        return (self.nt, self.ny, self.nx)

    @property
    def n_nodes(self):
        return (self.nx + 1) * (self.ny + 1) * (self.nt + 1)

    @property
    def n_elems(self):
        return self.nx * self.ny * self.nt

    def node(self, i, j, n):
        return (n * (self.ny + 1) + j) * (self.nx + 1) + i

    def connectivity(self):
        """[n_elems, 8] global node numbers of each element's local nodes."""
        nx, ny, nt = self.nx, self.ny, self.nt
        n, j, i = np.meshgrid(np.arange(nt), np.arange(ny), np.arange(nx), indexing="ij")
        n, j, i = n.ravel(), j.ravel(), i.ravel()
        conn = np.empty((nx * ny * nt, 8), dtype=np.int64)
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            conn[:, a] = self.node(i + a1, j + a2, n + a3)
        return conn


def patch_index_range(n_along, dx, centre, half_width):
    """Indices k along an edge whose node lies in [centre-hw, centre+hw].

    Reading: the patch is closed, with a 1e-12 slack so that nodes exactly on
    its ends are included (the paper gives only its width, §2.3.1).
    """
    k = np.arange(n_along + 1)
    inside = np.abs(k * dx - centre) <= half_width + 1e-12
    idx = np.nonzero(inside)[0]
    if idx.size == 0:
        return None
    return int(idx[0]), int(idx[-1])


def dirichlet_mask(grid, patches=(), ic_dirichlet=True):
    """Boolean [nt+1, ny+1, nx+1]: True on Dirichlet nodes.

    Reading: the initial condition is imposed strongly on the whole n = 0 plane
    (the paper is silent on how, §3.1.1); every patch (edge, centre, half
    width, in physical units) is T = 0 on that edge at every time level
    (§2.3.1 puts a sink of width L/10 on one edge).
    """
    m = np.zeros(grid.shape_nodes, dtype=bool)
    if ic_dirichlet:
        m[0] = True
    for (edge, centre, hw) in patches:
        if edge in (EDGE_X1_LO, EDGE_X1_HI):
            r = patch_index_range(grid.ny, grid.dx, centre, hw)
            if r is None:
                continue
            i = 0 if edge == EDGE_X1_LO else grid.nx
            m[:, r[0]:r[1] + 1, i] = True
        else:
            r = patch_index_range(grid.nx, grid.dx, centre, hw)
            if r is None:
                continue
            j = 0 if edge == EDGE_X2_LO else grid.ny
            m[:, j, r[0]:r[1] + 1] = True
    return m

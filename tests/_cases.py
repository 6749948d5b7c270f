"""Shared case builder for the GPU parity tests: seeded inputs plus the oracle's
matrices for the same problem.  (Test infrastructure; imports the oracle.)"""
import numpy as np

from oracle.assemble import Material, assemble_matrix, apply_dirichlet, load_vector, simp
from oracle.grid import Grid, dirichlet_mask
from oracle.hierarchy import build_hierarchy
from oracle.multigrid import build_operators

PATCH = ((0, 0.5, 0.05),)
MAT = dict(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0)


class Case:
    def __init__(self, nx, ny, nt, tv=False, seed=0, patches=PATCH, mat=None, q0=1.0,
                 max_coarse_nodes=4096, rho=None, dx=None, dt=None, full=False, source=None):
        self.nx, self.ny, self.nt = nx, ny, nt
        self.mat = dict(MAT if mat is None else mat)
        self.dx = 1.0 / max(nx, ny) if dx is None else dx
        self.dt = 1.0 / nt if dt is None else dt
        rng = np.random.default_rng(seed)
        if rho is None:
            rho = rng.uniform(1e-3, 1.0, (nt, ny, nx) if tv else (ny, nx))
        self.rho = np.asarray(rho, dtype=np.float64)
        self.tv = self.rho.ndim == 3 and self.rho.shape[0] == nt and nt > 1
        self.patches = tuple(patches)
        self.q0 = q0
        self.full = full
        self.source = None if source is None else np.asarray(source, dtype=np.float64)
        self.grid = Grid(nx, ny, nt, self.dx, self.dt)
        m = Material(**self.mat)
        self.k, self.C, self.dk, self.dC = simp(self.rho, m)
        self.mask = dirichlet_mask(self.grid, self.patches)
        self.f = load_vector(self.grid, q0, q_nodal=self.source)
        self.J = assemble_matrix(self.grid, self.k, self.C)
        self.Jm, self.fm = apply_dirichlet(self.J, self.f, self.mask)
        self.levels = build_hierarchy(nx, ny, nt, self.dx, self.dt, m.k_con, m.k_ins, m.c_con,
                                      m.c_ins, max_coarse_nodes=max_coarse_nodes, full=full)
        self._ops = None

    @property
    def ops(self):
        if self._ops is None:
            self._ops = build_operators(self.levels, self.Jm, self.mask)
        return self._ops

    def problem(self, **kw):
        import torch
        from paper_2508_09589_amd import Problem
        kw.setdefault("max_coarse_nodes", 4096)
        if self.full:
            kw.setdefault("coarsening", "full")
        if self.source is not None:
            kw.setdefault("source", torch.tensor(self.source))
        return Problem(self.nx, self.ny, self.nt, torch.tensor(self.rho), dx=self.dx, dt=self.dt,
                       patches=self.patches, q0=self.q0, **self.mat, **kw)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (s if s > 0 else 1.0)

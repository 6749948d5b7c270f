"""Objective and adjoint gradient of the differentiation workload on grids too
large for a global LU (oracle).

Same chain as design.objective_and_gradient (§3.3: filter -> SIMP -> state
solve -> J = f^T s -> adjoint solve -> element sensitivities -> filter
transpose), with the state and adjoint solved by block Gauss-Seidel in time
(solve.BlockTimeSystem: forward sweeps for J, backward sweeps for J^T)."""
import numpy as np

from .assemble import simp, load_vector
from .design import filter_apply, element_sensitivity, reduce_to_design, objective
from .grid import dirichlet_mask
from .solve import BlockTimeSystem


def objective_and_gradient_blocks(grid, mat, rho, patches, q0=1.0, r_elems=None, tol=1e-12,
                                  max_sweeps=60):
    rho = np.asarray(rho, dtype=np.float64)
    if r_elems is not None:
        rho_phys = filter_apply(rho, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    else:
        rho_phys = rho
    k, C, dk, dC = simp(rho_phys, mat)
    mask = dirichlet_mask(grid, patches)
    f = load_vector(grid, q0)
    bs = BlockTimeSystem(grid, k, C, mask)
    s, sw, rel = bs.gauss_seidel(bs.masked_rhs(f), tol=tol, max_sweeps=max_sweeps)
    lam, sw2, rel2 = bs.gauss_seidel(bs.masked_rhs(f), tol=tol, transpose=True,
                                     max_sweeps=max_sweeps)
    ge = element_sensitivity(grid, s, lam, dk, dC)
    g = reduce_to_design(ge, rho.shape)
    if r_elems is not None:
        g = filter_apply(g, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    return dict(J=objective(f, s), grad=g, s=s, lam=lam, sweeps=(sw, sw2), rel=(rel, rel2))

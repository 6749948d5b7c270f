"""Objective and adjoint gradient of the differentiation workload on grids too
large for a global LU (oracle).

Same chain as design.objective_and_gradient (§3.3: filter -> SIMP -> state
solve -> J = f^T s -> adjoint solve -> element sensitivities -> filter
transpose), with the state and adjoint solved by block Gauss-Seidel in time
(solve.BlockTimeSystem: forward sweeps for J, backward sweeps for J^T)."""
import numpy as np

from .assemble import simp, load_vector
from .design import (filter_apply, element_sensitivity, reduce_to_design, objective,
                     simp_difference)
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


def central_difference_blocks(grid, mat, rho, patches, e, h=1e-6, q0=1.0, r_elems=None,
                              tol=1e-13, max_sweeps=80, s0=None):
    """design.central_difference on grids too large for a global LU: the
    central difference of J = f^T s at rho +- h e_i from the difference
    system J+ (s+ - s-) = -(J+ - J-) s-, with J+ - J- assembled from
    k(rho+) - k(rho-) directly; both systems solved by block Gauss-Seidel in
    time (s- starting from s0, e.g. the state at rho, when given).
    Returns (dJ/drho_i estimate, sweeps of the two solves)."""
    rho = np.asarray(rho, dtype=np.float64)
    rp = rho.copy().ravel()
    rp[e] += h
    rm = rho.copy().ravel()
    rm[e] -= h
    rp, rm = rp.reshape(rho.shape), rm.reshape(rho.shape)
    if r_elems is not None:
        rx, rt = r_elems * grid.dx, r_elems * grid.dt
        fp = filter_apply(rp, grid.dx, grid.dt, rx, rt)
        fm_ = filter_apply(rm, grid.dx, grid.dt, rx, rt)
        dphys = filter_apply(rp - rm, grid.dx, grid.dt, rx, rt)
    else:
        fp, fm_, dphys = rp, rm, rp - rm
    kp, Cp, _, _ = simp(fp, mat)
    km, Cm, _, _ = simp(fm_, mat)
    dk, dC = simp_difference(fp, fm_, dphys, mat)
    mask = dirichlet_mask(grid, patches)
    f = load_vector(grid, q0)
    minus = BlockTimeSystem(grid, km, Cm, mask)
    sm, sw1, _ = minus.gauss_seidel(minus.masked_rhs(f), tol=tol, max_sweeps=max_sweeps, x0=s0)
    del minus
    diff = BlockTimeSystem(grid, dk, dC, mask)
    keep = ~np.asarray(mask, dtype=bool).ravel()
    rhs = np.where(keep, -diff.matvec(np.where(keep, sm, 0.0), masked=False), 0.0)
    del diff
    plus = BlockTimeSystem(grid, kp, Cp, mask)
    ds, sw2, _ = plus.gauss_seidel(rhs, tol=tol, max_sweeps=max_sweeps)
    return float(f @ ds) / (2 * h), (sw1, sw2)

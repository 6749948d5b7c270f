"""Density filter, objective and adjoint sensitivities (oracle).

Paper §3.3.2: the PDE (Helmholtz) filter -d_ij d^2 g~/dxi_i dxi_j + g~ = g with
d = diag(r_x^2, r_x^2, r_t^2)/12, and the chain rule that sends sensitivities
through the same filter equation.  §3.3.3: adjoint sensitivities
dphi/drho_e = -lambda^T dr/drho_e with J^T lambda = (dphi/ds)^T.

Readings:
  * the filter is discretised with the same trilinear elements (nodal g~),
    homogeneous Neumann boundaries, consistent mass; the element value is the
    mean of its 8 nodal values, and the element input enters through
    int_e N_a dV = V_e/8;  F = (1/8) E^T (K_d + M)^{-1} (V/8) E is symmetric;
  * a time-constant design ([ny, nx]) is filtered on a single slab, which is
    exactly the space-time filter of its extrusion (§3.4.1);
  * the objective of the differentiation workload is J = int Q T = f^T s with
    the unmasked consistent load f; it has no explicit density dependence.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import mass_1d, stiff_1d
from .grid import Grid


def filter_element_matrix(dx, dt, rx, rt):
    dxx = rx * rx / 12.0
    dtt = rt * rt / 12.0
    Mx, Sx, Mt, St = mass_1d(dx), stiff_1d(dx), mass_1d(dt), stiff_1d(dt)
    K = dxx * (np.kron(Mt, np.kron(Mx, Sx)) + np.kron(Mt, np.kron(Sx, Mx))) \
        + dtt * np.kron(St, np.kron(Mx, Mx))
    M = np.kron(Mt, np.kron(Mx, Mx))
    return K + M


def filter_operators(nx, ny, nt, dx, dt, rx, rt):
    """Return (H, E, V): nodal Helmholtz matrix, element->node incidence
    [n_nodes, n_elems], element volume."""
    g = Grid(nx, ny, nt, dx, dt)
    He = filter_element_matrix(dx, dt, rx, rt)
    conn = g.connectivity()
    rows = np.repeat(conn[:, :, None], 8, axis=2).ravel()
    cols = np.repeat(conn[:, None, :], 8, axis=1).ravel()
    vals = np.broadcast_to(He, (conn.shape[0], 8, 8)).ravel()
    H = sp.coo_matrix((vals, (rows, cols)), shape=(g.n_nodes, g.n_nodes)).tocsc()
    E = sp.coo_matrix((np.ones(conn.size), (conn.ravel(), np.repeat(np.arange(g.n_elems), 8))),
                      shape=(g.n_nodes, g.n_elems)).tocsr()
    return H, E, dx * dx * dt


def filter_apply(gamma, dx, dt, rx, rt, method=None):
    """Filtered element field F gamma for gamma of shape [nt, ny, nx] or [ny, nx].

    The nodal system is solved by sparse LU, or -- above 2e5 nodes -- by
    Jacobi-preconditioned CG to a relative residual of 1e-14 (H is SPD)."""
    gam = np.asarray(gamma, dtype=np.float64)
    two_d = gam.ndim == 2
    if two_d:
        gam = gam[None]
    nt, ny, nx = gam.shape
    H, E, V = filter_operators(nx, ny, nt, dx, dt, rx, rt)
    rhs = (V / 8.0) * (E @ gam.ravel())
    if method == "lu" or (method is None and H.shape[0] <= 200000):
        gn = spla.spsolve(H, rhs)
    else:
        dinv = 1.0 / H.diagonal()
        M = sp.diags(dinv)
        gn, info = spla.cg(H.tocsr(), rhs, rtol=1e-14, atol=0.0, M=M, maxiter=10000)
        assert info == 0
    out = (E.T @ gn / 8.0).reshape(gam.shape)
    return out[0] if two_d else out


def objective(f_full, s):
    """J = f^T s (int Q T with the consistent load)."""
    return float(np.dot(np.asarray(f_full).ravel(), np.asarray(s).ravel()))


def element_sensitivity(grid, s, lam, dk_e, dC_e):
    """g_e = -lambda_e^T (dk_e A + dC_e B) s_e per space-time element (§3.3.3).

    s holds the full state (Dirichlet values included), lam is zero on the
    Dirichlet set."""
    from .element import element_matrices
    from .assemble import broadcast_elements
    A, B = element_matrices(grid.dx, grid.dt)
    conn = grid.connectivity()
    se = np.asarray(s).ravel()[conn]          # [E, 8]
    le = np.asarray(lam).ravel()[conn]
    la = np.einsum("ea,ab,eb->e", le, A, se)
    lb = np.einsum("ea,ab,eb->e", le, B, se)
    dk = broadcast_elements(grid, dk_e).ravel()
    dC = broadcast_elements(grid, dC_e).ravel()
    return (-(dk * la + dC * lb)).reshape(grid.shape_elems)


def reduce_to_design(g_elem, design_shape):
    """Chain rule through the extrusion of a time-constant design (§3.4.1):
    the sensitivity of a driving variable is the sum over time slabs."""
    if len(design_shape) == 2 or design_shape[0] == 1:
        return g_elem.sum(axis=0).reshape(design_shape)
    return g_elem.reshape(design_shape)


def objective_and_gradient(grid, mat, rho, patches, q0=1.0, r_elems=None, with_grad=True):
    """Full chain of the differentiation workload (§3.3): filter -> SIMP ->
    state solve -> J = f^T s -> adjoint solve -> element sensitivities ->
    extrusion sum (time-constant designs) -> filter transpose.

    rho: unfiltered design, [ny, nx] (time-constant) or [nt, ny, nx].
    r_elems: filter radius in elements (r_x = r dx, r_t = r dt); None = no filter.
    Returns dict(J, grad, s, lam, rho_phys)."""
    from .assemble import simp, assemble_matrix, load_vector, apply_dirichlet
    from .grid import dirichlet_mask
    from .solve import solve_direct, solve_adjoint_direct
    rho = np.asarray(rho, dtype=np.float64)
    if r_elems is not None:
        rho_phys = filter_apply(rho, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    else:
        rho_phys = rho
    k, C, dk, dC = simp(rho_phys, mat)
    mask = dirichlet_mask(grid, patches)
    f = load_vector(grid, q0)
    J = assemble_matrix(grid, k, C)
    Jm, fm = apply_dirichlet(J, f, mask)
    s = solve_direct(Jm, fm)
    out = dict(J=objective(f, s), s=s, rho_phys=rho_phys)
    if not with_grad:
        return out
    lam = solve_adjoint_direct(Jm, f, mask)
    ge = element_sensitivity(grid, s, lam, dk, dC)
    g = reduce_to_design(ge, rho.shape)
    if r_elems is not None:
        g = filter_apply(g, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    out.update(grad=g, lam=lam)
    return out


def power_difference(a, b, p, d):
    """a^p - b^p formed from the difference d = a - b itself:
    (a - b) * sum_{q<p} a^q b^(p-1-q) for an integer exponent p (no
    subtraction of nearly equal powers); other exponents subtract."""
    pi = int(round(p))
    if abs(p - pi) > 0 or pi < 1:
        return a ** p - b ** p
    acc = np.zeros_like(a)
    for q in range(pi):
        acc = acc + a ** q * b ** (pi - 1 - q)
    return d * acc


def simp_difference(a, b, d, mat):
    """k(a) - k(b) and C(a) - C(b) of the SIMP laws (§2.2) for physical
    densities a, b with d = a - b given."""
    return ((mat.k_con - mat.k_ins) * power_difference(a, b, mat.p_k, d),
            (mat.c_con - mat.c_ins) * power_difference(a, b, mat.p_c, d))


def central_difference(grid, mat, rho, patches, e, h=1e-6, q0=1.0, r_elems=None):
    """(J(rho + h e_i) - J(rho - h e_i)) / (2h) without cancellation.

    With J+ and J- the masked matrices at rho +- h e_i, s+ - s- solves
    J+ (s+ - s-) = -(J+ - J-) s-, where J+ - J- is assembled directly from
    k(rho+) - k(rho-) and C(rho+) - C(rho-); then dJ = f^T (s+ - s-).  This is
    algebraically the two-solve central difference, but the small difference
    is never formed by subtracting two nearly equal objective values."""
    from .assemble import simp, assemble_matrix, load_vector, apply_dirichlet
    from .grid import dirichlet_mask
    from .solve import solve_direct
    rho = np.asarray(rho, dtype=np.float64)
    rp = rho.copy().ravel(); rp[e] += h
    rm = rho.copy().ravel(); rm[e] -= h
    rp, rm = rp.reshape(rho.shape), rm.reshape(rho.shape)
    if r_elems is not None:
        fp = filter_apply(rp, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
        fm_ = filter_apply(rm, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
        dphys = filter_apply((rp - rm), grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    else:
        fp, fm_, dphys = rp, rm, rp - rm
    kp, Cp, _, _ = simp(fp, mat)
    km, Cm, _, _ = simp(fm_, mat)
    dk, dC = simp_difference(fp, fm_, dphys, mat)
    mask = dirichlet_mask(grid, patches)
    f = load_vector(grid, q0)
    Jp, _ = apply_dirichlet(assemble_matrix(grid, kp, Cp), f, mask)
    Jn, fmask = apply_dirichlet(assemble_matrix(grid, km, Cm), f, mask)
    dJ = assemble_matrix(grid, dk, dC)
    keep = (~np.asarray(mask).ravel()).astype(np.float64)
    sm = solve_direct(Jn, fmask)
    ds = solve_direct(Jp, -(keep * (dJ @ (keep * sm))))
    return float(f @ ds) / (2 * h)


# ---------------------------------------------------------------------------
# The design chain of §3.3.1-§3.3.3 beyond the differentiation workload:
# Heaviside projection of the filtered field, the p-norm objective of the
# element-averaged temperature with its adjoint right-hand side, and the
# volume constraint.

def heaviside(x, beta, eta):
    """Projection of §3.3.2 (Wang et al.): (tanh(b e) + tanh(b (x - e))) /
    (tanh(b e) + tanh(b (1 - e)))."""
    x = np.asarray(x, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (x - eta))) / den


def heaviside_deriv(x, beta, eta):
    """d heaviside / dx = beta (1 - tanh^2(beta (x - eta))) / den."""
    x = np.asarray(x, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    t = np.tanh(beta * (x - eta))
    return beta * (1.0 - t * t) / den


def element_average(grid, s):
    """T_avg,e = (1/8) sum of the element's 8 nodal values (§3.3.1)."""
    conn = grid.connectivity()
    return np.asarray(s, dtype=np.float64).ravel()[conn].mean(axis=1)


def pnorm(grid, s, P):
    """phi = (sum_e T_avg,e^P)^(1/P) and its gradient with respect to the
    nodal state, assembled from dphi/ds_e = theta^((1-P)/P) T_avg,e^(P-1) / 8
    per element node (§3.3.3), theta = sum_e T_avg,e^P."""
    Tavg = element_average(grid, s)
    theta = float(np.sum(Tavg ** P))
    phi = theta ** (1.0 / P)
    w = theta ** ((1.0 - P) / P) * Tavg ** (P - 1.0) / 8.0
    conn = grid.connectivity()
    g = np.zeros(grid.n_nodes)
    np.add.at(g, conn.ravel(), np.repeat(w, 8))
    return phi, g


def volume(grid, rho_phys, vf):
    """chi = sum_e rho_e v_e / (vf |Pi|) - 1 over all space-time elements (a
    time-constant field counts in every slab), and d chi / d rho_e (per
    space-time element) = v_e / (vf |Pi|)."""
    from .assemble import broadcast_elements
    r = broadcast_elements(grid, rho_phys)
    ve = grid.dx * grid.dx * grid.dt
    vol = ve * grid.n_elems
    chi = float(np.sum(r) * ve / (vf * vol) - 1.0)
    return chi, np.full(grid.shape_elems, ve / (vf * vol))


def physical_design(grid, rho, r_elems=None, beta=None, eta=0.5):
    """gamma -> filtered -> projected (each step optional); returns the
    physical field and the filtered field."""
    rho = np.asarray(rho, dtype=np.float64)
    if r_elems is not None:
        rt = filter_apply(rho, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    else:
        rt = rho
    rp = heaviside(rt, beta, eta) if beta else rt
    return rp, rt


def chain_to_design(grid, g_phys_elem, rho_shape, rt, r_elems=None, beta=None, eta=0.5):
    """Chain rule from a per-space-time-element sensitivity with respect to
    the physical field back to the design variables: extrusion sum, the
    projection derivative, the (symmetric) filter."""
    g = reduce_to_design(g_phys_elem, rho_shape)
    if beta:
        g = g * heaviside_deriv(rt, beta, eta)
    if r_elems is not None:
        g = filter_apply(g, grid.dx, grid.dt, r_elems * grid.dx, r_elems * grid.dt)
    return g


def pnorm_chain(grid, mat, rho, patches, P=20.0, q0=1.0, r_elems=None, beta=None, eta=0.5,
                vf=0.3, with_grad=True):
    """phi(gamma) and chi(gamma) with gradients: filter -> projection -> SIMP
    -> state -> p-norm -> adjoint with J^T lambda = dphi/ds (lambda = 0 on the
    Dirichlet set) -> element sensitivities -> chain rule (§3.3)."""
    from .assemble import simp, assemble_matrix, load_vector, apply_dirichlet
    from .grid import dirichlet_mask
    from .solve import solve_direct, solve_adjoint_direct
    rho = np.asarray(rho, dtype=np.float64)
    rp, rt = physical_design(grid, rho, r_elems, beta, eta)
    k, C, dk, dC = simp(rp, mat)
    mask = dirichlet_mask(grid, patches)
    f = load_vector(grid, q0)
    Jm, fm = apply_dirichlet(assemble_matrix(grid, k, C), f, mask)
    s = solve_direct(Jm, fm)
    phi, dphids = pnorm(grid, s, P)
    chi, dchi = volume(grid, rp, vf)
    out = dict(phi=phi, chi=chi, s=s, rho_phys=rp, dphids=dphids)
    if not with_grad:
        return out
    lam = solve_adjoint_direct(Jm, dphids, mask)
    ge = element_sensitivity(grid, s, lam, dk, dC)
    out.update(lam=lam,
               grad=chain_to_design(grid, ge, rho.shape, rt, r_elems, beta, eta),
               dchi=chain_to_design(grid, dchi, rho.shape, rt, r_elems, beta, eta))
    return out

"""Element matrices of the stabilised CG space-time discretisation (oracle).

Paper §3.1.1: the weak form multiplies the space-time heat equation by a
continuous test function and integrates the conduction term by parts; the
time direction receives an artificial diffusivity k_ad = C*dt/2 (element
Peclet number one).  With trilinear basis functions on a dx x dx x dt brick
the element matrix splits into a conduction part scaled by k_e and a capacity
part scaled by C_e:

    J_e = k_e * A + C_e * B

Two independent constructions are kept:
  element_matrices()          -- Kronecker products of 1-D matrices
  element_matrix_quadrature() -- 3x3x3 Gauss quadrature of the weak form itself

Index order of the 8x8 matrices: local node a = a1 + 2*a2 + 4*a3, which is
numpy's kron order (t, x2, x1).  Row = test function, column = trial function.
"""
import numpy as np


def mass_1d(h):
    """int_0^h N_a N_b for linear N."""
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


def stiff_1d(h):
    """int_0^h N_a' N_b' for linear N."""
    return 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])


def deriv_1d():
    """int_0^h N_a N_b' (test a, trial b); independent of h."""
    return 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])


def element_matrices(dx, dt):
    """Return (A, B): J_e = k_e*A + C_e*B.

    A = Mt (x) Mx (x) Sx + Mt (x) Sx (x) Mx         (conduction in x1 and x2)
    B = (G + (dt/2)*St) (x) Mx (x) Mx                (capacity + artificial diffusion)
    The artificial diffusion k_ad = C dt / 2 of §3.1.1 enters as C*(dt/2)*St.
    """
    Mx, Sx = mass_1d(dx), stiff_1d(dx)
    Mt, St = mass_1d(dt), stiff_1d(dt)
    G = deriv_1d()
    A = np.kron(Mt, np.kron(Mx, Sx)) + np.kron(Mt, np.kron(Sx, Mx))
    B = np.kron(G + 0.5 * dt * St, np.kron(Mx, Mx))
    return A, B


def _basis_1d(xi, h):
    """Linear shape functions and derivatives on [0, h] at points xi."""
    N = np.stack([1.0 - xi / h, xi / h])
    dN = np.stack([-np.ones_like(xi) / h, np.ones_like(xi) / h])
    return N, dN


def element_matrix_quadrature(dx, dt, k, C):
    """Brute-force 8x8 element matrix by 3-point Gauss quadrature per axis.

    Integrand (row a = test v, column b = trial T), §3.1.1 with the stabilised
    conductivity tensor diag(k, k, k_ad), k_ad = C*dt/2:
        C v dT/dt + k (dv/dx1 dT/dx1 + dv/dx2 dT/dx2) + k_ad dv/dt dT/dt
    """
    gp = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
    gw = np.array([5.0, 8.0, 5.0]) / 9.0
    kad = 0.5 * C * dt
    Jm = np.zeros((8, 8))
    for q1, w1 in zip(gp, gw):
        x1 = 0.5 * dx * (q1 + 1.0)
        for q2, w2 in zip(gp, gw):
            x2 = 0.5 * dx * (q2 + 1.0)
            for q3, w3 in zip(gp, gw):
                t = 0.5 * dt * (q3 + 1.0)
                wq = w1 * w2 * w3 * (0.5 * dx) * (0.5 * dx) * (0.5 * dt)
                N1, d1 = _basis_1d(np.array(x1), dx)
                N2, d2 = _basis_1d(np.array(x2), dx)
                N3, d3 = _basis_1d(np.array(t), dt)
                N = np.zeros(8)
                g1 = np.zeros(8)
                g2 = np.zeros(8)
                g3 = np.zeros(8)
                for a in range(8):
                    a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    N[a] = N1[a1] * N2[a2] * N3[a3]
                    g1[a] = d1[a1] * N2[a2] * N3[a3]
                    g2[a] = N1[a1] * d2[a2] * N3[a3]
                    g3[a] = N1[a1] * N2[a2] * d3[a3]
                Jm += wq * (C * np.outer(N, g3)
                            + k * (np.outer(g1, g1) + np.outer(g2, g2))
                            + kad * np.outer(g3, g3))
    return Jm


def element_load_weights(dx, dt):
    """int_e N_a dV for each local node a (= V_e / 8 for trilinear N)."""
    return np.full(8, dx * dx * dt / 8.0)


def element_mass(dx, dt):
    """Consistent space-time mass matrix int_e N_a N_b dV (8x8)."""
    return np.kron(mass_1d(dt), np.kron(mass_1d(dx), mass_1d(dx)))

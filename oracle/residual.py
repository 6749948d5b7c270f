"""Matrix-free application of the masked system and its residual (oracle).

For grids too large to assemble (hundreds of millions of nodes) the oracle
still checks a solution: it applies J_m = N J N + (I - N) slab by slab from
the same element matrices (§3.1.2, element-wise integration) and forms
f_m - J_m s, either for every node or for a sample of nodes.  The arithmetic
is the element matrices of element.py summed with numpy; nothing is shared
with the GPU library.
"""
import numpy as np

from .element import element_matrices


def _slab_coeff(field, s):
    f = np.asarray(field, dtype=np.float64)
    if f.ndim == 2:
        return f
    return f[0] if f.shape[0] == 1 else f[s]


def apply_masked(grid, k_e, C_e, mask, x, transpose=False):
    """y = J_m x (or J_m^T x), computed slab by slab."""
    A, B = element_matrices(grid.dx, grid.dt)
    nx, ny, nt = grid.nx, grid.ny, grid.nt
    X = np.asarray(x, dtype=np.float64).reshape(grid.shape_nodes)
    M = np.asarray(mask, dtype=bool).reshape(grid.shape_nodes)
    Xm = np.where(M, 0.0, X)
    Y = np.zeros_like(X)
    for s in range(nt):
        k = _slab_coeff(k_e, s)
        C = _slab_coeff(C_e, s)
        xe = np.empty((ny, nx, 8))
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            xe[:, :, a] = Xm[s + a3, a2:a2 + ny, a1:a1 + nx]
        if transpose:
            ye = k[:, :, None] * (xe @ A) + C[:, :, None] * (xe @ B)
        else:
            ye = k[:, :, None] * (xe @ A.T) + C[:, :, None] * (xe @ B.T)
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            Y[s + a3, a2:a2 + ny, a1:a1 + nx] += ye[:, :, a]
    Y = np.where(M, X, Y)
    return Y.ravel()


def residual_norm(grid, k_e, C_e, mask, s, f_m, transpose=False):
    """||f_m - J_m s||_2 / ||f_m||_2."""
    r = np.asarray(f_m).ravel() - apply_masked(grid, k_e, C_e, mask, s, transpose)
    return float(np.linalg.norm(r) / np.linalg.norm(f_m))


def apply_masked_at(grid, k_e, C_e, mask, x, nodes):
    """(J_m x)[a] for a list of flat node indices a, one node at a time from
    the (up to) 8 elements around it."""
    A, B = element_matrices(grid.dx, grid.dt)
    nx, ny, nt = grid.nx, grid.ny, grid.nt
    X = np.asarray(x, dtype=np.float64).reshape(grid.shape_nodes)
    M = np.asarray(mask, dtype=bool).reshape(grid.shape_nodes)
    out = np.zeros(len(nodes))
    for q, a_flat in enumerate(nodes):
        n, j, i = np.unravel_index(int(a_flat), grid.shape_nodes)
        if M[n, j, i]:
            out[q] = X[n, j, i]
            continue
        acc = 0.0
        for en in (n - 1, n):
            for ej in (j - 1, j):
                for ei in (i - 1, i):
                    if not (0 <= en < nt and 0 <= ej < ny and 0 <= ei < nx):
                        continue
                    k = _slab_coeff(k_e, en)[ej, ei]
                    C = _slab_coeff(C_e, en)[ej, ei]
                    la = (i - ei) + 2 * (j - ej) + 4 * (n - en)
                    row = k * A[la] + C * B[la]
                    for b in range(8):
                        b1, b2, b3 = b & 1, (b >> 1) & 1, (b >> 2) & 1
                        xn, xj, xi = en + b3, ej + b2, ei + b1
                        if not M[xn, xj, xi]:
                            acc += row[b] * X[xn, xj, xi]
        out[q] = acc
    return out


def residual_by_planes(grid, k_e, C_e, mask, x, f_m, transpose=False):
    """(||f_m - J_m x||_2, max_a |(f_m - J_m x)_a|) for the full grid, formed
    one time level at a time: slab s adds its element contributions to levels
    s and s + 1, after which level s is complete and its residual is folded
    into the sums.  Temporaries are two node planes, so grids of hundreds of
    millions of nodes fit; the arithmetic is that of apply_masked."""
    A, B = element_matrices(grid.dx, grid.dt)
    Ae, Be = (A, B) if transpose else (A.T, B.T)
    nx, ny, nt = grid.nx, grid.ny, grid.nt
    X = np.asarray(x, dtype=np.float64).reshape(grid.shape_nodes)
    M = np.asarray(mask, dtype=bool).reshape(grid.shape_nodes)
    F = np.asarray(f_m, dtype=np.float64).reshape(grid.shape_nodes)
    acc = np.zeros((2, ny + 1, nx + 1))
    ss, mx = 0.0, 0.0

    def fold(n, y):
        nonlocal ss, mx
        r = np.where(M[n], F[n] - X[n], F[n] - y)
        ss += float(np.sum(r * r))
        mx = max(mx, float(np.max(np.abs(r))))

    for s in range(nt):
        k = _slab_coeff(k_e, s)
        C = _slab_coeff(C_e, s)
        planes = (np.where(M[s], 0.0, X[s]), np.where(M[s + 1], 0.0, X[s + 1]))
        xe = np.empty((ny, nx, 8))
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            xe[:, :, a] = planes[a3][a2:a2 + ny, a1:a1 + nx]
        ye = k[:, :, None] * (xe @ Ae) + C[:, :, None] * (xe @ Be)
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            acc[a3, a2:a2 + ny, a1:a1 + nx] += ye[:, :, a]
        fold(s, acc[0])
        acc[0] = acc[1]
        acc[1] = 0.0
    fold(nt, acc[0])
    return float(np.sqrt(ss)), mx

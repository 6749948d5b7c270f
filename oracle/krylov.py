"""Krylov solvers and the V-cycle, written from their definitions (oracle).

Paper §3.2: FGMRES (Saad 1993) preconditioned by one space-time multigrid
V-cycle; Jacobi-preconditioned GMRES (Saad & Schultz 1986) is both the
smoother (at most 10 iterations, rtol 1e-6) and the coarsest-level solver (at
most 200 iterations, rtol 1e-6).

These functions exist to pin the GPU smoother and coarse solver one
application at a time and to give an iteration-count sanity band for the full
solve; the parity gate for solutions is the direct solve in solve.py.

Readings (the paper gives only the parameters above):
  * the smoother and coarse solver use left Jacobi preconditioning with
    classical Gram-Schmidt and stop when the preconditioned residual estimate
    falls below rtol times its value at the start of the call;
  * the coarse solver restarts every 30 iterations, the smoother never does;
  * pre-smoothing starts from zero, post-smoothing from the current iterate;
  * the outer FGMRES uses classical Gram-Schmidt with one re-orthogonalisation
    pass and stops on ||f - J s||_2 <= rtol ||f||_2.
The V-cycle can also solve the coarsest level exactly (sparse LU), the
variant the GPU library uses by default, and smooth with the s-step form of
the same GMRES minimisation (gmres_jacobi_sstep).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def gmres_jacobi(A, b, x0=None, maxit=10, rtol=1e-6, restart=None, dinv=None):
    """Left-Jacobi-preconditioned GMRES with classical Gram-Schmidt.

    Returns (x, iterations, final residual estimate / initial)."""
    n = b.shape[0]
    if dinv is None:
        dinv = 1.0 / A.diagonal()
    restart = maxit if restart is None else restart
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = dinv * (b - A @ x)
    beta = np.linalg.norm(r)
    beta0 = beta
    its = 0
    if beta0 == 0.0:
        return x, 0, 0.0
    while its < maxit:
        m = min(restart, maxit - its)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        done = False
        for j in range(m):
            w = dinv * (A @ V[j])
            h = V[:j + 1] @ w                      # all projections against the same w
            w = w - h @ V[:j + 1]
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):                     # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= rtol * beta0 or hn == 0.0:
                done = True
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + y @ V[:k]
        if done or its >= maxit:
            est = abs(g[k]) / beta0
            return x, its, est
        r = dinv * (b - A @ x)
        beta = np.linalg.norm(r)
        if beta == 0.0:
            return x, its, 0.0
    return x, its, beta / beta0


SSTEP_MIN_PIVOT = 1e-11
SSTEP_MAX_ITS = 10      # longer smoothings keep the Arnoldi form


def gmres_jacobi_sstep(A, b, x0=None, maxit=10, rtol=1e-6, dinv=None):
    """The Jacobi-GMRES smoother's minimisation written without Arnoldi:
    over x in x0 + K_m(M, r0), M = D^{-1} A, r0 = D^{-1}(b - A x0), minimise
    ||D^{-1}(b - A x)||_2.  With w_0 = r0 and w_{j+1} = M w_j (monomial
    basis) and x = x0 + sum_{j<m} y_j w_j the preconditioned residual is
    w_0 - sum_{j<m} y_j w_{j+1}, so y solves the normal equations
    G[1:m+1, 1:m+1] y = G[1:m+1, 0] of the Gram matrix G = W^T W and the
    squared residual is G[0,0] - y . G[1:m+1, 0].  m is the smallest count
    whose residual is <= rtol ||r0|| (the GMRES stopping rule), else maxit.
    In exact arithmetic this is GMRES(maxit) without restart, stopped by the
    same test.  The normal equations are factored one row at a time in the
    basis scaled to unit length; the pivot of row m is the squared sine of
    the angle between w_m and the earlier vectors.  A pivot below
    SSTEP_MIN_PIVOT stops at the vectors before it: either the space is
    invariant (the residual is already minimal) or the monomial basis has
    become too ill-conditioned for the equations to carry information (the
    pivots fall about tenfold per vector; below ~1e-11 they are rounding).

    Returns (x, m, residual / ||r0||)."""
    n = b.shape[0]
    if dinv is None:
        dinv = 1.0 / A.diagonal()
    x0 = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    W = np.zeros((maxit + 1, n))
    W[0] = dinv * (b - A @ x0)
    for j in range(maxit):
        W[j + 1] = dinv * (A @ W[j])
    G = W @ W.T
    g00 = G[0, 0]
    if g00 == 0.0:
        return x0, 0, 0.0
    # the equations are solved in the basis scaled to unit length (the
    # monomial vectors grow like the spectral radius of M)
    sc = np.zeros(maxit + 1)
    nz = np.diag(G) > 0
    sc[nz] = 1.0 / np.sqrt(np.diag(G)[nz])
    Gs = G * np.outer(sc, sc)
    # Cholesky factor L of Gs[1:, 1:], extended by one row per vector, and
    # z = L^{-1} Gs[1:, 0]; the squared residual with m vectors is 1 - |z[:m]|^2
    L = np.zeros((maxit, maxit))
    z = np.zeros(maxit)
    m, res2 = 0, 1.0
    for r in range(maxit):
        if not nz[r + 1]:
            break
        for c in range(r):
            L[r, c] = (Gs[r + 1, c + 1] - L[r, :c] @ L[c, :c]) / L[c, c]
        piv = Gs[r + 1, r + 1] - L[r, :r] @ L[r, :r]
        if not piv > SSTEP_MIN_PIVOT:
            break
        L[r, r] = np.sqrt(piv)
        z[r] = (Gs[r + 1, 0] - L[r, :r] @ z[:r]) / L[r, r]
        m = r + 1
        res2 = max(1.0 - z[:m] @ z[:m], 0.0)
        if res2 <= rtol * rtol:
            break
    ys = np.linalg.solve(L[:m, :m].T, z[:m]) if m else np.zeros(0)
    y = ys * sc[1:m + 1] / sc[0]
    return x0 + y @ W[:m], m, np.sqrt(res2)


class VCycle:
    """One classical V-cycle over the Galerkin hierarchy (§3.2).

    coarse="gmres": the coarsest level is solved with Jacobi-GMRES as in §3.2;
    coarse="direct": it is solved exactly (sparse LU of the coarsest operator).
    smoother="gmres": Jacobi-GMRES by Arnoldi; "sstep": the same minimisation
    through the Gram matrix of the monomial Krylov basis (gmres_jacobi_sstep)
    for smoothings of at most SSTEP_MAX_ITS iterations, Arnoldi beyond.
    """

    def __init__(self, A, Pm, smooth_its=10, smooth_rtol=1e-6, coarse_its=200,
                 coarse_rtol=1e-6, coarse_restart=30, coarse="gmres", smoother="gmres",
                 pre_its=None, post_its=None):
        if coarse not in ("gmres", "direct"):
            raise ValueError(coarse)
        if smoother not in ("gmres", "sstep"):
            raise ValueError(smoother)
        self.smoother = smoother
        self.A, self.Pm = A, Pm
        self.dinv = [1.0 / a.diagonal() for a in A]
        self.si, self.sr = smooth_its, smooth_rtol
        # pre- and post-smoothing iteration counts (0 skips that smoothing);
        # both default to smooth_its, the paper's symmetric cycle
        self.pre = smooth_its if pre_its is None else pre_its
        self.post = smooth_its if post_its is None else post_its
        self.ci, self.cr, self.crs = coarse_its, coarse_rtol, coarse_restart
        self.coarse = coarse
        self._lu = None

    def __call__(self, b, l=0):
        A, dinv = self.A[l], self.dinv[l]
        if l == len(self.A) - 1:
            if self.coarse == "direct":
                if self._lu is None:
                    self._lu = spla.splu(sp.csc_matrix(A))
                return self._lu.solve(np.asarray(b, dtype=np.float64))
            return gmres_jacobi(A, b, None, self.ci, self.cr, self.crs, dinv)[0]
        # pre-smoothing from x = 0, residual, restriction, coarse correction,
        # post-smoothing from the corrected iterate
        x = self._smooth(A, b, np.zeros(b.shape[0]), dinv, self.pre)
        r = b - A @ x
        xc = self(self.Pm[l].T @ r, l + 1)
        x = x + self.Pm[l] @ xc
        return self._smooth(A, b, x, dinv, self.post)

    def _smooth(self, A, b, x0, dinv, its):
        if its == 0:
            return x0
        if self.smoother == "sstep" and its <= SSTEP_MAX_ITS:
            return gmres_jacobi_sstep(A, b, x0, its, self.sr, dinv)[0]
        return gmres_jacobi(A, b, x0, its, self.sr, None, dinv)[0]


def fgmres(A, b, prec, m=30, rtol=1e-8, maxit=1000, x0=None):
    """Right-preconditioned flexible GMRES(m) (Saad 1993), CGS with one
    re-orthogonalisation.  Returns (x, iterations, true relative residual)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    r = b - A @ x
    beta = np.linalg.norm(r)
    its = 0
    while its < maxit and beta > rtol * nb:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = A @ Z[j]
            h1 = V[:j + 1] @ w
            w = w - h1 @ V[:j + 1]
            h2 = V[:j + 1] @ w
            w = w - h2 @ V[:j + 1]
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h1 + h2
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= rtol * nb or hn == 0.0 or its >= maxit:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + y @ Z[:k]
        r = b - A @ x
        beta = np.linalg.norm(r)
    return x, its, beta / nb

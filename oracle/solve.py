"""Direct solves of the masked space-time system (oracle).

The method of the paper (§3.2) reaches the exact discrete solution of the
Dirichlet-eliminated system J s = f; the oracle computes that solution
directly, in FP64, two ways:

  solve_direct   -- global sparse LU (SuperLU) + iterative refinement
  BlockTimeSystem.gauss_seidel
                 -- block Gauss-Seidel over time levels; each diagonal block
                    (one time level of nodes) is solved exactly by sparse LU.
                    Every block is assembled from the same element matrices as
                    the global matrix, slab by slab.  Used where a global LU
                    does not fit.

Adjoints (§3.3.3, J^T lambda = dphi/ds, lambda = 0 on Dirichlet nodes) use the
transposed matrix with the same two routes.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import element_matrices


def solve_direct(Jm, fm, tol=1e-14, max_refine=10):
    """Sparse LU of Jm plus iterative refinement until ||f - J s|| <= tol*||f|| (the
    residual floors near 1e-14 relative in FP64, so refinement stops there)."""
    lu = spla.splu(sp.csc_matrix(Jm))
    s = lu.solve(fm)
    nf = np.linalg.norm(fm)
    for _ in range(max_refine):
        r = fm - Jm @ s
        if np.linalg.norm(r) <= tol * nf:
            break
        s = s + lu.solve(r)
    return s


def solve_adjoint_direct(Jm, g, mask, tol=1e-14):
    """Solve Jm^T lam = N g (lam = 0 on Dirichlet nodes), §3.3.3."""
    m = np.asarray(mask, dtype=bool).ravel()
    rhs = np.where(m, 0.0, np.asarray(g, dtype=np.float64).ravel())
    return solve_direct(sp.csr_matrix(Jm.T), rhs, tol=tol)


class BlockTimeSystem:
    """Block-tridiagonal-in-time view of the masked system.

    Slab s (elements between levels s and s+1) gives a two-level matrix
        [[Bbb, Bbt], [Btb, Btt]]
    from its element matrices; the block row of level n is
        A[n,n-1] = Btb(n-1),  A[n,n] = Btt(n-1) + Bbb(n),  A[n,n+1] = Bbt(n).
    Dirichlet rows become identity rows and Dirichlet columns are zeroed.
    """

    def __init__(self, grid, k_e, C_e, mask):
        from .assemble import broadcast_elements
        self.g = grid
        self.P = (grid.nx + 1) * (grid.ny + 1)
        self.mask = np.asarray(mask, dtype=bool).reshape(grid.shape_nodes)
        k = broadcast_elements(grid, k_e)
        C = broadcast_elements(grid, C_e)
        self.A, self.B = element_matrices(grid.dx, grid.dt)
        # Slabs with identical coefficient planes share their matrices.
        self._slab_cache = {}
        self._slab_key = []
        for s in range(grid.nt):
            key = (k[s].tobytes(), C[s].tobytes())
            if key not in self._slab_cache:
                self._slab_cache[key] = self._slab_blocks(k[s], C[s])
            self._slab_key.append(key)
        self._lu = {}
        self._blk = {}
        # Time levels whose Dirichlet rows coincide share one mask id.
        ids = {}
        self._mask_id = []
        for n in range(grid.nt + 1):
            key = self.mask[n].tobytes()
            self._mask_id.append(ids.setdefault(key, len(ids)))

    def _slab_blocks(self, k2, C2):
        g = self.g
        nx, ny, P = g.nx, g.ny, self.P
        j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        j, i = j.ravel(), i.ravel()
        loc = np.empty((nx * ny, 8), dtype=np.int64)
        for a in range(8):
            a1, a2, a3 = a & 1, (a >> 1) & 1, (a >> 2) & 1
            loc[:, a] = a3 * P + (j + a2) * (nx + 1) + (i + a1)
        vals = k2.ravel()[:, None, None] * self.A[None] + C2.ravel()[:, None, None] * self.B[None]
        rows = np.repeat(loc[:, :, None], 8, axis=2).ravel()
        cols = np.repeat(loc[:, None, :], 8, axis=1).ravel()
        S = sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(2 * P, 2 * P)).tocsr()
        return (S[:P, :P], S[:P, P:], S[P:, :P], S[P:, P:])  # bb, bt, tb, tt

    def _slab(self, s):
        return self._slab_cache[self._slab_key[s]]

    def block(self, n, m, masked=True):
        """Block A[n, m] (m in n-1, n, n+1) as CSR (cached by content)."""
        g = self.g
        kb = self._slab_key[n - 1] if 1 <= n <= g.nt else None
        ka = self._slab_key[n] if 0 <= n < g.nt else None
        ck = (m - n, kb, ka, self._mask_id[n], self._mask_id[m] if 0 <= m <= g.nt else -1, masked)
        if ck not in self._blk:
            self._blk[ck] = self._block_uncached(n, m, masked)
        return self._blk[ck]

    def _block_uncached(self, n, m, masked):
        g, P = self.g, self.P
        Z = sp.csr_matrix((P, P))
        if m == n - 1:
            blk = self._slab(n - 1)[2] if n >= 1 else Z
        elif m == n + 1:
            blk = self._slab(n)[1] if n < g.nt else Z
        elif m == n:
            blk = Z
            if n >= 1:
                blk = blk + self._slab(n - 1)[3]
            if n < g.nt:
                blk = blk + self._slab(n)[0]
        else:
            return Z
        if not masked:
            return sp.csr_matrix(blk)
        Nr = sp.diags((~self.mask[n]).ravel().astype(np.float64))
        Nc = sp.diags((~self.mask[m]).ravel().astype(np.float64))
        out = Nr @ blk @ Nc
        if m == n:
            out = out + sp.diags(self.mask[n].ravel().astype(np.float64))
        return sp.csr_matrix(out)

    def matvec(self, x, masked=True, transpose=False):
        g, P = self.g, self.P
        X = np.asarray(x, dtype=np.float64).reshape(g.nt + 1, P)
        Y = np.zeros_like(X)
        for n in range(g.nt + 1):
            for m in (n - 1, n, n + 1):
                if 0 <= m <= g.nt:
                    if transpose:
                        Y[n] += self.block(m, n, masked).T @ X[m]
                    else:
                        Y[n] += self.block(n, m, masked) @ X[m]
        return Y.ravel()

    def masked_rhs(self, f, gvals=None):
        """f_m = N (f - J g) + g with the unmasked blocks (see assemble.apply_dirichlet)."""
        m = self.mask.ravel()
        f = np.asarray(f, dtype=np.float64).ravel()
        if gvals is None:
            return np.where(m, 0.0, f)
        gv = np.where(m, np.asarray(gvals, dtype=np.float64).ravel(), 0.0)
        Jg = self.matvec(gv, masked=False)
        return np.where(m, gv, f - Jg)

    def _diag_lu(self, n, transpose):
        # Identical diagonal blocks (time-constant coefficients) share one LU.
        g = self.g
        kb = self._slab_key[n - 1] if n >= 1 else None
        ka = self._slab_key[n] if n < g.nt else None
        ck = (kb, ka, self._mask_id[n], transpose)
        if ck not in self._lu:
            D = self.block(n, n)
            self._lu[ck] = spla.splu(sp.csc_matrix(D.T if transpose else D))
        return self._lu[ck]

    def gauss_seidel(self, fm, tol=1e-13, max_sweeps=200, transpose=False, x0=None, log=None):
        """Block GS sweeps (forward in time; backward for the transpose) until
        ||fm - A s|| <= tol*||fm||.  Returns (s, sweeps, rel_res).  log: a
        callable that receives (sweep, rel_res) after every sweep."""
        g, P = self.g, self.P
        F = np.asarray(fm, dtype=np.float64).reshape(g.nt + 1, P)
        S = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.float64).reshape(g.nt + 1, P)
        nf = np.linalg.norm(F)
        order = range(g.nt, -1, -1) if transpose else range(0, g.nt + 1)
        tcache = {}

        def off(n, m):
            if not transpose:
                return self.block(n, m)
            b = self.block(m, n)
            if id(b) not in tcache:
                tcache[id(b)] = sp.csr_matrix(b.T)
            return tcache[id(b)]
        rel = np.inf
        for sweep in range(1, max_sweeps + 1):
            for n in order:
                rhs = F[n].copy()
                for m in (n - 1, n + 1):
                    if 0 <= m <= g.nt:
                        rhs -= off(n, m) @ S[m]
                S[n] = self._diag_lu(n, transpose).solve(rhs)
            r = F.ravel() - self.matvec(S.ravel(), transpose=transpose)
            rel = np.linalg.norm(r) / nf if nf > 0 else np.linalg.norm(r)
            if log is not None:
                log(sweep, rel)
            if rel <= tol:
                return S.ravel(), sweep, rel
        return S.ravel(), max_sweeps, rel

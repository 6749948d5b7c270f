"""Python face of the space-time solver: a thin wrapper over include/st_api.h.

PyTorch supplies device memory (one workspace tensor per problem, plus the
caller's input/output tensors) and the HIP stream; every computation happens
in libst.so.
"""
import ctypes as C

import torch

from . import _lib as L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(x, device):
    t = torch.as_tensor(x, dtype=torch.float64)
    return t.to(device=device).contiguous()


class Problem:
    """One space-time problem (grid, material, design, boundary conditions)
    with its multigrid hierarchy resident on the GPU.

    rho: [ny, nx] or [1, ny, nx] (time-constant design) or [nt, ny, nx].
    patches: iterable of (edge, centre, half_width) T = 0 patches.
    coarse: "direct" (exact block-tridiagonal solve on the coarsest level) or
    "gmres" (the paper's Jacobi-GMRES coarse solve, §3.2).
    coarsening: "semi" (Algorithm 1) or "full" (every level halves space and
    time, the comparison of §5.1.2).
    smoother: "gmres" (Jacobi-GMRES by Arnoldi, §3.2) or "sstep" (the same
    minimisation from the Gram matrix of the monomial Krylov basis).
    orthogonalisation: outer FGMRES basis by "delayed" CGS2 (two passes per
    step) or "classical" CGS2 (three).
    """

    def __init__(self, nx, ny, nt, rho, dx=None, dt=None, k_ins=1e-3, k_con=1.0, p_k=3.0,
                 c_ins=1.0, c_con=1.0, p_c=1.0, patches=((0, 0.5, 0.05),), q0=1.0, ic=None,
                 source=None, precision="fp64", filter_r=0.0, device="cuda", stream=None,
                 time_kernels=False, coarse="direct", coarsening="semi", smoother="gmres",
                 orthogonalisation="delayed", **opt_overrides):
        self.lib = L.load()
        self.device = torch.device(device)
        self.nx, self.ny, self.nt = int(nx), int(ny), int(nt)
        dx = 1.0 / max(nx, ny) if dx is None else float(dx)
        dt = 1.0 / nt if dt is None else float(dt)
        self.grid = L.st_grid(self.nx, self.ny, self.nt, dx, dt)
        self.mat = L.st_material(k_ins, k_con, p_k, c_ins, c_con, p_c)
        rho = _dev_f64(rho, self.device)
        if rho.dim() == 2:
            rho = rho.unsqueeze(0)
        if rho.shape[1:] != (self.ny, self.nx) or rho.shape[0] not in (1, self.nt):
            raise ValueError(f"rho shape {tuple(rho.shape)} does not match grid")
        self.rho_tv = 1 if (rho.shape[0] == self.nt and self.nt > 1) else 0
        if self.rho_tv == 0 and rho.shape[0] != 1:
            rho = rho[:1].contiguous()
        self.design_shape = tuple(rho.shape)
        self.opts = L.default_opts()
        self.opts.precision = L.ST_MIXED if precision == "mixed" else L.ST_FP64
        self.opts.filter_r = float(filter_r)
        if time_kernels:
            self.opts.flags |= L.ST_FLAG_TIME_KERNELS
        if coarse not in ("direct", "gmres"):
            raise ValueError(f"coarse must be 'direct' or 'gmres', not {coarse!r}")
        if coarse == "gmres":
            self.opts.flags |= L.ST_FLAG_COARSE_GMRES
        if coarsening not in ("semi", "full"):
            raise ValueError(f"coarsening must be 'semi' or 'full', not {coarsening!r}")
        if coarsening == "full":
            self.opts.flags |= L.ST_FLAG_FULL_COARSENING
        if smoother not in ("gmres", "sstep"):
            raise ValueError(f"smoother must be 'gmres' or 'sstep', not {smoother!r}")
        if smoother == "sstep":
            self.opts.flags |= L.ST_FLAG_SSTEP_SMOOTHER
        if orthogonalisation not in ("delayed", "classical"):
            raise ValueError("orthogonalisation must be 'delayed' or 'classical', "
                             f"not {orthogonalisation!r}")
        if orthogonalisation == "classical":
            self.opts.flags |= L.ST_FLAG_OUTER_CGS2
        for k, v in opt_overrides.items():
            if not hasattr(self.opts, k):
                raise KeyError(k)
            setattr(self.opts, k, v)
        pl = list(patches)
        parr = (L.st_patch * max(1, len(pl)))()
        for i, (e, c, hw) in enumerate(pl):
            parr[i] = L.st_patch(int(e), float(c), float(hw))
        nbytes = C.c_size_t(0)
        L.check("st_footprint_bytes", self.lib.st_footprint_bytes(
            C.byref(self.grid), C.byref(self.mat), C.byref(self.opts), self.rho_tv, C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                         device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.density_version = 0
        icd = _dev_f64(ic, self.device).reshape(-1) if ic is not None else None
        srcd = _dev_f64(source, self.device).reshape(-1) if source is not None else None
        h = C.c_void_p()
        self._order()
        code = self.lib.st_setup(C.byref(self.grid), C.byref(self.mat), _ptr(rho), self.rho_tv,
                                 _ptr(icd), _ptr(srcd), float(q0), parr, len(pl),
                                 C.byref(self.opts), _ptr(self.workspace),
                                 self.workspace_bytes + 256, C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h))
        if code == L.ST_NOT_CONVERGED:          # the density filter reached its cap
            self.lib.st_destroy(h)
        L.check("st_setup", code)
        self.h = h
        self.n_nodes = (self.nx + 1) * (self.ny + 1) * (self.nt + 1)

    # ------------------------------------------------------------------
    def _order(self):
        """Inputs are made (allocated, zeroed, copied) on torch's current
        stream; the library reads them on the problem's stream.  Make the
        latter wait for the former.  Every entry point synchronises its own
        stream before returning, so outputs need no ordering back."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _new_nodal(self):
        return torch.zeros((self.nt + 1, self.ny + 1, self.nx + 1), dtype=torch.float64,
                           device=self.device)

    def solve(self, x0=None, allow_not_converged=False):
        """Forward solve; returns (T [nt+1, ny+1, nx+1], info)."""
        T = self._new_nodal() if x0 is None else _dev_f64(x0, self.device).clone().reshape(
            self.nt + 1, self.ny + 1, self.nx + 1)
        info = L.st_info()
        self._order()
        code = self.lib.st_solve(self.h, _ptr(T), C.byref(info))
        L.check("st_solve", code, allow_not_converged)
        return T, info

    def adjoint(self, g, lam0=None, allow_not_converged=False):
        g = _dev_f64(g, self.device).reshape(self.nt + 1, self.ny + 1, self.nx + 1)
        lam = self._new_nodal() if lam0 is None else _dev_f64(lam0, self.device).clone().reshape(
            self.nt + 1, self.ny + 1, self.nx + 1)
        info = L.st_info()
        self._order()
        code = self.lib.st_adjoint_solve(self.h, _ptr(g), _ptr(lam), C.byref(info))
        L.check("st_adjoint_solve", code, allow_not_converged)
        return lam, info

    def sensitivity(self, T, lam):
        out = torch.empty(self.design_shape, dtype=torch.float64, device=self.device)
        T = _dev_f64(T, self.device)
        lam = _dev_f64(lam, self.device)
        self._order()
        L.check("st_sensitivity", self.lib.st_sensitivity(self.h, _ptr(T), _ptr(lam), _ptr(out)))
        return out

    def objective(self, T):
        J = C.c_double(0.0)
        T = _dev_f64(T, self.device)
        self._order()
        L.check("st_objective", self.lib.st_objective(self.h, _ptr(T), C.byref(J)))
        return J.value

    def pnorm(self, T, P=20.0, grad=True):
        """p-norm objective (§3.3.1) of the state T: (phi, dphi/dT or None)."""
        T = _dev_f64(T, self.device)
        phi = C.c_double(0.0)
        g = self._new_nodal() if grad else None
        self._order()
        L.check("st_pnorm", self.lib.st_pnorm(self.h, _ptr(T), float(P), C.byref(phi),
                                              _ptr(g) if grad else None))
        return phi.value, g

    def volume(self, vf, grad=True):
        """Volume constraint (§3.3.1) of the physical design: (chi, dchi/drho or
        None), the gradient in the design's layout."""
        chi = C.c_double(0.0)
        g = torch.empty(self.design_shape, dtype=torch.float64, device=self.device) if grad else None
        self._order()
        L.check("st_volume", self.lib.st_volume(self.h, float(vf), C.byref(chi),
                                                _ptr(g) if grad else None))
        return chi.value, g

    def load_vector(self):
        f = self._new_nodal()
        self._order()
        L.check("st_load_vector", self.lib.st_load_vector(self.h, _ptr(f)))
        return f

    def filter(self, x):
        x = _dev_f64(x, self.device).reshape(self.design_shape)
        out = torch.empty_like(x)
        self._order()
        L.check("st_filter", self.lib.st_filter(self.h, _ptr(x), _ptr(out)))
        return out

    def update_density(self, rho):
        rho = _dev_f64(rho, self.device).reshape(self.design_shape)
        self._order()
        L.check("st_update_density", self.lib.st_update_density(self.h, _ptr(rho)))
        self.density_version += 1

    def set_stream(self, stream):
        L.check("st_set_stream", self.lib.st_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def set_flags(self, flags):
        L.check("st_set_flags", self.lib.st_set_flags(self.h, int(flags)))

    def hierarchy(self):
        info = L.st_info()
        L.check("st_hierarchy", self.lib.st_hierarchy(self.h, C.byref(info)))
        return [tuple(info.level_dims[l]) for l in range(info.levels)], \
            [info.level_planes[l] for l in range(info.levels)]

    # ---- single pieces, for tests --------------------------------------
    def level_shape(self, level):
        dims, _ = self.hierarchy()
        nx, ny, nt = dims[level]
        return (nt + 1, ny + 1, nx + 1)

    def debug_apply(self, level, x, transpose=False, mixed=False):
        x = _dev_f64(x, self.device)
        y = torch.empty_like(x)
        self._order()
        L.check("st_debug_apply", self.lib.st_debug_apply(
            self.h, level, int(transpose), L.ST_MIXED if mixed else L.ST_FP64, _ptr(x), _ptr(y)))
        return y

    def debug_stencil(self, level):
        shp = self.level_shape(level)
        out = torch.empty((27,) + shp, dtype=torch.float64, device=self.device)
        self._order()
        L.check("st_debug_stencil", self.lib.st_debug_stencil(self.h, level, _ptr(out)))
        return out

    def debug_diag(self, level):
        shp = self.level_shape(level)
        d = torch.empty(shp, dtype=torch.float64, device=self.device)
        m = torch.empty(shp, dtype=torch.uint8, device=self.device)
        self._order()
        L.check("st_debug_diag", self.lib.st_debug_diag(self.h, level, _ptr(d), _ptr(m)))
        return d, m

    def debug_transfer(self, level, x, prolong):
        x = _dev_f64(x, self.device)
        shp = self.level_shape(level if prolong else level + 1)
        out = torch.empty(shp, dtype=torch.float64, device=self.device)
        self._order()
        L.check("st_debug_transfer", self.lib.st_debug_transfer(
            self.h, level, int(prolong), _ptr(x), _ptr(out)))
        return out

    def debug_smooth(self, level, b, x0=None, its=10, rtol=1e-6, transpose=False):
        b = _dev_f64(b, self.device)
        x = torch.zeros_like(b) if x0 is None else _dev_f64(x0, self.device).clone()
        self._order()
        L.check("st_debug_smooth", self.lib.st_debug_smooth(
            self.h, level, int(transpose), _ptr(b), _ptr(x), int(x0 is None), its, rtol))
        return x

    def debug_vcycle(self, b, transpose=False):
        b = _dev_f64(b, self.device)
        x = torch.empty_like(b)
        self._order()
        L.check("st_debug_vcycle", self.lib.st_debug_vcycle(self.h, int(transpose), _ptr(b),
                                                            _ptr(x)))
        return x

    def close(self):
        if getattr(self, "h", None):
            self.lib.st_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def info_dict(info):
    """Plain-Python view of an st_info."""
    d = dict(iterations=info.iterations, restarts=info.restarts, levels=info.levels,
             rel_res_est=info.rel_res_est, true_rel_res=info.true_rel_res,
             t_solve_s=info.t_solve_s, res_hist=[info.res_hist[i] for i in range(info.n_hist)])
    d["kernels"] = {L.KCLASS_NAMES[c]: dict(ms=info.kclass_ms[c], launches=info.kclass_launches[c],
                                            bytes=info.kclass_bytes[c])
                    for c in range(L.ST_NUM_KCLASS) if info.kclass_launches[c]}
    return d


def _reload_if_changed(problem, version, rho):
    """The adjoint operator and the sensitivities belong to the design a
    forward call loaded.  If the problem has been given another design since
    (a second forward call on the same problem, or update_density), load that
    forward call's design again before the backward solve; the problem then
    holds it."""
    if problem.density_version != version:
        problem.update_density(rho.detach())


class STSolve(torch.autograd.Function):
    """T = STSolve.apply(rho, problem): the design is loaded into the problem
    (filter + SIMP + Galerkin rebuild), the state solved; the backward pass is
    one adjoint solve plus the sensitivity kernel (§3.3.3)."""

    @staticmethod
    def forward(ctx, rho, problem):
        problem.update_density(rho.detach())
        T, _ = problem.solve()
        ctx.problem = problem
        ctx.version = problem.density_version
        ctx.save_for_backward(T, rho)
        return T

    @staticmethod
    def backward(ctx, gT):
        problem = ctx.problem
        T, rho = ctx.saved_tensors
        _reload_if_changed(problem, ctx.version, rho)
        lam, _ = problem.adjoint(gT.contiguous())
        grad = problem.sensitivity(T, lam)
        return grad.reshape(problem.design_shape), None


class STPNorm(torch.autograd.Function):
    """phi = STPNorm.apply(rho, problem, P): design -> (filter, projection,
    SIMP, Galerkin rebuild) -> state -> p-norm of the element-averaged
    temperature (§3.3.1).  Backward: one adjoint solve with the right-hand
    side dphi/dT, the sensitivity kernel and the chain rule (§3.3.3)."""

    @staticmethod
    def forward(ctx, rho, problem, P=20.0):
        problem.update_density(rho.detach())
        T, _ = problem.solve()
        phi, dphi = problem.pnorm(T, P)
        ctx.problem = problem
        ctx.version = problem.density_version
        ctx.save_for_backward(T, dphi, rho)
        return torch.tensor(phi, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, gphi):
        problem = ctx.problem
        T, dphi, rho = ctx.saved_tensors
        _reload_if_changed(problem, ctx.version, rho)
        lam, _ = problem.adjoint(dphi)
        grad = problem.sensitivity(T, lam)
        return gphi * grad.reshape(problem.design_shape), None, None


class STObjective(torch.autograd.Function):
    """J = f^T T (int Q T dV) computed by the library; dJ/dT = f."""

    @staticmethod
    def forward(ctx, T, problem):
        ctx.problem = problem
        return torch.tensor(problem.objective(T), dtype=torch.float64, device=T.device)

    @staticmethod
    def backward(ctx, gJ):
        f = ctx.problem.load_vector()
        return gJ * f, None

"""st_solve_noalloc (static device scratch, no allocation) against the
caller-workspace entry points st_setup + st_solve on the same inputs: two
calls in a row, the second on a smaller grid, each equal to the existing
path's solution (bitwise: same kernels, same reduction trees) and to the
oracle's direct solve to 1e-10; a problem over the scratch size is refused
before any GPU work."""
import ctypes as C

import numpy as np
import pytest

from oracle.assemble import assemble_matrix, apply_dirichlet, load_vector
from oracle.grid import Grid, dirichlet_mask
from oracle.solve import solve_direct

pytestmark = pytest.mark.gpu
PATCH = (0, 0.5, 0.05)


def _noalloc(n, nt, rho, precision, T0=None):
    import torch
    from paper_2508_09589_amd import _lib as L
    lib = L.load()
    g = L.st_grid(n, n, nt, 1.0 / n, 1.0 / nt)
    m = L.st_material(1e-3, 1.0, 3.0, 1.0, 1.0, 1.0)
    o = L.default_opts()
    o.precision = L.ST_MIXED if precision == "mixed" else L.ST_FP64
    o.rtol = 1e-12
    if precision == "mixed":
        o.bf16_from_level = 1
    o.flags |= L.ST_FLAG_SSTEP_SMOOTHER
    r = torch.tensor(rho, dtype=torch.float64, device="cuda").contiguous()
    T = torch.zeros((nt + 1, n + 1, n + 1), dtype=torch.float64, device="cuda")
    parr = (L.st_patch * 1)(L.st_patch(*PATCH))
    info = L.st_info()
    torch.cuda.synchronize()
    rc = lib.st_solve_noalloc(C.byref(g), C.byref(m), C.c_void_p(r.data_ptr()),
                              1 if rho.ndim == 3 else 0, None, None, 1.0, parr, 1, C.byref(o),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream),
                              C.c_void_p(T.data_ptr()), C.byref(info))
    return rc, T, info


def _reference(n, nt, rho, precision):
    import torch
    from paper_2508_09589_amd import Problem
    kw = dict(bf16_from_level=1) if precision == "mixed" else {}
    p = Problem(n, n, nt, torch.tensor(rho), precision=precision, rtol=1e-12, smoother="sstep",
                **kw)
    T, info = p.solve()
    p.close()
    return T, info


def _oracle(n, nt, rho):
    g = Grid(n, n, nt, 1.0 / n, 1.0 / nt)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    if k.ndim == 2:
        k = np.broadcast_to(k, (nt, n, n)).copy()
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0),
                             dirichlet_mask(g, [PATCH]))
    return solve_direct(Jm, fm)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_workspace_path_twice(require_gpu, precision):
    import torch
    from paper_2508_09589_amd import _lib as L
    rng = np.random.default_rng(3)
    cases = [(24, 32, rng.uniform(0.001, 1.0, (32, 24, 24))),
             (16, 8, rng.uniform(0.001, 1.0, (16, 16)))]
    for n, nt, rho in cases:
        print(f"noalloc {precision} {n}^2 x {nt}", flush=True)
        rc, T, info = _noalloc(n, nt, rho, precision)
        assert rc == L.ST_OK, L.status_string(rc)
        Tr, ir = _reference(n, nt, rho, precision)
        assert info.iterations == ir.iterations
        assert torch.equal(T, Tr), float((T - Tr).abs().max())
        s = _oracle(n, nt, rho)
        err = np.linalg.norm(T.cpu().numpy().ravel() - s) / np.linalg.norm(s)
        assert err <= 1e-10, err


def test_noalloc_refuses_problems_over_the_scratch(require_gpu):
    from paper_2508_09589_amd import _lib as L
    n, nt = 128, 256
    rho = np.full((n, n), 0.5)
    rc, T, info = _noalloc(n, nt, rho, "fp64")
    assert rc == L.ST_ERR_OOM
    assert float(T.abs().max()) == 0.0

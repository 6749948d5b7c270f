"""Failure behaviour on the GPU, forced from the host: an iteration cap that
stops FGMRES early, a non-finite density, a filter whose CG reaches its cap,
and a workspace smaller than the footprint.  Every kernel still runs to its
normal end; the conditions come from the arguments."""
import ctypes as C

import numpy as np
import pytest

from oracle.assemble import assemble_matrix, apply_dirichlet, load_vector
from oracle.grid import Grid, dirichlet_mask

pytestmark = pytest.mark.gpu
PATCH = [(0, 0.5, 0.05)]


@pytest.fixture(scope="module")
def torch_cuda(require_gpu):
    import torch
    return torch


def test_iteration_cap_returns_not_converged_with_iterate(torch_cuda):
    """max_it = 1: st_solve returns ST_NOT_CONVERGED, reports one iteration,
    and writes the iterate whose true residual it reports (checked with the
    oracle's assembled matrix)."""
    import torch
    from paper_2508_09589_amd import Problem, _lib as L
    n, nt = 16, 16
    rho = np.random.default_rng(2).uniform(0.001, 1.0, (n, n))
    p = Problem(n, n, nt, torch.tensor(rho), max_it=1)
    with pytest.raises(L.StError) as ei:
        p.solve()
    assert ei.value.code == L.ST_NOT_CONVERGED
    T, info = p.solve(allow_not_converged=True)
    assert info.iterations == 1
    g = Grid(n, n, nt, 1 / n, 1 / nt)
    k = 1e-3 + (1 - 1e-3) * rho ** 3
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g, 1.0),
                             dirichlet_mask(g, PATCH))
    r = np.linalg.norm(fm - Jm @ T.cpu().numpy().ravel()) / np.linalg.norm(fm)
    assert 1e-8 < r < 1.0
    assert abs(r - info.true_rel_res) <= 1e-8 * r
    lam, ainfo = p.adjoint(p.load_vector(), allow_not_converged=True)
    assert ainfo.iterations == 1 and 1e-8 < ainfo.true_rel_res < 1.0
    p.close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_density_is_rejected(torch_cuda, bad):
    import torch
    from paper_2508_09589_amd import Problem, _lib as L
    n, nt = 8, 8
    rho = np.full((nt, n, n), 0.5)
    rho[3, 2, 5] = bad
    with pytest.raises(L.StError) as ei:
        Problem(n, n, nt, torch.tensor(rho))
    assert ei.value.code == L.ST_ERR_ARG
    p = Problem(n, n, nt, torch.tensor(np.full((nt, n, n), 0.5)))
    with pytest.raises(L.StError) as ei:
        p.update_density(torch.tensor(rho))
    assert ei.value.code == L.ST_ERR_ARG
    # a finite design makes the handle usable again
    p.update_density(torch.tensor(np.full((nt, n, n), 0.5)))
    T, info = p.solve()
    assert info.true_rel_res <= 1e-8
    p.close()


def test_filter_cap_returns_not_converged(torch_cuda):
    """A density filter limited to 2 CG iterations: st_setup returns
    ST_NOT_CONVERGED (the Python wrapper raises it), and a direct st_setup
    call yields a usable handle whose st_filter also reports it."""
    import torch
    from paper_2508_09589_amd import Problem, _lib as L
    n, nt = 12, 10
    rho = np.random.default_rng(4).uniform(0.0, 1.0, (nt, n, n))
    with pytest.raises(L.StError) as ei:
        Problem(n, n, nt, torch.tensor(rho), filter_r=1.5, filter_max_it=2)
    assert ei.value.code == L.ST_NOT_CONVERGED
    lib = L.load()
    g = L.st_grid(n, n, nt, 1.0 / n, 1.0 / nt)
    m = L.st_material(1e-3, 1.0, 3.0, 1.0, 1.0, 1.0)
    o = L.default_opts()
    o.filter_r, o.filter_max_it = 1.5, 2
    b = C.c_size_t(0)
    assert lib.st_footprint_bytes(C.byref(g), C.byref(m), C.byref(o), 1, C.byref(b)) == 0
    ws = torch.empty(b.value + 256, dtype=torch.uint8, device="cuda")
    r = torch.tensor(rho, device="cuda")
    parr = (L.st_patch * 1)(L.st_patch(0, 0.5, 0.05))
    h = C.c_void_p()
    torch.cuda.synchronize()
    rc = lib.st_setup(C.byref(g), C.byref(m), C.c_void_p(r.data_ptr()), 1, None, None, 1.0,
                      parr, 1, C.byref(o), C.c_void_p(ws.data_ptr()), b.value + 256,
                      C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h))
    assert rc == L.ST_NOT_CONVERGED and h.value
    out = torch.empty_like(r)
    assert lib.st_filter(h, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr())) == \
        L.ST_NOT_CONVERGED
    assert torch.isfinite(out).all()
    lib.st_destroy(h)
    # with the default cap the same design filters to convergence
    p = Problem(n, n, nt, torch.tensor(rho), filter_r=1.5)
    p.filter(torch.tensor(rho))
    p.close()


def test_workspace_smaller_than_footprint_is_rejected(torch_cuda):
    import torch
    from paper_2508_09589_amd import _lib as L
    lib = L.load()
    n, nt = 8, 8
    g = L.st_grid(n, n, nt, 1.0 / n, 1.0 / nt)
    m = L.st_material(1e-3, 1.0, 3.0, 1.0, 1.0, 1.0)
    o = L.default_opts()
    b = C.c_size_t(0)
    assert lib.st_footprint_bytes(C.byref(g), C.byref(m), C.byref(o), 0, C.byref(b)) == 0
    ws = torch.empty(b.value // 2, dtype=torch.uint8, device="cuda")
    r = torch.full((1, n, n), 0.5, dtype=torch.float64, device="cuda")
    h = C.c_void_p()
    rc = lib.st_setup(C.byref(g), C.byref(m), C.c_void_p(r.data_ptr()), 0, None, None, 1.0, None,
                      0, C.byref(o), C.c_void_p(ws.data_ptr()), b.value // 2, None, C.byref(h))
    assert rc == L.ST_ERR_OOM and not h.value

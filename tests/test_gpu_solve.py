"""GPU parity of complete solves against the FP64 oracle, plus closed forms
that hold at any size."""
import numpy as np
import pytest

from oracle.solve import solve_direct, solve_adjoint_direct
from tests._cases import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda(require_gpu):
    import torch
    return torch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("coarse", ["direct", "gmres"])
def test_small_workload_parity(torch_cuda, precision, coarse):
    """32^2 x 32, time-constant uniform-random density, left-edge patch: the
    solution in parity mode (rtol 1e-12) matches the direct solve to 1e-10,
    with either coarsest-level solver."""
    from paper_2508_09589_amd.inputs import uniform_density
    c = Case(32, 32, 32, rho=uniform_density(32, seed=0))
    p = c.problem(precision=precision, rtol=1e-12, coarse=coarse)
    T, info = p.solve()
    s = solve_direct(c.Jm, c.fm)
    assert info.true_rel_res <= 1e-12
    assert rel(T.cpu().numpy(), s) <= 1e-10, rel(T.cpu().numpy(), s)
    assert info.levels == 4
    p.close()


@pytest.mark.parametrize("tv", [False, True])
def test_bf16_coarse_levels_solve_parity(torch_cuda, tv):
    """Mixed precision with BF16 coarse stencils: the FP64 outer FGMRES still
    reaches the direct solution (rtol 1e-12 -> 1e-10)."""
    c = Case(32, 32, 32, tv=tv, seed=23)
    p = c.problem(precision="mixed", bf16_from_level=1, rtol=1e-12)
    T, info = p.solve()
    s = solve_direct(c.Jm, c.fm)
    assert info.true_rel_res <= 1e-12
    assert rel(T.cpu().numpy(), s) <= 1e-10, rel(T.cpu().numpy(), s)
    p.close()


@pytest.mark.parametrize("nx,ny,nt,tv", [(24, 16, 12, True), (20, 28, 16, False), (1, 1, 1, False),
                                         (2, 2, 1, True)])
def test_ragged_and_tiny_grids(torch_cuda, nx, ny, nt, tv):
    c = Case(nx, ny, nt, tv=tv, seed=nx * ny + nt,
             patches=((0, 0.5 * ny / max(nx, ny), 0.2), (2, 0.3, 0.3)))
    p = c.problem(rtol=1e-12)
    T, info = p.solve()
    s = solve_direct(c.Jm, c.fm)
    assert rel(T.cpu().numpy(), s) <= 1e-10, (rel(T.cpu().numpy(), s), info.iterations)
    p.close()


def test_adjoint_parity(torch_cuda):
    c = Case(24, 24, 16, tv=True, seed=21)
    p = c.problem(rtol=1e-12)
    f = p.load_vector()
    assert rel(f.cpu().numpy(), c.f) < 1e-15
    lam, info = p.adjoint(f)
    ref = solve_adjoint_direct(c.Jm, c.f, c.mask)
    assert rel(lam.cpu().numpy(), ref) <= 1e-10
    p.close()


@pytest.mark.parametrize("n,nt,tv", [(64, 64, True), (128, 64, False)])
def test_sink_free_closed_form(torch_cuda, n, nt, tv):
    """No patch, C = 1, Q = q0: T = n q0 dt (n < nt), (nt - 1/2) q0 dt at nt,
    for any conductivity field -- checked without the oracle."""
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import smooth_density
    rho = smooth_density(n, n, nt, seed=3) if tv else np.random.default_rng(3).uniform(1e-3, 1, (n, n))
    q0 = 1.0
    p = Problem(n, n, nt, torch.tensor(rho), patches=(), q0=q0, rtol=1e-12)
    T, info = p.solve()
    dt = 1.0 / nt
    expect = np.arange(nt + 1) * q0 * dt
    expect[-1] = (nt - 0.5) * q0 * dt
    err = np.max(np.abs(T.cpu().numpy() - expect[:, None, None])) / expect.max()
    assert err < 1e-10, err
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_coarsening_solve_parity(torch_cuda, precision):
    """Full space-time coarsening (the comparison hierarchy of §5.1.2): state
    and adjoint still reach the direct solutions, and the level count is the
    oracle's."""
    c = Case(32, 32, 32, tv=True, seed=31, full=True)
    p = c.problem(precision=precision, rtol=1e-12)
    dims, _ = p.hierarchy()
    assert [tuple(d) for d in dims] == [(L["nx"], L["ny"], L["nt"]) for L in c.levels]
    T, info = p.solve()
    assert info.true_rel_res <= 1e-12
    assert rel(T.cpu().numpy(), solve_direct(c.Jm, c.fm)) <= 1e-10
    lam, _ = p.adjoint(p.load_vector())
    assert rel(lam.cpu().numpy(), solve_adjoint_direct(c.Jm, c.f, c.mask)) <= 1e-10
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tv", [False, True])
def test_sstep_smoother_solve_parity(torch_cuda, precision, tv):
    """FGMRES with s-step-smoothed V-cycles reaches the direct solution (state
    and adjoint) in the iterations the Arnoldi-smoothed solver needs (+-1)."""
    c = Case(32, 32, 32, tv=tv, seed=41)
    p = c.problem(precision=precision, rtol=1e-12, smoother="sstep")
    T, info = p.solve()
    assert info.true_rel_res <= 1e-12
    assert rel(T.cpu().numpy(), solve_direct(c.Jm, c.fm)) <= 1e-10
    lam, _ = p.adjoint(p.load_vector())
    assert rel(lam.cpu().numpy(), solve_adjoint_direct(c.Jm, c.f, c.mask)) <= 1e-10
    q = c.problem(precision=precision, rtol=1e-12)
    _, ref = q.solve()
    assert abs(info.iterations - ref.iterations) <= 1, (info.iterations, ref.iterations)
    p.close()
    q.close()


@pytest.mark.parametrize("restart", [30, 5])
def test_delayed_cgs2_matches_classical_cgs2(torch_cuda, restart):
    """The outer FGMRES orthogonalises with delayed CGS2 (one reduction and one
    update pass per step, the re-orthogonalisation of each basis vector lagging
    by one step); classical CGS2 gives the same iterates in exact arithmetic.
    Both reach the direct solution, state and adjoint, with the same iteration
    counts (+-1), also across restarts."""
    from paper_2508_09589_amd import _lib as L
    c = Case(24, 24, 32, tv=True, seed=37)
    out = {}
    for name, flags in (("delayed", 0), ("classical", L.ST_FLAG_OUTER_CGS2)):
        p = c.problem(rtol=1e-12, restart=restart)
        p.set_flags(flags)
        T, info = p.solve()
        lam, ainfo = p.adjoint(p.load_vector())
        out[name] = (T.cpu().numpy(), info.iterations, lam.cpu().numpy(), ainfo.iterations)
        assert info.true_rel_res <= 1e-12 and ainfo.true_rel_res <= 1e-12
        p.close()
    s = solve_direct(c.Jm, c.fm)
    la = solve_adjoint_direct(c.Jm, c.f, c.mask)
    for name in out:
        assert rel(out[name][0], s) <= 1e-10, name
        assert rel(out[name][2], la) <= 1e-10, name
    assert abs(out["delayed"][1] - out["classical"][1]) <= 1
    assert abs(out["delayed"][3] - out["classical"][3]) <= 1


def test_repeated_solves_are_bitwise_identical(torch_cuda):
    """Every reduction on the path is a fixed tree (no floating-point
    atomics), so two solves of one problem, and the solve of a second problem
    set up from the same input, return the same iterate bit for bit after the
    same number of iterations.  64^2 x 128 elements, time-varying density,
    the benchmark's mixed configuration with FGMRES(20): enough restarts for a
    rounding difference anywhere to change the count."""
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import smooth_density
    rho = torch.tensor(smooth_density(64, 64, 128, seed=5))
    kw = dict(precision="mixed", restart=20, rtol=1e-10, bf16_from_level=1, smoother="sstep")
    p = Problem(64, 64, 128, rho, **kw)
    T1, i1 = p.solve()
    T1 = T1.clone()
    T2, i2 = p.solve()
    q = Problem(64, 64, 128, rho, **kw)
    T3, i3 = q.solve()
    print(f"iterations {i1.iterations} {i2.iterations} {i3.iterations}", flush=True)
    assert i1.iterations == i2.iterations == i3.iterations
    assert torch.equal(T1, T2) and torch.equal(T1, T3)
    p.close()
    q.close()

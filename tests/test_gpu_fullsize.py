"""Full-size GPU checks, in the configuration the benchmark times (mixed
precision with BF16 coarse stencils from level 1, s-step smoothing,
FGMRES(30) on the medium grid, FGMRES(20) on the large one, relative residual
1e-8).  The FP64 oracle recomputes the residual of the GPU solution from its
own element matrices at every node: of the medium grid (256^2 x 256, 17M
nodes) and, one time level at a time, of the large one (512^2 x 1024, 269M
nodes)."""
import numpy as np
import pytest

from oracle.assemble import Material, load_vector_uniform, simp
from oracle.grid import Grid, dirichlet_mask
from oracle.hierarchy import build_hierarchy
from oracle.residual import apply_masked, apply_masked_at, residual_by_planes

pytestmark = pytest.mark.gpu

MAT = Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0)
PATCHES = [(0, 0.5, 0.05)]


@pytest.fixture(scope="module")
def torch_cuda(require_gpu):
    import torch
    return torch


def _workload(name, **kw):
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import WORKLOADS, workload_density
    w = WORKLOADS[name]
    rho = workload_density(name)
    g = Grid(w["nx"], w["ny"], w["nt"], 1.0 / w["nx"], 1.0 / w["nt"])
    p = Problem(w["nx"], w["ny"], w["nt"], torch.tensor(rho), precision="mixed",
                restart=20 if name == "large" else 30, rtol=1e-8, bf16_from_level=1,
                smoother="sstep", **kw)
    return p, g, rho


def _check_hierarchy(p, g):
    dims, _ = p.hierarchy()
    ref = build_hierarchy(g.nx, g.ny, g.nt, g.dx, g.dt, MAT.k_con, MAT.k_ins, MAT.c_con,
                          MAT.c_ins, max_coarse_nodes=4096)
    assert [tuple(d) for d in dims] == [(lv["nx"], lv["ny"], lv["nt"]) for lv in ref]


def test_medium_residual_every_node(torch_cuda):
    p, g, rho = _workload("medium")
    _check_hierarchy(p, g)
    T, info = p.solve()
    print(f"medium: {info.iterations} its, GPU true rel res {info.true_rel_res:.3e}", flush=True)
    lam, ainfo = p.adjoint(p.load_vector())
    Tn = T.cpu().numpy().ravel()
    ln = lam.cpu().numpy().ravel()
    p.close()
    k, C, _, _ = simp(rho, MAT)
    mask = dirichlet_mask(g, PATCHES).ravel()
    fm = np.where(mask, 0.0, load_vector_uniform(g, 1.0))
    nf = np.linalg.norm(fm)
    r = np.linalg.norm(fm - apply_masked(g, k, C, mask, Tn)) / nf
    assert r <= 1e-8, r
    assert abs(r - info.true_rel_res) <= 1e-3 * r, (r, info.true_rel_res)
    # adjoint: J_m^T lam = N f, lam = 0 on the Dirichlet set
    ra = np.linalg.norm(fm - apply_masked(g, k, C, mask, ln, transpose=True)) / nf
    assert ra <= 1e-8, ra
    assert np.all(ln[mask] == 0.0)
    assert np.all(Tn[mask] == 0.0)


def test_large_residual_full_field(torch_cuda):
    """The oracle's residual of the GPU solution over the whole large grid
    (269.7 M nodes, formed one time level at a time): ||f_m - J_m T|| <=
    1e-8 (1 + 1e-6) ||f_m||, equal to the GPU's own true residual to 1e-3;
    and at sampled nodes (3000 random ones, the nodes next to the patch, the
    first and last time levels, the corners) the node-by-node residual of
    the oracle agrees."""
    p, g, rho = _workload("large", max_it=1000)
    _check_hierarchy(p, g)
    T, info = p.solve()
    print(f"large: {info.iterations} its, GPU true rel res {info.true_rel_res:.3e}", flush=True)
    Tn = T.cpu().numpy()
    p.close()
    del T
    k, C, _, _ = simp(rho, MAT)
    mask = dirichlet_mask(g, PATCHES)
    fm = load_vector_uniform(g, 1.0)
    fm[mask.ravel()] = 0.0
    nf = np.linalg.norm(fm)
    shape = g.shape_nodes
    rng = np.random.default_rng(11)
    picks = list(rng.choice(g.n_nodes, 3000, replace=False))
    pj = np.nonzero(mask[1, :, 0])[0]
    for n in (1, 2, g.nt // 2, g.nt):
        for j in (pj[0] - 1, pj[0], pj[-1], pj[-1] + 1):
            for i in (0, 1):
                picks.append(np.ravel_multi_index((n, j, i), shape))
        for (j, i) in [(0, 0), (0, g.nx), (g.ny, 0), (g.ny, g.nx), (g.ny // 2, g.nx // 2)]:
            picks.append(np.ravel_multi_index((n, j, i), shape))
    nodes = np.array(picks)
    r = fm[nodes] - apply_masked_at(g, k, C, mask, Tn.ravel(), nodes)
    assert info.true_rel_res <= 1e-8
    assert np.max(np.abs(r)) <= 1e-8 * nf, np.max(np.abs(r)) / nf
    rn, rmax = residual_by_planes(g, k, C, mask, Tn.ravel(), fm)
    print(f"large: oracle full-field rel res {rn / nf:.4e} (GPU {info.true_rel_res:.4e}), "
          f"max |r_a| / ||f_m|| {rmax / nf:.3e}", flush=True)
    assert rn <= 1e-8 * (1 + 1e-6) * nf, rn / nf
    assert abs(rn / nf - info.true_rel_res) <= 1e-3 * info.true_rel_res
    assert np.max(np.abs(r)) <= rmax * (1 + 1e-12)
    on_mask = nodes[mask.ravel()[nodes]]
    assert np.all(Tn.ravel()[on_mask] == 0.0)

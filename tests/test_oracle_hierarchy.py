"""Pins of Algorithm 1 (semi-coarsening choice) against the paper's tables."""
import os

import pytest

from oracle.hierarchy import build_hierarchy

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    cases, cur = [], None
    for line in open(os.path.join(GOLD, "hierarchies.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("case"):
            parts = line.split()
            kv = dict(p.split("=") for p in parts[2:])
            cur = dict(name=parts[1], params=kv, levels=[])
            cases.append(cur)
        else:
            cur["levels"].append(tuple(int(v) for v in line.split()))
    return cases


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_printed_hierarchies(case):
    p = case["params"]
    nx, nt = int(p["nx"]), int(p["nt"])
    lv = build_hierarchy(nx, nx, nt, 1.0 / nx, 1.0 / nt, float(p["k_con"]), float(p["k_ins"]),
                         float(p["c_con"]), float(p["c_ins"]), lambda_crit=0.5,
                         n_levels=int(p["levels"]))
    got = [(L["nx"], L["ny"], L["nt"]) for L in lv]
    assert got == case["levels"]


@pytest.mark.parametrize("n,nt,expect", [
    (32, 32, [(32, 32), (16, 32), (16, 16), (8, 16)]),
    (256, 256, [(256, 256), (128, 256), (64, 256), (32, 256), (32, 128), (32, 64), (16, 64),
                (16, 32)]),
    (512, 1024, [(512, 1024), (256, 1024), (128, 1024), (64, 1024), (64, 512), (64, 256),
                 (32, 256), (32, 128)]),
    (128, 128, [(128, 128), (64, 128), (32, 128), (32, 64), (16, 64), (16, 32), (16, 16), (8, 16)]),
])
def test_workload_hierarchies(n, nt, expect):
    """Unit square, tau = 1, k in [1e-3, 1], C = 1: Algorithm 1 with N_l = 8
    levels (the paper's space-time runs), or fewer once a level has at most
    4096 nodes."""
    lv = build_hierarchy(n, n, nt, 1.0 / n, 1.0 / nt, 1.0, 1e-3, 1.0, 1.0)
    assert [(L["nx"], L["nt"]) for L in lv] == expect
    assert len(lv) == 8 or (lv[-1]["nx"] + 1) ** 2 * (lv[-1]["nt"] + 1) <= 4096
    # without the level cap: down to at most 4096 nodes
    deep = build_hierarchy(n, n, nt, 1.0 / n, 1.0 / nt, 1.0, 1e-3, 1.0, 1.0, max_levels=32)
    assert [(L["nx"], L["nt"]) for L in deep[:len(lv)]] == expect
    assert (deep[-1]["nx"] + 1) ** 2 * (deep[-1]["nt"] + 1) <= 4096


def test_level_cap_yields_to_the_coarsest_factorisation():
    """Past N_l coarsening goes on while the coarsest planes are over the
    exact factorisation's limit (2048 nodes): 512^2 x 4096 has 64^2-element
    planes (4225 nodes) on its eighth level and takes a ninth (32^2)."""
    lv = build_hierarchy(512, 512, 4096, 1 / 512, 1 / 4096, 1.0, 1e-3, 1.0, 1.0)
    assert (lv[7]["nx"] + 1) * (lv[7]["ny"] + 1) > 2048
    assert len(lv) == 9 and (lv[-1]["nx"], lv[-1]["nt"]) == (32, 256)
    # the level count alone when the planes fit
    lv = build_hierarchy(512, 512, 1024, 1 / 512, 1 / 1024, 1.0, 1e-3, 1.0, 1.0)
    assert len(lv) == 8 and (lv[-1]["nx"] + 1) ** 2 <= 2048


def test_tie_goes_to_space():
    # k_con = k_ins = 0.25, C = 1: D_eff = 0.25 and lambda = 0.25 * 0.125 / 0.25^2 = 0.5.
    lv = build_hierarchy(4, 4, 8, 0.25, 0.125, 0.25, 0.25, 1.0, 1.0, lambda_crit=0.125, n_levels=2)
    assert lv[0]["lam"] == 0.5
    assert lv[1]["how"] == "space"            # 0.5 >= 0.125
    # lambda exactly at lambda_crit: the strict comparison coarsens in space ...
    lv = build_hierarchy(4, 4, 8, 0.25, 0.125, 0.25, 0.25, 1.0, 1.0, lambda_crit=0.5, n_levels=2)
    assert lv[1]["how"] == "space"
    # ... and just above it, in time
    lv = build_hierarchy(4, 4, 8, 0.25, 0.125, 0.25, 0.25, 1.0, 1.0, lambda_crit=0.5 + 1e-12,
                         n_levels=2)
    assert lv[1]["how"] == "time"


def test_printed_dof_counts():
    for line in open(os.path.join(GOLD, "dof_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        nx, ny, nt, dofs = (int(v) for v in line.split()[:4])
        assert (nx + 1) * (ny + 1) * (nt + 1) == dofs


def test_full_coarsening_hierarchy_and_galerkin():
    """Full space-time coarsening halves all three counts per level; its
    masked P is the Kronecker product of the three 1-D interpolations, and
    the Galerkin operators stay 27-point (coarse stencil radius 1)."""
    import numpy as np
    from oracle.assemble import assemble_matrix, apply_dirichlet, load_vector
    from oracle.grid import Grid, dirichlet_mask
    from oracle.multigrid import build_operators
    lv = build_hierarchy(16, 16, 16, 1 / 16, 1 / 16, 1.0, 1e-3, 1.0, 1.0, full=True,
                         max_coarse_nodes=200)
    assert [(l["nx"], l["ny"], l["nt"], l["how"]) for l in lv] == [
        (16, 16, 16, None), (8, 8, 8, "full"), (4, 4, 4, "full")]
    g = Grid(16, 16, 16, 1 / 16, 1 / 16)
    rng = np.random.default_rng(0)
    k = rng.uniform(0.1, 1.0, (16, 16, 16))
    mask = dirichlet_mask(g, [(0, 0.5, 0.2)])
    Jm, _ = apply_dirichlet(assemble_matrix(g, k, np.ones_like(k)), load_vector(g), mask)
    A, masks, Pm = build_operators(lv, Jm, mask)
    for l in (1, 2):
        L = lv[l]
        Ac = A[l].tocoo()
        shp = (L["nt"] + 1, L["ny"] + 1, L["nx"] + 1)
        rn, rj, ri = np.unravel_index(Ac.row, shp)
        cn, cj, ci = np.unravel_index(Ac.col, shp)
        assert max(abs(rn - cn).max(), abs(rj - cj).max(), abs(ri - ci).max()) <= 1
    # an odd count stops full coarsening
    lv = build_hierarchy(12, 12, 6, 1 / 12, 1 / 6, 1.0, 1e-3, 1.0, 1.0, full=True, max_coarse_nodes=10)
    assert [(l["nx"], l["nt"]) for l in lv] == [(12, 6), (6, 3)]

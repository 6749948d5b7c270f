"""The example problems of §2.3 as input generators (CPU): the source
formulas at points where they have closed values, the rescaling, and the
oracle's FGMRES + V-cycle converging on them under both coarsenings."""
import numpy as np
import pytest

from oracle.assemble import Material, apply_dirichlet, assemble_matrix, load_vector, simp
from oracle.grid import Grid, dirichlet_mask
from oracle.hierarchy import build_hierarchy
from oracle.krylov import VCycle, fgmres
from oracle.multigrid import build_operators
from oracle.solve import solve_direct
from paper_2508_09589_amd.inputs import (example1_source, example2_centre, example2_source,
                                         example_design, example_problem, PAPER_MATERIAL)


def test_example1_source_closed_values():
    q = example1_source(4, 100)
    assert q.shape == (101, 5, 5)
    assert np.all(q == q[:, :1, :1])                 # uniform in space
    assert q[0, 0, 0] == pytest.approx(100.0)         # (1 - 0)(1 + cos 0) q0 / 2
    assert q[-1, 0, 0] == pytest.approx(0.0, abs=1e-12)
    assert q.min() >= 0.0
    t = 0.5
    assert q[50, 2, 3] == pytest.approx(50.0 * (1 - t) * (1 + np.cos(50 * t)))


def test_example2_source_path_and_width():
    # start at (L/2, 3L/4); half a rotation (physical t = 1, rescaled 1/6) later
    # at (L/2, L/4); one full rotation (t = 2) later back at the start
    c1, c2 = example2_centre(np.array([0.0, 1.0, 2.0, 0.5]))
    assert np.allclose(c1, [0.5, 0.5, 0.5, 0.25]) and np.allclose(c2, [0.75, 0.25, 0.75, 0.5])
    q = example2_source(8, 12)          # rescaled t~ = n / 12, physical t = n / 2
    assert q.shape == (13, 9, 9)
    assert q[0, 6, 4] == pytest.approx(1.0)          # node (0.5, 0.75)
    assert q[2, 2, 4] == pytest.approx(1.0)          # t = 1: node (0.5, 0.25)
    assert q[1, 4, 2] == pytest.approx(1.0)          # t = 1/2: node (0.25, 0.5)
    # one sigma-free offset: at distance d the value is exp(-d^2 / (2 sigma^2))
    assert q[0, 6, 5] == pytest.approx(np.exp(-(0.125 ** 2) / (2 * 0.05 ** 2)))
    assert q.max() <= 1.0


def test_example_rescaling_and_variants():
    e1 = example_problem("1B", 8, 16)
    e2 = example_problem("2C", 8, 16)
    assert e1["k_con"] == PAPER_MATERIAL["k_con"] and e1["k_ins"] == PAPER_MATERIAL["k_ins"]
    assert e2["k_con"] == pytest.approx(6 * 3.0) and e2["k_ins"] == pytest.approx(6 * 0.03)
    assert e2["c_con"] == 100.0 and example_problem("1D", 8, 16)["p_c"] == 4.0
    assert e1["patches"] == ((2, 0.5, 0.05),) and len(e2["patches"]) == 4
    d = example_design("tree", 16)
    assert d[0, 8] == 1.0 and d[0, 0] < 0.01          # trunk leaves the lower edge at x1 = 0.5


def _oracle_case(variant, n, nt, full):
    kw = example_problem(variant, n, nt)
    m = Material(**{k: kw[k] for k in ("k_ins", "k_con", "p_k", "c_ins", "c_con", "p_c")})
    g = Grid(n, n, nt, kw["dx"], kw["dt"])
    k, C, _, _ = simp(example_design("tree", n), m)
    mask = dirichlet_mask(g, kw["patches"])
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, C), load_vector(g, q_nodal=kw["source"]), mask)
    lv = build_hierarchy(n, n, nt, g.dx, g.dt, m.k_con, m.k_ins, m.c_con, m.c_ins,
                         max_coarse_nodes=100, full=full)
    return Jm, fm, mask, lv


@pytest.mark.parametrize("full", [False, True])
@pytest.mark.parametrize("variant", ["1B", "2B"])
def test_oracle_fgmres_converges_on_examples(variant, full):
    Jm, fm, mask, lv = _oracle_case(variant, 8, 16, full)
    assert len(lv) >= 3 and all(L["how"] == ("full" if full else L["how"]) for L in lv[1:])
    A, masks, Pm = build_operators(lv, Jm, mask)
    x, its, rr = fgmres(Jm, fm, VCycle(A, Pm, coarse="direct"), rtol=1e-10, maxit=200)
    assert rr <= 1e-10 and its < 60
    s = solve_direct(Jm, fm)
    assert np.linalg.norm(x - s) <= 1e-8 * np.linalg.norm(s)

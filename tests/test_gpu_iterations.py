"""Outer FGMRES iteration counts on the heat-sink design against the FP64
oracle (tests/golden/heatsink_iterations.txt, written by
heatsink_iterations.py from oracle/ only), in the settings of the large
benchmark: FGMRES(20) to 1e-8, s-step Jacobi-GMRES(10) smoothing, exact
coarsest solve, Algorithm 1 hierarchy; FP32 V-cycle with BF16 stencils from
level 1 under FP64 FGMRES, and plain FP64.

FGMRES converges with any preconditioner, so a V-cycle defect shows as extra
iterations; the counts must agree within 2 (the smoother's s-step form is
exact only up to rounding, which moves a count by one or two)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "heatsink_iterations.txt")


def _cases():
    rows = []
    with open(GOLD) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            n, nt, its, rel, nl = ln.split()
            rows.append((int(n), int(nt), int(its), int(nl)))
    return rows


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}x{c[0]}x{c[1]}")
def test_heat_sink_iterations_match_oracle(require_gpu, case, precision):
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import heat_sink_density
    n, nt, its_or, nl = case
    kw = dict(bf16_from_level=1) if precision == "mixed" else {}
    p = Problem(n, n, nt, torch.tensor(heat_sink_density(n)), precision=precision, restart=20,
                rtol=1e-8, smoother="sstep", max_it=400, **kw)
    T, info = p.solve()
    print(f"{n}^2 x {nt} {precision}: GPU {info.iterations} its, oracle {its_or}, "
          f"true rel res {info.true_rel_res:.2e}", flush=True)
    assert info.levels == nl
    assert info.true_rel_res <= 1e-8
    assert abs(info.iterations - its_or) <= 2, (info.iterations, its_or)
    p.close()

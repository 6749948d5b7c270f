"""Writes heatsink_iterations.txt: outer FGMRES(20) iteration counts of the
FP64 oracle on the heat-sink design (time-constant, rho in {0.001, 1}) at
reduced grids, with the solver settings of the large benchmark: Algorithm 1
hierarchy down to <= 4096 nodes, Jacobi-GMRES(10) smoothing in s-step form,
exact coarsest-level solve, stop at ||f - J s|| <= 1e-8 ||f||.

    python tests/golden/heatsink_iterations.py [n:nt ...]

Everything here is oracle/ (assembled sparse matrices, Galerkin products,
scipy solves); nothing comes from the GPU path.  The GPU test
(tests/test_gpu_iterations.py) compares its counts with these.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.assemble import Material, assemble_matrix, apply_dirichlet, load_vector, simp  # noqa
from oracle.grid import Grid, dirichlet_mask                                             # noqa
from oracle.hierarchy import build_hierarchy                                             # noqa
from oracle.krylov import VCycle, fgmres                                                 # noqa
from oracle.multigrid import build_operators                                             # noqa
from paper_2508_09589_amd.inputs import heat_sink_density, PATCH_LEFT_CENTRED            # noqa

MAT = Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0)
OUT = os.path.join(HERE, "heatsink_iterations.txt")


def count(n, nt, restart=20, rtol=1e-8):
    g = Grid(n, n, nt, 1.0 / n, 1.0 / nt)
    k, C, _, _ = simp(heat_sink_density(n), MAT)
    mask = dirichlet_mask(g, [PATCH_LEFT_CENTRED])
    Jm, fm = apply_dirichlet(assemble_matrix(g, k, C), load_vector(g, 1.0), mask)
    lv = build_hierarchy(n, n, nt, g.dx, g.dt, MAT.k_con, MAT.k_ins, MAT.c_con, MAT.c_ins)
    A, _, Pm = build_operators(lv, Jm, mask)
    x, its, rel = fgmres(Jm, fm, VCycle(A, Pm, coarse="direct", smoother="sstep"), m=restart,
                         rtol=rtol, maxit=400)
    return its, rel, len(lv)


def main(cases):
    rows = []
    for n, nt in cases:
        t = time.time()
        its, rel, nl = count(n, nt)
        rows.append((n, nt, its, rel, nl))
        print(f"{n}^2 x {nt}: {its} iterations, true rel. residual {rel:.2e}, {nl} levels, "
              f"{time.time() - t:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# oracle FGMRES(20) iterations to 1e-8, heat-sink design, s-step smoother, "
                "exact coarse solve\n# n nt iterations true_rel_res levels\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]} {r[2]} {r[3]:.3e} {r[4]}\n")


if __name__ == "__main__":
    args = sys.argv[1:] or ["64:128", "64:256"]
    main([tuple(int(v) for v in a.split(":")) for a in args])

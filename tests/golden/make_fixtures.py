"""Writes the oracle fixtures of the full-size GPU parity tests.

    python tests/golden/make_fixtures.py

Every value comes from oracle/ (FP64, direct block-in-time solves) on the
seeded inputs of paper_2508_09589_amd/inputs.py; nothing comes from the GPU.
  grad_128.npz   differentiation workload (128^2 x 128, smooth density seed 2,
                 PDE filter r = 1.5 elements): J, the gradient at the 16
                 elements default_rng(3).choice(N_e, 16), its norm, and the
                 state at 2000 sampled nodes.
  grad_128_fd.npz  the central differences (h = 1e-6) of J at the same 16
                 elements in the difference-system form (J+ ds = -(J+ - J-) s-,
                 block Gauss-Seidel solves; no cancellation).
  medium_256.npz  the state of the medium workload (256^2 x 256, smooth
                 time-varying density seed 1) by 80 sweeps of block
                 Gauss-Seidel in time (the relative residual stagnates at
                 5.7e-12 from sweep 17 on, the rounding floor of the residual
                 on this grid): ||s||, the full time levels n = 128 and 256
                 and 20000 random nodes.
The large workload is checked without a fixture: the oracle recomputes the
residual of the GPU solution at every node (tests/test_gpu_fullsize.py).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.assemble import Material                               # noqa: E402
from oracle.blockgrad import (objective_and_gradient_blocks,       # noqa: E402
                              central_difference_blocks)
from oracle.grid import Grid                                       # noqa: E402
from paper_2508_09589_amd.inputs import workload_density, PATCH_LEFT_CENTRED  # noqa: E402

MAT = Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0)


def grad():
    n = 128
    g = Grid(n, n, n, 1.0 / n, 1.0 / n)
    rho = workload_density("grad")
    t = time.time()
    out = objective_and_gradient_blocks(g, MAT, rho, [PATCH_LEFT_CENTRED], 1.0, 1.5)
    idx = np.random.default_rng(3).choice(g.n_elems, 16, replace=False)
    nodes = np.random.default_rng(5).choice(g.n_nodes, 2000, replace=False)
    np.savez(os.path.join(HERE, "grad_128.npz"), J=out["J"], elems=idx,
             grad_at=out["grad"].ravel()[idx], grad_norm=np.linalg.norm(out["grad"]),
             nodes=nodes, s_at=out["s"][nodes], s_norm=np.linalg.norm(out["s"]),
             lam_at=out["lam"][nodes], lam_norm=np.linalg.norm(out["lam"]),
             rel_res=np.array(out["rel"]), sweeps=np.array(out["sweeps"]))
    print("grad fixture", out["J"], out["sweeps"], out["rel"], f"{time.time() - t:.1f} s")


_S0 = None


def _fd_init(s0):
    global _S0
    _S0 = s0


def _fd_one(e):
    n = 128
    g = Grid(n, n, n, 1.0 / n, 1.0 / n)
    rho = workload_density("grad")
    t = time.time()
    fd, sweeps = central_difference_blocks(g, MAT, rho, [PATCH_LEFT_CENTRED], int(e), 1e-6, 1.0,
                                           1.5, tol=3e-12, max_sweeps=200, s0=_S0)
    print(f"element {e}: fd {fd:.12e}, sweeps {sweeps}, {time.time() - t:.1f} s", flush=True)
    return fd


def grad_fd(workers=4):
    """The state at rho (solved once) starts every s- solve.  Block
    Gauss-Seidel stagnates near a relative residual of 1.2e-12 on this grid
    (rounding of the residual itself), so the solves stop at 3e-12."""
    from concurrent.futures import ProcessPoolExecutor
    from oracle.assemble import load_vector, simp
    from oracle.design import filter_apply
    from oracle.grid import dirichlet_mask
    from oracle.solve import BlockTimeSystem
    n = 128
    g = Grid(n, n, n, 1.0 / n, 1.0 / n)
    rho = workload_density("grad")
    k, C, _, _ = simp(filter_apply(rho, g.dx, g.dt, 1.5 * g.dx, 1.5 * g.dt), MAT)
    bs = BlockTimeSystem(g, k, C, dirichlet_mask(g, [PATCH_LEFT_CENTRED]))
    s0, sw, rel = bs.gauss_seidel(bs.masked_rhs(load_vector(g, 1.0)), tol=3e-12, max_sweeps=200)
    print(f"base state: {sw} sweeps, rel. residual {rel:.2e}", flush=True)
    del bs
    idx = np.random.default_rng(3).choice(n * n * n, 16, replace=False)
    with ProcessPoolExecutor(workers, initializer=_fd_init, initargs=(s0,)) as ex:
        fd = np.array(list(ex.map(_fd_one, idx)))
    np.savez(os.path.join(HERE, "grad_128_fd.npz"), elems=idx, h=np.array(1e-6), fd=fd)
    print("grad fd fixture written")


def medium():
    from oracle.assemble import load_vector, simp
    from oracle.grid import dirichlet_mask
    from oracle.solve import BlockTimeSystem
    n = 256
    g = Grid(n, n, n, 1.0 / n, 1.0 / n)
    rho = workload_density("medium")
    k, C, _, _ = simp(rho, MAT)
    t = time.time()
    bs = BlockTimeSystem(g, k, C, dirichlet_mask(g, [PATCH_LEFT_CENTRED]))
    s, sweeps, rel = bs.gauss_seidel(bs.masked_rhs(load_vector(g, 1.0)), tol=3e-12,
                                     max_sweeps=80,
                                     log=lambda k, r: print(f"sweep {k}: {r:.3e}", flush=True))
    S = s.reshape(g.shape_nodes)
    nodes = np.random.default_rng(6).choice(g.n_nodes, 20000, replace=False)
    levels = np.array([128, 256])
    np.savez(os.path.join(HERE, "medium_256.npz"), s_norm=np.linalg.norm(s), levels=levels,
             s_levels=S[levels], nodes=nodes, s_at=s[nodes], rel_res=np.array(rel),
             sweeps=np.array(sweeps))
    print(f"medium fixture: {sweeps} sweeps, rel. residual {rel:.2e}, {time.time() - t:.0f} s")


if __name__ == "__main__":
    which = sys.argv[1:] or ["grad", "grad_fd", "medium"]
    if "grad" in which:
        grad()
    if "grad_fd" in which:
        grad_fd()
    if "medium" in which:
        medium()

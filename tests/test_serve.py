"""Serving loop: scheduling logic on a CPU mock backend, and on the GPU the
continuous-batching run with the alone-vs-in-the-mix equality."""
import threading
import time

import numpy as np
import pytest
import torch

from paper_2508_09589_amd.serve import Request, Server, request_density, run_stream


class MockProblem:
    """Stand-in with the Problem interface: a scripted duration per solve."""
    live = 0
    peak = 0
    lock = threading.Lock()

    def __init__(self, req, nbytes):
        self.workspace_bytes = nbytes - 256
        self.created_for = req.id
        self.updates = 0
        with MockProblem.lock:
            MockProblem.live += 1

    def set_stream(self, s):
        pass

    def update_density(self, rho):
        self.updates += 1

    def solve(self, allow_not_converged=False):
        time.sleep(0.01)
        if getattr(self, "fail_next", False):
            raise RuntimeError("scripted solve failure")
        info = type("I", (), dict(iterations=3, true_rel_res=1e-9))()
        return np.zeros(1), info

    def load_vector(self):
        return np.zeros(1)

    def adjoint(self, f, allow_not_converged=False):
        time.sleep(0.01)
        return np.zeros(1), type("I", (), dict(iterations=4, true_rel_res=1e-9))()

    def sensitivity(self, T, lam):
        return np.zeros(1)

    def objective(self, T):
        return 0.0

    def close(self):
        with MockProblem.lock:
            MockProblem.live -= 1


def _mock_server(budget, slots=3):
    fp = lambda n, nt, tv, prec: n * n * nt * 100 + 256
    mk = lambda req, dev, s: MockProblem(req, fp(req.n, req.nt, True, req.precision))
    return Server(budget, slots=slots, device="cpu", make_problem=mk, footprint_fn=fp)


def test_admission_respects_budget_and_reuses_resident_problems():
    budget = 32 * 32 * 32 * 100 * 2 + 1000        # room for two 32^3 problems
    srv = _mock_server(budget, slots=4)
    reqs = [Request(i, 32, 32, np.zeros((32, 32, 32)), adjoint=(i % 2 == 1)) for i in range(12)]
    futs = [srv.submit(r) for r in reqs]
    out = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [o["id"] for o in out] == list(range(12))
    assert srv.peak_bytes <= budget
    assert all("grad" in o for o in out if o["id"] % 2 == 1)
    # at most two problems were ever built; the rest reused them
    assert MockProblem.live == 0


def test_oversized_request_is_rejected_not_stuck():
    srv = _mock_server(1000, slots=1)
    f = srv.submit(Request(0, 32, 32, np.zeros((32, 32, 32))))
    with pytest.raises(MemoryError):
        f.result(timeout=10)
    srv.close()


def test_eviction_makes_room_for_new_shapes():
    fp32 = 32 * 32 * 32 * 100 + 256
    srv = _mock_server(fp32 + 100, slots=1)     # room for one problem at a time
    a = srv.submit(Request(0, 32, 32, np.zeros((32, 32, 32)))).result(timeout=10)
    b = srv.submit(Request(1, 16, 16, np.zeros((16, 16, 16)))).result(timeout=10)
    c = srv.submit(Request(2, 32, 32, np.zeros((32, 32, 32)))).result(timeout=10)
    srv.close()
    assert srv.peak_bytes <= fp32 + 100 and a and b and c


def _failing_server(budget, fail_ids, slots=2, bad_ids=()):
    """Mock server whose problems fail the solve of the requests in fail_ids
    and whose footprint function rejects the requests in bad_ids."""
    def fp(n, nt, tv, prec):
        if n == 7:
            raise ValueError("grid rejected by the footprint function")
        return n * n * nt * 100 + 256

    def mk(req, dev, s):
        p = MockProblem(req, fp(req.n, req.nt, True, req.precision))
        return p

    srv = Server(budget, slots=slots, device="cpu", make_problem=mk, footprint_fn=fp)
    orig = srv._solve

    def solve(req, prob, stream, made):
        if prob is not None:
            prob.fail_next = req.id in fail_ids
        else:
            def mk2(r, dev, s, _mk=mk):
                p = _mk(r, dev, s)
                p.fail_next = r.id in fail_ids
                return p
            srv.make_problem = mk2
        return orig(req, prob, stream, made)
    srv._solve = solve
    return srv


def test_failing_solves_release_memory_and_close_problems():
    """A solve that raises fails only its request: a new problem is closed,
    a pooled one too (its state is not trusted), the bytes go back, and the
    slot serves the next requests."""
    MockProblem.live = 0
    budget = 32 * 32 * 32 * 100 * 3 + 1000
    srv = _failing_server(budget, fail_ids={0, 3, 4})
    reqs = [Request(i, 32, 32, np.zeros((32, 32, 32))) for i in range(8)]
    futs = [srv.submit(r) for r in reqs]
    ok, failed = [], []
    for f in futs:
        try:
            ok.append(f.result(timeout=30)["id"])
        except RuntimeError:
            failed.append(f)
    assert len(failed) == 3 and sorted(ok) == [1, 2, 5, 6, 7]
    with srv.cv:
        assert srv.busy_bytes == 0
    srv.close()
    assert MockProblem.live == 0


def test_invalid_request_fails_alone():
    """A request the footprint function rejects fails its own future; the
    slot threads survive and serve the requests behind it."""
    MockProblem.live = 0
    srv = _failing_server(10 ** 9, fail_ids=set(), slots=1)
    bad = srv.submit(Request(0, 7, 8, np.zeros((8, 7, 7))))
    good = [srv.submit(Request(i, 16, 16, np.zeros((16, 16, 16)))) for i in (1, 2)]
    with pytest.raises(ValueError):
        bad.result(timeout=10)
    assert [g.result(timeout=10)["id"] for g in good] == [1, 2]
    srv.close()
    assert MockProblem.live == 0 and srv.busy_bytes == 0


def test_cancelled_request_is_skipped():
    """A future cancelled while queued is never run and holds no memory."""
    MockProblem.live = 0
    fp32 = 32 * 32 * 32 * 100 + 256
    srv = _mock_server(fp32 + 100, slots=1)
    first = srv.submit(Request(0, 32, 32, np.zeros((32, 32, 32))))
    second = srv.submit(Request(1, 32, 32, np.zeros((32, 32, 32))))
    third = srv.submit(Request(2, 16, 16, np.zeros((16, 16, 16))))
    second.cancel()
    assert first.result(timeout=10)["id"] == 0
    assert third.result(timeout=10)["id"] == 2
    assert second.cancelled()
    srv.close()
    assert MockProblem.live == 0 and srv.busy_bytes == 0


def test_pool_key_separates_solver_options():
    """A resident problem built for one smoother is not reused for a request
    asking for the other."""
    a = Request(0, 32, 32, np.zeros((32, 32, 32)), smoother="sstep")
    b = Request(1, 32, 32, np.zeros((32, 32, 32)), smoother="gmres")
    c = Request(2, 32, 32, np.zeros((32, 32, 32)), smoother="sstep", precision="fp64")
    assert len({a.key, b.key, c.key}) == 3


def test_request_density_range_and_determinism():
    a = request_density(32, 16, 7)
    b = request_density(32, 16, 7)
    assert a.shape == (16, 32, 32) and np.array_equal(a, b)
    assert a.min() >= 0.001 and a.max() <= 1.0


@pytest.mark.gpu
def test_alone_equals_in_the_mix(require_gpu):
    """Each request's temperature (and gradient) is bitwise the same when it
    runs alone and when it runs concurrently with others."""
    specs = [(32, 32, False), (64, 32, True), (32, 64, True), (64, 64, False), (32, 32, True)]
    reqs = lambda: [Request(i, n, nt, request_density(n, nt, 100 + i), adjoint=adj, precision="mixed")
                    for i, (n, nt, adj) in enumerate(specs)]
    alone = {}
    srv = Server(8 << 30, slots=1)
    for r in reqs():
        alone[r.id] = srv.submit(r).result(timeout=120)
    srv.close()
    srv = Server(8 << 30, slots=4)
    futs = [srv.submit(r) for r in reqs()]
    mix = {f.result(timeout=120)["id"]: f.result() for f in futs}
    srv.close()
    for i in alone:
        assert torch.equal(alone[i]["T"], mix[i]["T"]), i
        if "grad" in alone[i]:
            assert torch.equal(alone[i]["grad"], mix[i]["grad"]), i
        assert alone[i]["true_rel_res"] <= 1e-8


@pytest.mark.gpu
def test_served_requests_against_the_oracle(require_gpu):
    """16 requests drawn at random (default_rng(5)) from the serving workload's
    256 (square grids of 32..256 elements, 32..256 slabs, time-varying
    densities, half with a gradient), served concurrently in 4 slots at the
    benchmark's settings: the oracle recomputes, with its own element
    matrices, the residual of every served state and adjoint over the whole
    field (<= 1e-8 (1 + 1e-6) of the right-hand side) and the sensitivities
    from the served state and adjoint (1e-12)."""
    from oracle.assemble import Material, load_vector_uniform, simp
    from oracle.design import element_sensitivity, reduce_to_design
    from oracle.grid import Grid, dirichlet_mask
    from oracle.residual import residual_by_planes
    from paper_2508_09589_amd.inputs import serving_requests
    specs = serving_requests(256)
    pick = sorted(np.random.default_rng(5).choice(256, 16, replace=False))
    reqs = [Request(specs[i]["id"], specs[i]["n"], specs[i]["nt"],
                    request_density(specs[i]["n"], specs[i]["nt"], specs[i]["seed"]),
                    adjoint=specs[i]["adjoint"], precision="mixed") for i in pick]
    srv = Server(64 << 30, slots=4)
    futs = [srv.submit(r) for r in reqs]
    outs = {f.result(timeout=300)["id"]: f.result() for f in futs}
    srv.close()
    mat = Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0)
    assert sum(r.adjoint for r in reqs) >= 4
    for r in reqs:
        o = outs[r.id]
        g = Grid(r.n, r.n, r.nt, 1.0 / r.n, 1.0 / r.nt)
        k, C, dk, dC = simp(r.rho, mat)
        mask = dirichlet_mask(g, [(0, 0.5, 0.05)])
        fm = load_vector_uniform(g, 1.0)
        fm[mask.ravel()] = 0.0
        nf = np.linalg.norm(fm)
        T = o["T"].cpu().numpy().ravel()
        rn, _ = residual_by_planes(g, k, C, mask, T, fm)
        print(f"request {r.id} {r.n}^2 x {r.nt}: state res {rn / nf:.3e}", flush=True)
        assert rn <= 1e-8 * (1 + 1e-6) * nf, (r.id, rn / nf)
        if r.adjoint:
            lam = o["lam"].cpu().numpy().ravel()
            ra, _ = residual_by_planes(g, k, C, mask, lam, fm, transpose=True)
            assert ra <= 1e-8 * (1 + 1e-6) * nf, (r.id, ra / nf)
            ge = reduce_to_design(element_sensitivity(g, T, lam, dk, dC), r.rho.shape)
            gg = o["grad"].cpu().numpy()
            assert np.linalg.norm(gg - ge) <= 1e-12 * np.linalg.norm(ge), r.id

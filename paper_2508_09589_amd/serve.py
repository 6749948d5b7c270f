"""Continuous-batching request server for space-time solves on one GPU.

Requests (a grid, a design, forward-only or forward + adjoint gradient) arrive
at any time.  A fixed number of worker slots, each with its own HIP stream,
take requests from the queue as soon as a slot and enough HBM are free, so
requests that arrive while others run are admitted and their kernels overlap
on the device.  Admission is by the exact workspace footprint reported by the
library (st_footprint_bytes).  Multigrid hierarchies stay resident: a finished
request returns its problem (workspace, level buffers) to a pool keyed by
grid shape and precision, and the next request of that shape only reloads its
density (st_update_density), without allocating.  Idle pooled problems are
evicted, least recently used first, when a new shape needs the memory.

Every solve is deterministic (fixed reduction trees, grid sizes that depend
only on the problem), so a request gives bitwise the same result alone and in
the mix.
"""
import collections
import ctypes as C
import threading
import time
from concurrent.futures import Future

import numpy as np
import torch

from . import _lib as L
from .solver import Problem


class Request:
    def __init__(self, rid, n, nt, rho, adjoint=False, t_arrive=None, precision="mixed",
                 smoother="sstep"):
        self.id = rid
        self.smoother = smoother
        self.n, self.nt = int(n), int(nt)
        self.rho = rho                      # host array [nt, n, n] or [n, n]
        self.adjoint = bool(adjoint)
        self.t_arrive = t_arrive
        self.precision = precision
        self.t_admit = None
        self.t_done = None

    @property
    def key(self):
        """Requests with equal keys can share a resident problem: same grid,
        design layout and solver options."""
        tv = np.asarray(self.rho).ndim == 3
        return (self.n, self.nt, tv, self.precision, self.smoother)

    @property
    def dofs(self):
        return (self.n + 1) ** 2 * (self.nt + 1) * (2 if self.adjoint else 1)


def footprint(n, nt, time_varying, precision):
    lib = L.load()
    g = L.st_grid(n, n, nt, 1.0 / n, 1.0 / nt)
    m = L.st_material(1e-3, 1.0, 3.0, 1.0, 1.0, 1.0)
    o = L.default_opts()
    o.precision = L.ST_MIXED if precision == "mixed" else L.ST_FP64
    b = C.c_size_t(0)
    L.check("st_footprint_bytes", lib.st_footprint_bytes(C.byref(g), C.byref(m), C.byref(o),
                                                         int(time_varying), C.byref(b)))
    return int(b.value) + 256


def _gpu_problem(req, device, stream):
    rho = torch.as_tensor(req.rho, dtype=torch.float64)
    return Problem(req.n, req.n, req.nt, rho, precision=req.precision, device=device,
                   stream=stream, smoother=req.smoother)


class Server:
    """Server(hbm_budget_bytes, slots).submit(request) -> Future of a dict with
    the temperature (and the gradient for adjoint requests) and timings.

    make_problem(req, device, stream) and footprint_fn(n, nt, tv, precision)
    default to the GPU library; tests substitute a CPU mock."""

    def __init__(self, hbm_budget, slots=4, device="cuda", keep_outputs=True,
                 make_problem=None, footprint_fn=None):
        self.budget = int(hbm_budget)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.keep_outputs = keep_outputs
        self.make_problem = make_problem or _gpu_problem
        self.footprint_fn = footprint_fn or footprint
        self.cv = threading.Condition()
        self.queue = collections.deque()
        self.pool = collections.OrderedDict()   # key -> list of idle Problems (LRU order)
        self.pool_bytes = 0                      # bytes held by idle pooled problems
        self.busy_bytes = 0                      # bytes held by running requests
        self.peak_bytes = 0
        self.closed = False
        self.admission_waits = 0
        self.stats = []
        if self.device.type == "cuda":
            self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        else:
            self.streams = [None] * slots
        self.threads = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                        for s in self.streams]
        for t in self.threads:
            t.start()

    # ------------------------------------------------------------------
    def submit(self, req):
        fut = Future()
        if req.t_arrive is None:
            req.t_arrive = time.perf_counter()
        with self.cv:
            self.queue.append((req, fut))
            self.cv.notify_all()
        return fut

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        for lst in self.pool.values():
            for p in lst:
                p.close()
        self.pool.clear()

    # ------------------------------------------------------------------
    def _take(self):
        """Next admissible request (FIFO order; a request that does not fit
        waits, later requests that fit may pass it) plus its problem source."""
        while True:
            if self.closed and not self.queue:
                return None
            for i, (req, fut) in enumerate(self.queue):
                if fut.cancelled():
                    del self.queue[i]
                    break
                try:
                    key = req.key
                    pooled = bool(self.pool.get(key))
                    need = 0 if pooled else self.footprint_fn(req.n, req.nt, key[2],
                                                              req.precision)
                except Exception as e:          # an invalid request fails alone
                    del self.queue[i]
                    if fut.set_running_or_notify_cancel():
                        fut.set_exception(e)
                    break
                if pooled:
                    if not fut.set_running_or_notify_cancel():
                        del self.queue[i]
                        break
                    p = self.pool[key].pop()
                    if not self.pool[key]:
                        del self.pool[key]
                    self.pool_bytes -= p.workspace_bytes + 256
                    self.busy_bytes += p.workspace_bytes + 256
                    del self.queue[i]
                    return req, fut, p, 0
                if need > self.budget:
                    del self.queue[i]
                    if fut.set_running_or_notify_cancel():
                        fut.set_exception(MemoryError(
                            f"request {req.id} needs {need} bytes, over the {self.budget}-byte "
                            "budget"))
                    break
                # evict idle problems (least recently used) until it fits
                while self.busy_bytes + self.pool_bytes + need > self.budget and self.pool:
                    k0 = next(iter(self.pool))
                    victim = self.pool[k0].pop(0)
                    if not self.pool[k0]:
                        del self.pool[k0]
                    self.pool_bytes -= victim.workspace_bytes + 256
                    victim.close()
                if self.busy_bytes + self.pool_bytes + need <= self.budget:
                    if not fut.set_running_or_notify_cancel():
                        del self.queue[i]
                        break
                    self.busy_bytes += need
                    self.peak_bytes = max(self.peak_bytes, self.busy_bytes + self.pool_bytes)
                    del self.queue[i]
                    return req, fut, None, need
            else:
                if self.queue:
                    self.admission_waits += 1
                self.cv.wait(timeout=0.05)

    def _worker(self, stream):
        try:
            if self.device.type == "cuda":
                torch.cuda.set_device(self.device)
        except Exception as e:          # a slot that cannot start fails its requests
            self._fail_all(e)
            return
        while True:
            with self.cv:
                try:
                    item = self._take()
                except Exception as e:      # scheduler bug: fail what waits, stop cleanly
                    item = e
            if isinstance(item, Exception):
                self._fail_all(item)
                return
            if item is None:
                return
            req, fut, prob, need = item
            # the future is already running (set in _take), so it cannot be
            # cancelled any more and takes exactly one result or exception
            try:
                req.t_admit = time.perf_counter()
                out = self._run(req, prob, need, stream)
            except Exception as e:      # the request fails, the slot goes on
                fut.set_exception(e)
            else:
                fut.set_result(out)

    def _fail_all(self, exc):
        with self.cv:
            while self.queue:
                _, fut = self.queue.popleft()
                if fut.set_running_or_notify_cancel():
                    fut.set_exception(exc)
            self.closed = True
            self.cv.notify_all()

    def _run(self, req, prob, need, stream):
        """Runs one admitted request.  It holds `need` bytes (a new problem)
        or its pooled problem's bytes; on success the problem goes back to
        the pool, on failure it is closed (its state is not trusted) and the
        bytes are released before the exception propagates."""
        holding = need if prob is None else prob.workspace_bytes + 256
        made = []                       # the problem _solve builds, if any
        try:
            out = self._solve(req, prob, stream, made)
        except BaseException:
            prob = made[0] if prob is None and made else prob
            if prob is not None:
                prob.close()
            with self.cv:
                self.busy_bytes -= holding
                self.cv.notify_all()
            raise
        prob = out.pop("_problem")
        with self.cv:
            key = req.key
            self.busy_bytes -= holding
            self.pool.setdefault(key, []).append(prob)
            self.pool.move_to_end(key)
            self.pool_bytes += prob.workspace_bytes + 256
            self.peak_bytes = max(self.peak_bytes, self.busy_bytes + self.pool_bytes)
            self.stats.append(out)
            self.cv.notify_all()
        return out

    def _solve(self, req, prob, stream, made):
        ctx = torch.cuda.stream(stream) if stream is not None else _nullctx()
        with ctx:
            if prob is None:
                prob = self.make_problem(req, self.device, stream)
                made.append(prob)
            else:
                if stream is not None:
                    prob.set_stream(stream)
                prob.update_density(torch.as_tensor(req.rho, dtype=torch.float64))
            T, info = prob.solve(allow_not_converged=True)
            out = dict(id=req.id, iterations=info.iterations, true_rel_res=info.true_rel_res)
            if req.adjoint:
                f = prob.load_vector()
                lam, ainfo = prob.adjoint(f, allow_not_converged=True)
                out["grad"] = prob.sensitivity(T, lam)
                out["adjoint_iterations"] = ainfo.iterations
                out["adjoint_true_rel_res"] = ainfo.true_rel_res
                out["J"] = prob.objective(T)
                out["lam"] = lam if self.keep_outputs else None
            out["T"] = T if self.keep_outputs else None
            if stream is not None:
                stream.synchronize()
        req.t_done = time.perf_counter()
        out.update(latency_s=req.t_done - req.t_arrive, queue_s=req.t_admit - req.t_arrive,
                   dofs=req.dofs, _problem=prob)
        return out


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def request_density(n, nt, seed):
    """Random time-varying density for a serving request: Gaussian noise on a
    coarse 8^3 lattice, trilinearly interpolated to the element grid and mapped
    to [0.001, 1] through the normal CDF."""
    from scipy.ndimage import zoom
    from scipy.special import ndtr
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((8, 8, 8))
    z = zoom(z, (nt / 8, n / 8, n / 8), order=1, mode="nearest")[:nt, :n, :n]
    z = (z - z.mean()) / (z.std() + 1e-30)
    return 0.001 + 0.999 * ndtr(z)


def run_stream(requests, server, realtime=True):
    """Replays (request, arrival offset) pairs against a server; returns the
    per-request results and the makespan."""
    t0 = time.perf_counter()
    futs = []
    for req, t_off in requests:
        if realtime:
            dt = t0 + t_off - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        req.t_arrive = time.perf_counter()
        futs.append(server.submit(req))
    results = [f.result() for f in futs]
    return results, time.perf_counter() - t0

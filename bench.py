"""Benchmark: space-time DOFs solved per second to a 1e-8 relative residual.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|medium|...]
                    [--precision mixed|fp64] [--no-cpu-baseline] [--no-compare-fp64]

A step is one complete st_solve (FGMRES + space-time multigrid V-cycles, from
a zero initial guess) of the workload; the design, hierarchy and right-hand
side are resident in HBM before the timed region starts (setup is reported
separately).  DOFs = all (nx+1)(ny+1)(nt+1) nodes, Dirichlet nodes included.

Prints one JSON line with the throughput, the roofline of the dominant kernel
class (algorithmic bytes / GPU time from HIP events recorded around each of
its launches on the solver's stream during the timed steps) and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2508_09589_amd", "csrc", "kernels_fine.hip")
ROOF_KERNEL = {"mixed": "k_fine_apply<float, float, float, false",
               "fp64": "k_fine_apply<double, double, double, false"}
COPY_KIB = 1 << 20      # the calibration copy moves 1 GiB each way


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_problem(name, precision, time_kernels, bf16_from_level=0, max_it=1000,
                     smoother="gmres", restart=None, coarse="direct", max_levels=None):
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import WORKLOADS, workload_density
    w = WORKLOADS[name]
    rho = workload_density(name)
    if restart is None:
        restart = 20 if name == "large" else 30
    t0 = time.perf_counter()
    extra = {} if max_levels is None else dict(max_levels=max_levels)
    p = Problem(w["nx"], w["ny"], w["nt"], torch.tensor(rho), precision=precision, restart=restart,
                rtol=1e-8, time_kernels=time_kernels, bf16_from_level=bf16_from_level,
                smoother=smoother, coarse=coarse,
                max_it=max_it, **extra)
    torch.cuda.synchronize()
    log(f"{name} {precision}: setup {time.perf_counter() - t0:.2f} s, {p.n_nodes} nodes, "
        f"levels {p.hierarchy()[0]}")
    return p, time.perf_counter() - t0, restart


def _kernel_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_path(workload, precision):
    return os.path.join(ROOT, "profiles", f"fine_apply_{workload}_{precision}_hbm_traffic.md")


def recorded_traffic(workload, precision):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when there is none or it was taken on other kernel source."""
    path = traffic_path(workload, precision)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != _kernel_sha():
        return None
    try:
        return float(fields["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def summarize_counters(fetch_dir, write_dir, workload, precision, out):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; each with
    --copy-calibration) into the traffic summary of the roofline kernel:
    counters averaged over its dispatches and scaled by what they read for the
    1 GiB copies."""
    import csv
    import glob

    def rows(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        out_rows = []
        for fn in files:
            with open(fn) as f:
                out_rows += [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        return out_rows

    fr, wr = rows(fetch_dir, "FETCH_SIZE"), rows(write_dir, "WRITE_SIZE")
    kern = ROOF_KERNEL[precision]
    fk = [float(r["Counter_Value"]) for r in fr if kern in r["Kernel_Name"]]
    wk = [float(r["Counter_Value"]) for r in wr if kern in r["Kernel_Name"]]
    cw = [r for r in wr if "copy" in r["Kernel_Name"].lower()
          and abs(float(r["Counter_Value"]) - COPY_KIB) <= 0.01 * COPY_KIB]
    ids = {r["Dispatch_Id"] for r in cw}
    cf = [float(r["Counter_Value"]) for r in fr if r["Dispatch_Id"] in ids and "copy" in r["Kernel_Name"].lower()]
    if not fk or not wk or not cw or not cf:
        raise SystemExit("counter runs lack the roofline kernel or the calibration copies")
    ff = COPY_KIB / (sum(cf) / len(cf))
    fw = COPY_KIB / (sum(float(r["Counter_Value"]) for r in cw) / len(cw))
    fa, wa = sum(fk) / len(fk), sum(wk) / len(wk)
    total = (fa * ff + wa * fw) * 1024.0
    cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 240 rocprofv3 --pmc {c} "
           "--kernel-include-regex 'k_fine_apply|copy' --output-format csv -d <dir> -o run -- "
           f"python -u /root/repo/bench.py --workload {workload} --precision {precision} "
           "--steps 1 --warmup 1 --no-cpu-baseline --no-compare-fp64 --max-levels 32 "
           "--copy-calibration")
    text = f"""# HBM traffic of the fine-level apply, {workload} workload, {precision} precision

Two rocprofv3 counter runs of the same command, one counter each:

    {cmd.format(c="FETCH_SIZE")}
    {cmd.format(c="WRITE_SIZE")}

then `python bench.py --summarize-counters <fetch dir> <write dir> --workload {workload} --precision {precision}`.
The counters are averaged over the kernel's dispatches and scaled by what they read for
the 1 GiB device copies at the end of the run (1 GiB read and 1 GiB written each).
The counter runs coarsen down to at most 4096 nodes (`--max-levels 32`): rocprofv3's
counter collection ends the process in the launch of the coarsest-level factorisation's
panel kernel (148 KB of LDS) that the default 8-level hierarchy uses; the fine-level
apply, whose traffic this is, is the same kernel with the same launch shape either way.

kernel: {kern} ... ({len(fk)} / {len(wk)} dispatches)
source_sha256: {_kernel_sha()}
fetch_kib_per_dispatch: {fa:.1f}
write_kib_per_dispatch: {wa:.1f}
copy_fetch_kib: {sum(cf) / len(cf):.1f}
copy_write_kib: {sum(float(r["Counter_Value"]) for r in cw) / len(cw):.1f}
fetch_scale: {ff:.4f}
write_scale: {fw:.4f}
bytes_per_launch: {total:.0f}
"""
    with open(out, "w") as f:
        f.write(text)
    print(text)


def summarize_stats(stats_dir, title, command, out, top=20):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (the
    *kernel_stats.csv it writes): calls, total and average time per kernel,
    largest first."""
    import csv
    import glob
    files = glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {stats_dir}")
    rows = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                name = r["Name"]
                c, t = int(r["Calls"]), float(r["TotalDurationNs"])
                pc, pt = rows.get(name, (0, 0.0))
                rows[name] = (pc + c, pt + t)
    total = sum(t for _, t in rows.values())
    lines = [f"# rocprofv3 kernel statistics: {title}", "",
             "Command (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             f"    {command}", "",
             f"Total kernel time {total / 1e6:.1f} ms. Top kernels by total time:", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, (c, t) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:top]:
        short = name.split("(")[0]
        lines.append(f"| `{short}` | {c} | {t / 1e6:.2f} | {t / c / 1e3:.1f} | "
                     f"{100 * t / total:.1f} |")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


def cpu_baseline(name):
    """The FP64 oracle (block Gauss-Seidel in time with exact 2-D sparse LU
    blocks) on the first few time slabs of the same grid, same dt, to the same
    1e-8 relative residual.  Single-threaded (SuperLU)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.assemble import Material, load_vector, simp
    from oracle.grid import Grid, dirichlet_mask
    from oracle.solve import BlockTimeSystem
    from paper_2508_09589_amd.inputs import WORKLOADS, workload_density
    w = WORKLOADS[name]
    rho = workload_density(name)
    slabs = {"large": 8, "medium": 32, "grad": 32, "small": 32}[name]
    k, _, _, _ = simp(rho, Material(k_ins=1e-3, k_con=1.0, p_k=3.0, c_ins=1.0, c_con=1.0, p_c=1.0))
    if k.ndim == 3:
        k = k[:slabs]
    g = Grid(w["nx"], w["ny"], slabs, 1.0 / w["nx"], 1.0 / w["nt"])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        mask = dirichlet_mask(g, [(0, 0.5, 0.05)])
        f = load_vector(g, 1.0)
        bs = BlockTimeSystem(g, k, np.ones_like(k), mask)
        s, sweeps, rel = bs.gauss_seidel(bs.masked_rhs(f), tol=1e-8)
        dt = time.perf_counter() - t0
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": g.n_nodes / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"first {slabs} of {w['nt']} time slabs of the {w['nx']}x{w['ny']} grid "
                      f"({g.n_nodes} nodes), block Gauss-Seidel in time with SuperLU blocks, "
                      f"{sweeps} sweeps to rel. residual {rel:.1e}, {dt:.1f} s",
            "seconds": dt, "threads_used": 1, "host_cpu_count": os.cpu_count(),
            "host_affinity_cores": affinity,
            "note": "the oracle as written (SuperLU factorisations and triangular solves, "
                    "one thread); not an optimised CPU solver"}


def run(args):
    import torch
    from paper_2508_09589_amd.solver import info_dict
    from paper_2508_09589_amd import _lib as L

    p, t_setup, restart = workload_problem(args.workload, args.precision, True,
                                           args.bf16_from_level, args.max_it, args.smoother,
                                           args.restart, args.coarse, args.max_levels)
    n_nodes = p.n_nodes
    # The first warm-up solve times every kernel class (one event pair per
    # launch); the others run untimed.
    kern = None
    for w in range(max(args.warmup, 1)):
        t0 = time.perf_counter()
        T, info = p.solve(allow_not_converged=True)
        if w == 0:
            kern = info_dict(info)["kernels"]
            p.set_flags(p.opts.flags & ~L.ST_FLAG_TIME_KERNELS)
        log(f"warm-up solve: {info.iterations} its, true rel res {info.true_rel_res:.2e}, "
            f"{time.perf_counter() - t0:.2f} s" + (" (all kernel classes timed)" if w == 0 else ""))
    # The roofline names the fine-level matrix-free apply in the precision the
    # V-cycle runs in: the defining operator of the method, one kernel of one
    # shape per launch, and with the coarse-level stencils and the smoother's
    # vector passes one of the three largest shares of GPU time.  The
    # coarsest-level solve (one workgroup, L2-resident) has no byte model and
    # is reported as a share.
    dom = "fine_apply_vcycle" if args.precision == "mixed" else "fine_apply_fp64"
    total_ms = sum(v["ms"] for v in kern.values())
    dom_idx = L.KCLASS_NAMES.index(dom)
    # Timed steps record events only around launches of the dominant class.
    p.set_flags(p.opts.flags | L.ST_FLAG_TIME_KERNELS | (1 << (8 + dom_idx)))
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        T, info = p.solve(allow_not_converged=True)
        infos.append(info_dict(info))
        log(f"step {k}: {info.iterations} its, {info.t_solve_s:.3f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = n_nodes * args.steps / elapsed
    ms = sum(i["kernels"].get(dom, {}).get("ms", 0.0) for i in infos)
    launches = sum(i["kernels"].get(dom, {}).get("launches", 0) for i in infos)
    nbytes = sum(i["kernels"].get(dom, {}).get("bytes", 0) for i in infos)
    achieved = (nbytes / (ms * 1e-3)) / 1e9 if ms > 0 else 0.0
    last = infos[-1]
    out = {
        "metric": "space-time DOFs solved/s to 1e-8 rel. residual; operator-apply HBM GB/s",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [p.nx, p.ny, p.nt], "dofs": n_nodes,
                   "precision": args.precision, "fgmres_restart": restart, "rtol": 1e-8,
                   "levels": last["levels"], "iterations": last["iterations"],
                   "true_rel_res": last["true_rel_res"], "setup_s": t_setup,
                   "converged": last["true_rel_res"] <= 1e-8,
                   "bf16_from_level": args.bf16_from_level, "smoother": args.smoother,
                   "coarse": args.coarse, "hierarchy": [list(d) for d in p.hierarchy()[0]]},
        "roofline": {"bound": "hbm", "kernel_class": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(args.workload, args.precision),
                     "launches": launches,
                     "avg_launch_ms": ms / launches if launches else None,
                     "bytes_per_launch": nbytes / launches if launches else None},
        "kernel_classes_warmup_ms": {c: round(v["ms"], 3) for c, v in kern.items()},
        # algorithmic bytes / GPU time of every kernel class in the warm-up
        # solve (GB/s; against the 8 TB/s HBM peak)
        "kernel_classes_warmup_gbs": {c: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
                                      for c, v in kern.items() if v["ms"] > 0 and v["bytes"] > 0},
        "coarse_solve_share": kern.get("coarse_solve", {}).get("ms", 0.0) / total_ms if total_ms else None,
    }
    p.close()
    out["copy_ceiling"] = copy_ceiling()
    out["roofline"]["frac_of_copy_ceiling"] = achieved / out["copy_ceiling"]["gbs"]
    torch.cuda.empty_cache()
    if not args.no_compare_fp64 and args.precision != "fp64":
        # Plain FP64 at the same settings (smoother, coarse solve, restart,
        # 1e-8): the mixed problem is closed first (both do not fit at once on
        # the large grid); its solution stays for the difference.
        out["fp64_compare"] = fp64_compare(args, T, n_nodes, out["value"])
    del T
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    return out


def fp64_compare(args, T_mixed, n_nodes, mixed_value):
    """Plain FP64 solve of the same workload with the same smoother, coarse
    solve, restart and tolerance; timed solves from a zero initial guess
    (one on the large grid, two elsewhere, after one warm-up)."""
    import torch
    q, ts, _ = workload_problem(args.workload, "fp64", False, 0, args.max_it, args.smoother,
                                args.restart, args.coarse, args.max_levels)
    timed = 1 if args.workload == "large" else 2
    if args.workload != "large":
        q.solve(allow_not_converged=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(timed):
        Tq, iq = q.solve(allow_not_converged=True)
    torch.cuda.synchronize()
    dtq = (time.perf_counter() - t0) / timed
    diff = float(torch.linalg.vector_norm(T_mixed - Tq) / torch.linalg.vector_norm(Tq))
    log(f"fp64 compare: {iq.iterations} its, true rel res {iq.true_rel_res:.2e}, {dtq:.2f} s/solve, "
        f"|T_mixed - T_fp64| / |T_fp64| = {diff:.2e}")
    res = {"value": n_nodes / dtq, "unit": "DOF/s", "ms_per_step": dtq * 1e3, "timed_solves": timed,
           "iterations": iq.iterations, "true_rel_res": iq.true_rel_res,
           "converged": iq.true_rel_res <= 1e-8, "setup_s": ts,
           "mixed_over_fp64": mixed_value / (n_nodes / dtq),
           "rel_diff_mixed_vs_fp64": diff,
           "settings": {"smoother": args.smoother, "coarse": args.coarse,
                        "fgmres_restart": 20 if args.workload == "large" and args.restart is None
                        else (args.restart or 30), "rtol": 1e-8}}
    q.close()
    del Tq
    return res


def copy_ceiling():
    """Measured device-copy bandwidth: a 1 GiB FP32 copy (1 GiB read + 1 GiB
    written), best of five, timed with HIP events."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del x, y
    return {"gbs": 2 * (1 << 30) / (best * 1e-3) / 1e9, "bytes": 2 * (1 << 30),
            "what": "1 GiB FP32 device copy, read + write, best of 5"}


def run_serving(args):
    """Serving workload: 256 requests, exponential inter-arrival times (mean
    20 ms), n ~ U{32,64,128,256}, nt ~ U{32,64,128,256}, half forward-only and
    half forward + adjoint gradient; continuous batching over 4 slots."""
    import numpy as np
    import torch
    from paper_2508_09589_amd.inputs import serving_requests
    from paper_2508_09589_amd.serve import Request, Server, request_density, run_stream
    specs = serving_requests(args.requests)
    t0 = time.perf_counter()
    dens = {r["id"]: request_density(r["n"], r["nt"], r["seed"]) for r in specs}
    log(f"serving: {len(specs)} request densities generated in {time.perf_counter() - t0:.1f} s")
    res = {}
    for prec in (["mixed", "fp64"] if args.compare_fp64 else [args.precision]):
        srv = Server(int(args.hbm_budget_gb * (1 << 30)), slots=args.slots, keep_outputs=False)
        stream = [(Request(r["id"], r["n"], r["nt"], dens[r["id"]], adjoint=r["adjoint"],
                           precision=prec, smoother=args.smoother), r["t_arrive"]) for r in specs]
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        out, makespan = run_stream(stream, srv)
        srv.close()
        lat = np.array([o["latency_s"] for o in out])
        dofs = sum(o["dofs"] for o in out)
        its = np.array([o["iterations"] for o in out])
        res[prec] = {"value": dofs / makespan, "makespan_s": makespan,
                     "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)),
                     "mean_queue_s": float(np.mean([o["queue_s"] for o in out])),
                     "admission_waits": srv.admission_waits,
                     "peak_workspace_gb": srv.peak_bytes / 2 ** 30,
                     "peak_torch_allocated_gb": torch.cuda.max_memory_allocated() / 2 ** 30,
                     "median_iterations": float(np.median(its)),
                     "max_true_rel_res": float(max(o["true_rel_res"] for o in out))}
        log(f"serving {prec}: {dofs / makespan / 1e6:.2f} MDOF/s, p50 {res[prec]['p50_latency_s']:.3f} s, "
            f"p99 {res[prec]['p99_latency_s']:.3f} s, makespan {makespan:.1f} s")
        torch.cuda.empty_cache()
    main_prec = "mixed" if "mixed" in res else args.precision
    out = {"metric": "space-time DOFs solved/s to 1e-8 rel. residual (serving, aggregate)",
           "value": res[main_prec]["value"], "unit": "DOF/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": res[main_prec]["makespan_s"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if main_prec == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": "serving", "requests": len(specs), "arrival_rate_per_s": 50,
                      "slots": args.slots, "hbm_budget_gb": args.hbm_budget_gb},
           "serving": res}
    return out


def run_design(args):
    """Design iterations of the §3.3 chain on the differentiation grid
    (128^2 x 128, time-varying design, PDE filter r = 1.5 elements, Heaviside
    projection beta = 32, p-norm P = 20, volume fraction 0.3): per iteration
    the design is updated by a fixed-size normalised descent step (a stand-in
    for MMA, which is out of scope), then filter + projection + SIMP +
    Galerkin rebuild, the warm-started state solve, the p-norm and its
    adjoint solve (warm-started from the previous adjoint), the sensitivities
    and the volume constraint."""
    import numpy as np
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import workload_density
    rho = torch.tensor(workload_density("grad"), dtype=torch.float64, device="cuda")
    n = rho.shape[-1]
    p = Problem(n, n, rho.shape[0], rho, filter_r=1.5, proj_beta=32.0, proj_eta=0.5,
                precision=args.precision, rtol=1e-8, bf16_from_level=args.bf16_from_level,
                smoother=args.smoother)
    T = lam = None
    rec = []

    def iteration():
        nonlocal rho, T, lam
        t0 = time.perf_counter()
        T, i1 = p.solve(x0=T, allow_not_converged=True)
        phi, dphi = p.pnorm(T, 20.0)
        lam, i2 = p.adjoint(dphi, lam0=lam, allow_not_converged=True)
        g = p.sensitivity(T, lam)
        chi, dchi = p.volume(0.3)
        step = 0.02 * g / (g.abs().max() + 1e-300)
        rho = torch.clamp(rho - step, 0.0, 1.0)
        p.update_density(rho)
        torch.cuda.synchronize()
        return dict(phi=phi, chi=chi, fwd_its=i1.iterations, adj_its=i2.iterations,
                    s=time.perf_counter() - t0)

    for _ in range(max(args.warmup, 1)):
        r = iteration()
        log(f"design warm-up: phi {r['phi']:.6g}, chi {r['chi']:.4f}, its {r['fwd_its']}/{r['adj_its']}")
    t0 = time.perf_counter()
    for k in range(args.steps):
        rec.append(iteration())
        log(f"design iteration {k}: phi {rec[-1]['phi']:.6g}, its {rec[-1]['fwd_its']}/{rec[-1]['adj_its']}, "
            f"{rec[-1]['s']:.3f} s")
    elapsed = time.perf_counter() - t0
    nodes = p.n_nodes
    p.close()
    return {"metric": "design iterations/s (state + adjoint solve, p-norm, sensitivities, "
                      "filter, projection, rebuild)",
            "value": args.steps / elapsed, "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
            "config": {"workload": "design", "grid": [n, n, n], "dofs": nodes, "filter_r": 1.5,
                       "proj_beta": 32.0, "P": 20.0, "vf": 0.3,
                       "fwd_its": [r["fwd_its"] for r in rec], "adj_its": [r["adj_its"] for r in rec],
                       "phi": [r["phi"] for r in rec]},
            "dofs_per_s_both_solves": 2 * nodes * args.steps / elapsed}


def run_coarsening(args):
    """Semi- against full space-time coarsening on the paper's examples (§2.3)
    at a reduced grid (default 160^2 x 320): per material variant (1B, 1D, 2B,
    2C), design (uniform 0.3 start, binary tree) and coarsest-level solver
    (exact, or the paper's Jacobi-GMRES), the FGMRES iterations and solve
    times of the state solve and of the adjoint solve for the p-norm
    objective (P = 20), at the paper's outer tolerance 1e-5.  The value is
    the state + adjoint DOF throughput of the semi-coarsened, exact-coarse
    runs."""
    import numpy as np
    import torch
    from paper_2508_09589_amd import Problem
    from paper_2508_09589_amd.inputs import example_design, example_problem
    n, nt = args.example_n, 2 * args.example_n
    rows = []
    for variant in ("1B", "1D", "2B", "2C"):
        kw = example_problem(variant, n, nt)
        for design in ("uniform", "tree"):
            rho = torch.tensor(example_design(design, n))
            for coarse in ("direct", "gmres"):
                for coarsening in ("semi", "full"):
                    t0 = time.perf_counter()
                    p = Problem(rho=rho, precision=args.precision, rtol=args.rtol, coarse=coarse,
                                coarsening=coarsening, max_it=args.max_it,
                                bf16_from_level=args.bf16_from_level, smoother=args.smoother,
                                **kw)
                    torch.cuda.synchronize()
                    setup = time.perf_counter() - t0
                    t0 = time.perf_counter()
                    T, si = p.solve(allow_not_converged=True)
                    torch.cuda.synchronize()
                    ts = time.perf_counter() - t0
                    _, dphi = p.pnorm(T, 20.0)
                    t0 = time.perf_counter()
                    lam, ai = p.adjoint(dphi, allow_not_converged=True)
                    torch.cuda.synchronize()
                    ta = time.perf_counter() - t0
                    r = dict(variant=variant, design=design, coarse=coarse, coarsening=coarsening,
                             levels=len(p.hierarchy()[0]), state_its=si.iterations,
                             adjoint_its=ai.iterations, state_s=ts, adjoint_s=ta, setup_s=setup,
                             state_rel_res=si.true_rel_res, adjoint_rel_res=ai.true_rel_res,
                             dofs=p.n_nodes)
                    rows.append(r)
                    log(f"{variant} {design:7s} {coarse:6s} {coarsening}: levels {r['levels']}, "
                        f"its {si.iterations}/{ai.iterations}, {ts:.3f}/{ta:.3f} s, "
                        f"res {si.true_rel_res:.2e}/{ai.true_rel_res:.2e}")
                    p.close()
                    del T, lam, dphi
    sel = [r for r in rows if r["coarse"] == "direct" and r["coarsening"] == "semi"]
    secs = sum(r["state_s"] + r["adjoint_s"] for r in sel)
    dofs = sum(2 * r["dofs"] for r in sel)

    def mean_its(coarse, coarsening, key):
        v = [r[key] for r in rows if r["coarse"] == coarse and r["coarsening"] == coarsening]
        return float(np.mean(v))

    summary = {f"{c}/{m}": {"state": mean_its(c, m, "state_its"), "adjoint": mean_its(c, m, "adjoint_its")}
               for c in ("direct", "gmres") for m in ("semi", "full")}
    return {"metric": "state + adjoint DOFs solved/s on the example problems (semi-coarsening)",
            "value": dofs / secs, "unit": "DOF/s", "n_gpus": 1, "steps": len(sel), "warmup": 0,
            "ms_per_step": secs / len(sel) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64" if args.precision == "mixed" else "f64",
            "data": "synthetic",
            "config": {"workload": "coarsening", "grid": [n, n, nt], "rtol": args.rtol,
                       "variants": ["1B", "1D", "2B", "2C"], "designs": ["uniform", "tree"]},
            "mean_iterations": summary, "runs": rows}


def copy_calibration():
    """Three copies of a 1 GiB FP32 buffer: 1 GiB read and 1 GiB written per
    dispatch, the reference for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copy calibration: 3 x 1 GiB device copies done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large",
                    choices=["small", "medium", "large", "grad", "serving", "design", "coarsening"])
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--bf16-from-level", type=int, default=1,
                    help="mixed precision: store coarse stencils of levels >= this in BF16 "
                         "(0 = FP32 everywhere)")
    ap.add_argument("--smoother", default="sstep", choices=["gmres", "sstep"],
                    help="Jacobi-GMRES smoothing in s-step form (one Gram pass) or by "
                         "Arnoldi steps")
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES restart length (default 30; 20 for the large workload)")
    ap.add_argument("--coarse", default="direct", choices=["direct", "gmres"],
                    help="coarsest-level solve: exact, or the paper's Jacobi-GMRES")
    ap.add_argument("--max-levels", type=int, default=None,
                    help="multigrid levels N_l (default: the library's, 8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="serving workload: also run the request stream in plain FP64")
    ap.add_argument("--no-compare-fp64", action="store_true",
                    help="skip the plain FP64 solve that follows the timed mixed solves")
    ap.add_argument("--max-it", type=int, default=400)
    ap.add_argument("--example-n", type=int, default=160,
                    help="coarsening workload: spatial elements per side (nt = 2 n)")
    ap.add_argument("--rtol", type=float, default=1e-5,
                    help="coarsening workload: outer FGMRES tolerance (the paper's 1e-5)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the roofline kernel's HBM traffic summary from two rocprofv3 "
                         "--pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--out", default=None, help="output path of --summarize-counters / -stats")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("STATS_DIR", "TITLE", "COMMAND"),
                    help="write a markdown summary of a rocprofv3 --kernel-trace --stats run "
                         "to --out and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 1 GiB device buffers three times (a plain copy "
                         "kernel of known size, for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, out=args.out or "kernel_stats.md")
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.workload,
                           args.precision, args.out or traffic_path(args.workload, args.precision))
        return
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU time-slab sharding is a design only)", file=sys.stderr)
        sys.exit(2)
    runner = {"serving": run_serving, "design": run_design,
              "coarsening": run_coarsening}.get(args.workload, run)
    print(json.dumps(runner(args)), flush=True)
    if args.copy_calibration:
        copy_calibration()


if __name__ == "__main__":
    main()

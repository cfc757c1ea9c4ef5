#!/usr/bin/env python3
"""Benchmark of the spectral two-level PCG hot path on one MI355X.

One step = one robust design iteration of the paper's method on the
1024 x 512 bilinear-element cantilever (1,051,650 DOFs, 3 realisations at
eta = 0.3 / 0.5 / 0.7): density filter and projection, the spectral coarse
basis (local eigenproblems of the dilated design) with every local and coarse
factor, the batched PCG solve of the three systems to a relative residual of
1e-8 from a zero start, compliance and sensitivities, and the chain rule back
to the design field. All inputs are resident on the GPU before timing.

value = sum over systems of (DOFs x PCG iterations) / step time (FP64).
The same steps are then run with the mixed-precision preconditioner. After
the timed steps, the paper's own solver (restarted GMRES with the MsFEM coarse
solve between symmetric Gauss-Seidel steps, and with additive Schwarz) is
timed on the last build and reported beside them ("paper_solver").

--workload cantilever3d runs the trilinear-element cantilever of 192 x 96 x
96 elements (5,447,811 DOFs, one system, layered 0/1 microstructure, no
filter) on subdomains of 16^3 elements instead: one step = coarse basis and
factors, PCG to 1e-8, compliance and sensitivities. Its layered design has
about twelve near-zero modes per subdomain (two solid plates joined by void),
so it runs with the paper's eigenvalue threshold (--lambda-thresh, default
1e-6) and at most 16 coarse vectors per subdomain; --lambda-thresh 0
--ncoarse 8 runs the fixed count of 8.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILES = {
    "cantilever2d": os.path.join(ROOT, "profiles", "local_solves_cantilever2d_1024x512_traffic.json"),
    "cantilever3d": os.path.join(ROOT, "profiles", "local_solves_cantilever3d_192x96x96_traffic.json"),
}
TRAFFIC_FILE = TRAFFIC_FILES["cantilever2d"]
KERNEL_SOURCES = {
    "cantilever2d": ["paper_1411_3923_amd/csrc/btri.h", "paper_1411_3923_amd/csrc/local.hip"],
    "cantilever3d": ["paper_1411_3923_amd/csrc/btri.h", "paper_1411_3923_amd/csrc/big.hip",
                     "paper_1411_3923_amd/csrc/big.h"],
}
ROOFLINE_KERNEL = {"cantilever2d": "k_local_solves<double>",
                   "cantilever3d": "k_big_solve_{fwd,mid,bwd}<double>"}
COPY_BYTES = 1 << 30


def kernel_hash(workload="cantilever2d"):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[workload]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def run_gpu(precision, args, p, rho_h, f_h):
    import numpy as np
    import torch

    import paper_1411_3923_amd as T
    from paper_1411_3923_amd import workloads as W

    pr = T.make_problem(p.dim, p.nel[:p.dim], p.sub, p.k, p.nsys, p.E0, p.Emin, p.penal, p.nu,
                        precision, eig_iters=args.eig_iters, eig_extra=args.eig_extra,
                        lambda_thresh=args.lambda_thresh)
    h = T.Handle(pr, W.fixed_mask(p))
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    rho = d(rho_h)
    F = d(np.stack([f_h] * p.nsys))
    rt = torch.zeros(p.n_el, dtype=torch.float64, device="cuda")
    rb = torch.zeros((p.nsys, p.n_el), dtype=torch.float64, device="cuda")
    u = torch.zeros((p.nsys, p.n_dof), dtype=torch.float64, device="cuda")
    c = torch.zeros(p.nsys, dtype=torch.float64, device="cuda")
    dc = torch.zeros((p.nsys, p.n_el), dtype=torch.float64, device="cuda")
    dcr = torch.zeros((p.nsys, p.n_el), dtype=torch.float64, device="cuda")

    filtered = p.rmin > 0.0
    if not filtered:
        rb.copy_(rho.view(1, -1).expand(p.nsys, -1))   # unfiltered design: rho_phys = rho

    def step():
        t0 = time.perf_counter()
        if filtered:
            h.filter_project(rho, p.rmin, p.beta, p.etas, rt, rb)
        h.build_coarse_basis(rb, rep=0)          # blocks until the factors are done
        t1 = time.perf_counter()
        u.zero_()
        info = h.pcg_solve(rb, F, u, rtol=args.rtol, maxit=args.maxit)   # blocks
        h.compliance_and_sensitivity(rb, u, F, c, dc)
        if filtered:
            h.filter_project_adjoint(rt, p.rmin, p.beta, p.etas, dc, dcr)
        return info, (t1 - t0) * 1e3

    # long steps (3-d: seconds each) report their end on stderr
    tw = time.perf_counter()
    report = lambda what: (print(f"{'mixed' if precision == T.MIXED else 'fp64'} {what} done at "
                                 f"{time.perf_counter() - tw:.1f} s", file=sys.stderr, flush=True)
                           if p.dim == 3 else None)
    for i in range(args.warmup):
        step()
        report(f"warm-up step {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    h.set_profiling(True)
    infos, setup_ms, solve_ms = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        info, sm = step()
        infos.append(info)
        setup_ms.append(sm)
        solve_ms.append(info[0]["seconds"] * 1e3)
        report(f"timed step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile_block_solves()
    h.set_profiling(False)
    # the paper's own solver (Sec. 2.4.2) on the same preconditioner build:
    # restarted GMRES with the MsFEM cycle between symmetric Gauss-Seidel
    # steps, and with additive Schwarz; its stopping test is the
    # preconditioned residual. Reported beside the timed steps, not in them.
    paper = {"restart": args.gmres_restart, "rtol_preconditioned": args.rtol}
    kinds = (("gmres_msfem_sgs", T.PC_MSFEM_SGS), ("gmres_additive", T.PC_ADDITIVE))
    for name, pc in (kinds if args.gmres_reps > 0 else ()):
        ms, info = [], None
        for _ in range(args.gmres_reps):
            ug = torch.zeros_like(u)
            info = h.gmres_solve(rb, F, ug, rtol=args.rtol, maxit=args.maxit,
                                 restart=args.gmres_restart, precond=pc)
            ms.append(info[0]["seconds"] * 1e3)
        its = [i["iters"] for i in info]
        paper[name] = {"iters": its, "status": [i["status"] for i in info],
                       "solve_ms_p50": percentile(ms, 50),
                       "dof_iters_per_s": sum(p.n_dof * it for it in its) / (percentile(ms, 50) * 1e-3),
                       "relres_preconditioned": [i["relres"] for i in info],
                       "true_relres": [i["true_relres"] for i in info]}
    _, lam, eres = h.export_coarse_basis()
    _, kj = h.export_eigenvalues()
    ms_step = (t1 - t0) * 1e3 / args.steps
    iters = [i["iters"] for i in infos[-1]]
    work = sum(p.n_dof * it for it in iters)
    out = {
        "ms_per_step": ms_step,
        "dof_iters_per_s": work / (ms_step * 1e-3),
        "solve_only_dof_iters_per_s": work / (percentile(solve_ms, 50) * 1e-3),
        "solve_ms_p50": percentile(solve_ms, 50),
        "solve_ms_p99": percentile(solve_ms, 99),
        "setup_ms_p50": percentile(setup_ms, 50),
        "iters": iters,
        "relres": [i["relres"] for i in infos[-1]],
        "true_relres": [i["true_relres"] for i in infos[-1]],
        "status": [i["status"] for i in infos[-1]],
        "compliance": [float(x) for x in c.cpu()],
        "block_solves": prof,
        "paper_solver": paper,
        "eig_max_ritz_residual": float(np.max(eres)),
        "coarse_vectors_per_subdomain": {"min": int(kj.min()), "max": int(kj.max()),
                                         "mean": float(kj.mean()), "total": int(kj.sum())},
        "u": u.cpu().numpy(),
        "dc": dc.cpu().numpy(),
    }
    h.close()
    return out


def cpu_baseline(args):
    """The oracle on a bounded sample of the same workload, same step definition."""
    import numpy as np

    from oracle import density, fem, schwarz
    from paper_1411_3923_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    if args.workload == "cantilever3d":
        # a 32 x 16 x 16 section (two of the 16^3 cells) of the same layered
        # design, the same coarse-space rule, the oracle's sparse shift-invert
        # eigensolver (its dense one does not finish on cells of 14,739 DOFs)
        p = W.cantilever3d(32, 16, 16, sub=16, k=args.ncoarse)
        rho = W.design_field(p)
        fixed, f = W.fixed_mask(p), W.load_vector(p)
        t0 = time.perf_counter()
        res = schwarz.solve_pcg(p, [rho], rho, f, fixed, rtol=args.rtol, maxit=args.maxit,
                                thresh=args.lambda_thresh, eig_method="sparse")
        fem.sensitivity(p, rho, res[0][0])
        fem.compliance(f, res[0][0])
        t1 = time.perf_counter()
        work = p.n_dof * res[0][1]
        sample = (f"one full step (spectral basis, PCG to {args.rtol:g}, sensitivities) on a "
                  f"32x16x16-element section of the layered 3D cantilever (two 16^3 cells, "
                  f"{p.n_dof} DOFs); {t1 - t0:.1f} s, {res[0][1]} iterations")
    else:
        p = W.cantilever2d(512, 128, 32, 6)
        rho = W.design_field(p)
        fixed, f = W.fixed_mask(p), W.load_vector(p)
        t0 = time.perf_counter()
        rt, rb = density.filter_project(p, rho, p.rmin, p.beta, p.etas)
        res = schwarz.solve_pcg(p, list(rb), rb[0], f, fixed, rtol=args.rtol, maxit=args.maxit)
        dcs = np.stack([fem.sensitivity(p, rb[s], res[s][0]) for s in range(p.nsys)])
        [fem.compliance(f, r[0]) for r in res]
        density.filter_project_adjoint(p, rt, p.rmin, p.beta, p.etas, dcs)
        t1 = time.perf_counter()
        work = sum(p.n_dof * r[1] for r in res)
        sample = (f"one full step (filter+projection, spectral basis, 3-realisation PCG to "
                  f"{args.rtol:g}, sensitivities, chain rule) on a 512x128-element section of "
                  f"the cantilever workload (64 subdomains of 32x32, k=6; "
                  f"{p.n_dof} DOFs/system); {t1 - t0:.1f} s, iterations "
                  f"{[r[1] for r in res]}")
    return {"value": work / (t1 - t0), "unit": "DOF-iters/s", "cores": int(threads),
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "kind": "oracle", "sample": sample}


def section_errors(args):
    """Errors of the GPU's FP64 and mixed results (u, c, dc of the three
    realisations, PCG to the bench's rtol) against the oracle's sparse direct
    solves, on the 512 x 128 section of the cantilever workload."""
    import numpy as np
    import torch

    import paper_1411_3923_amd as T
    from oracle import density, fem
    from paper_1411_3923_amd import workloads as W

    p = W.cantilever2d(512, 128, 32, 6)
    rho = W.design_field(p)
    f = W.load_vector(p)
    _, rb = density.filter_project(p, rho, p.rmin, p.beta, p.etas)
    uo = [fem.solve(p, rb[s]) for s in range(p.nsys)]
    co = [fem.compliance(f, u) for u in uo]
    dco = [fem.sensitivity(p, rb[s], uo[s]) for s in range(p.nsys)]
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = {}
    for name, prec in (("fp64", T.FP64), ("mixed", T.MIXED)):
        pr = T.make_problem(2, p.nel[:2], p.sub, p.k, p.nsys, p.E0, p.Emin, p.penal, p.nu, prec)
        h = T.Handle(pr, W.fixed_mask(p))
        R, F = d(rb), d(np.stack([f] * p.nsys))
        h.build_coarse_basis(R, rep=0)
        u = torch.zeros((p.nsys, p.n_dof), dtype=torch.float64, device="cuda")
        h.pcg_solve(R, F, u, rtol=args.rtol, maxit=args.maxit)
        c = torch.zeros(p.nsys, dtype=torch.float64, device="cuda")
        dc = torch.zeros((p.nsys, p.n_el), dtype=torch.float64, device="cuda")
        h.compliance_and_sensitivity(R, u, F, c, dc)
        uh, ch, dch = u.cpu().numpy(), c.cpu().numpy(), dc.cpu().numpy()
        out[name] = {
            "u": [float(np.linalg.norm(uh[s] - uo[s]) / np.linalg.norm(uo[s])) for s in range(p.nsys)],
            "compliance": [abs(float(ch[s]) - co[s]) / abs(co[s]) for s in range(p.nsys)],
            "dc": [float(np.linalg.norm(dch[s] - dco[s]) / np.linalg.norm(dco[s]))
                   for s in range(p.nsys)],
            "against": "oracle sparse direct solve (SuperLU, two refinement steps), "
                       "512x128 section of the cantilever workload, 3 realisations, "
                       f"GPU PCG to {args.rtol:g}"}
        h.close()
    return out


def hbm_measured():
    """Achievable HBM bandwidth on this GPU, beside the 8 TB/s spec peak: a
    device-to-device copy of 2 GiB (read + write bytes) and a read-only sum
    over 4 GiB, each the median of 10 event-timed launches."""
    import torch
    out = {}
    n = (2 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    big = torch.ones(2 * n, dtype=torch.float64, device="cuda")

    def timed(fn, nbytes):
        fn()
        ms = []
        for _ in range(10):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return nbytes / (percentile(ms, 50) * 1e-3) / 1e9

    out["copy_GBs"] = timed(lambda: dst.copy_(src), 2 * 8 * n)
    out["read_GBs"] = timed(lambda: big.sum(), 8 * 2 * n)
    out["note"] = ("torch copy_ (read + write bytes) and sum (read bytes) on the current "
                   "stream; the roofline frac is against the 8 TB/s spec peak")
    del src, dst, big
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return None


def run_serving(args, precision):
    """The serving stream: requests with Poisson arrivals over a mix of 2D
    and 3D meshes, each a robust optimisation run of `updates` warm-started
    design updates with resident factors, admitted by device memory. Returns
    per-request latencies (arrival to the last update's result) and totals."""
    import collections

    import numpy as np
    import torch

    import paper_1411_3923_amd as T
    from paper_1411_3923_amd import workloads as W

    budget = int(args.serving_budget_gb * (1 << 30))
    srv = T.Server(budget, max_active=args.serving_slots)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    class Req:
        def __init__(self, t, p, i):
            self.t, self.p, self.i = t, p, i
            self.nsys = 3 if p.dim == 2 else 1
            self.step = 0
            self.job = None
            self.work = 0
            self.solves = []

        def start(self, sid):
            p = self.p
            self.sid = sid
            self.rho = W.design_field(p)
            self.F = d(np.stack([W.load_vector(p)] * self.nsys))
            self.u = torch.zeros((self.nsys, p.n_dof), dtype=torch.float64, device="cuda")
            self.c = torch.zeros(self.nsys, dtype=torch.float64, device="cuda")
            self.dc = torch.zeros((self.nsys, p.n_el), dtype=torch.float64, device="cuda")
            self.submit()

        def submit(self):
            p = self.p
            if self.step > 0:
                self.rho = np.clip(self.rho + 0.02 * W.design_noise(p, self.step, 100 + self.i), 0, 1)
            self.R = d(self.rho)
            kw = (dict(rmin=p.rmin, beta=p.beta, etas=p.etas) if p.dim == 2 else dict(rmin=0.0))
            self.job = srv.submit(self.sid, self.R, self.F, self.u, self.c, self.dc, rtol=args.rtol,
                                  maxit=args.maxit, rebuild=0, growth=1.5, **kw)

    def problem(p):
        return T.make_problem(p.dim, p.nel[:p.dim], p.sub, p.k, 3 if p.dim == 2 else 1, p.E0, p.Emin,
                              p.penal, p.nu, precision,
                              lambda_thresh=0.0 if p.dim == 2 else 1e-6)

    def drive(reqs):
        pending = collections.deque(sorted(reqs, key=lambda r: r.t))
        waiting, active, done = collections.deque(), {}, []
        t0 = time.perf_counter()
        while pending or waiting or active:
            now = time.perf_counter() - t0
            busy = False
            while pending and pending[0].t <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                sid = srv.open(problem(r.p), W.fixed_mask(r.p), r.nsys)
                if sid is None:
                    break
                waiting.popleft()
                r.admitted = time.perf_counter() - t0
                r.start(sid)
                active[sid] = r
                busy = True
            for sid, r in list(active.items()):
                res = srv.test(r.job)
                if res is None:
                    continue
                busy = True
                r.solves.append(res)
                r.work += r.p.n_dof * sum(res["iters"])
                r.step += 1
                print(f"serving: {r.p.name} update {r.step} iters {res['iters']} "
                      f"at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
                if r.step < args.serving_updates:
                    r.submit()
                else:
                    srv.close(sid)
                    r.finished = time.perf_counter() - t0
                    done.append(r)
                    del active[sid]
            if not busy:
                if pending and not waiting and not active:
                    time.sleep(max(0.0, pending[0].t - (time.perf_counter() - t0)))
                else:
                    time.sleep(0.0002)
        return done, time.perf_counter() - t0

    # single-stream capacity: one request of every mesh kind, one at a time
    kinds = [(0.0, p) for _, p in W.serving_requests(64, 1.0, seed=args.serving_seed,
                                                      with_3d=not args.serving_2d_only)]
    seen, calib = set(), []
    for _, p in kinds:
        key = (p.dim, p.nel)
        if key not in seen:
            seen.add(key)
            calib.append(Req(0.0, p, 900 + len(calib)))
    service = []
    for r in calib:
        done, wall = drive([r])
        service.append(wall)
    capacity = 1.0 / float(np.mean(service))
    rate = 0.8 * capacity
    reqs = [Req(t, p, i) for i, (t, p) in enumerate(
        W.serving_requests(args.serving_requests, rate, seed=args.serving_seed,
                           with_3d=not args.serving_2d_only))]
    done, wall = drive(reqs)
    srv.destroy()
    lat = [r.finished - r.t for r in done]
    solves = [s for r in done for s in r.solves]
    return {
        "requests": len(done), "updates_per_request": args.serving_updates,
        "arrival_rate_per_s": rate, "single_stream_capacity_per_s": capacity,
        "wall_s": wall, "requests_per_s": len(done) / wall,
        "dof_iters_per_s": sum(r.work for r in done) / wall,
        "latency_s_p50": percentile(lat, 50), "latency_s_p99": percentile(lat, 99),
        "queue_wait_s_mean": float(np.mean([r.admitted - r.t for r in done])),
        "job_solve_ms_p50": percentile([s["solve_ms"] for s in solves], 50),
        "job_solve_ms_p99": percentile([s["solve_ms"] for s in solves], 99),
        "basis_rebuilds_per_job": sum(s["rebuilt"] for s in solves) / len(solves),
        "iters_mean": float(np.mean([max(s["iters"]) for s in solves])),
        "failed_jobs": sum(1 for s in solves if s["status_all"] != 0 or max(s["status"]) != 0),
        "meshes": sorted({r.p.name.split("_", 1)[1] for r in done}),
        "budget_gb": args.serving_budget_gb, "slots": args.serving_slots,
    }


def short_name(name):
    """Kernel name without namespace, template arguments or parameter list."""
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    base = base.split("<")[0]
    return base.split("::")[-1].replace("void ", "")


def summarize_trace(stats_csv, command, out, title, bench_json=None):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel summary."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel trace: {title}", "", "Command (on one MI355X, from the repository root):",
             "", "    " + command, "",
             "| kernel | calls | total ms | avg us | min us | max us |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    if bench_json:
        b = json.loads([ln for ln in open(bench_json).read().splitlines()
                        if ln.startswith("{")][-1])
        rl = b["roofline"]
        lines += ["", f"The bench line of the same run timed {rl['kernel']} with HIP events on its "
                  f"stream: {rl['launches']} launches with work, {rl['avg_launch_ms'] * 1e3:.1f} us "
                  f"per launch, {rl['algorithmic_bytes_per_launch'] / 1e9:.3f} GB algorithmic "
                  f"bytes per launch, {rl['achieved']:.0f} GB/s. The trace average above also "
                  f"counts the near-empty launches after the systems converge."]
        trace_csv = os.path.join(os.path.dirname(stats_csv), "run_kernel_trace.csv")
        if os.path.exists(trace_csv):
            base = rl["kernel"].split("<")[0]
            if "{" in base:   # a set of kernels launched once each per iteration
                stem, alts = base.split("{")
                keys = [stem + a for a in alts.rstrip("}").split(",")]
            else:
                keys = [base]
            trace = list(csv.DictReader(open(trace_csv)))
            total = 0.0
            for key in keys:
                d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                     for r in trace
                     if r["Kernel_Name"].split("<")[0].split("(")[0].strip() == key]
                busy = [x for x in d if x > 20.0][-rl["launches"]:]
                avg = sum(busy) / len(busy) if busy else 0.0
                total += avg
                lines += ["", f"In the trace, the last {len(busy)} launches of {key} that do "
                          f"work (the timed steps) average {avg:.1f} us."]
            if len(keys) > 1:
                lines += ["", f"Together: {total:.1f} us per iteration."]
    open(out, "w").write("\n".join(lines) + "\n")


def summarize_traffic(fetch_csv, write_csv, command, out_json, out_md, kernel="k_local_solves<double>",
                      workload="cantilever2d"):
    """HBM bytes per launch of the roofline kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch). Each counter is scaled by
    what it reads for the first device-to-device copy of the run, a copy of
    COPY_BYTES bytes in each direction. A kernel name with {a,b,c} counts the
    three kernels of one local solve together (their i-th dispatches summed)."""
    import csv

    if "{" in kernel:
        head, rest = kernel.split("{", 1)
        alts, tail = rest.split("}", 1)
        keys = [head + a + tail.rstrip(">") for a in alts.split(",")]
    else:
        keys = [kernel.rstrip(">")]   # template arguments beyond the element type vary

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        copy = next(r for r in rows if "copyBuffer" in r["Kernel_Name"])
        kib_copy = float(copy["Counter_Value"])
        assert kib_copy * 1024 > COPY_BYTES / 4, "calibration copy not found"
        per = [[float(r["Counter_Value"]) for r in rows if k in r["Kernel_Name"]] for k in keys]
        n = min(len(v) for v in per)
        vals = [sum(v[i] for v in per) for i in range(n)]
        return COPY_BYTES / (kib_copy * 1024), vals

    ff, fv = load(fetch_csv, "FETCH_SIZE")
    wf, wv = load(write_csv, "WRITE_SIZE")
    # launches with work, as the bench counts them: once every system has
    # converged a launch only reads the gate flags
    busy = [i for i, v in enumerate(fv) if v * 1024 * ff > 1e6]
    fv = [fv[i] for i in busy]
    wv = [wv[i] for i in busy if i < len(wv)]
    fetch = sum(fv) / len(fv) * 1024 * ff
    write = sum(wv) / len(wv) * 1024 * wf
    res = {"kernel": kernel, "kernel_hash": kernel_hash(workload),
           "kernel_sources": KERNEL_SOURCES[workload],
           "bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
           "write_bytes_per_launch": write, "fetch_scale": ff, "write_scale": wf,
           "launches": len(fv), "command": command}
    json.dump(res, open(out_json, "w"), indent=1)
    title = ("192x96x96 layered 3D cantilever, FP64" if workload == "cantilever3d"
             else "1024x512 cantilever, 3 realisations, FP64")
    lines = [f"# HBM traffic of {kernel}: {title}", "",
             "Commands (on one MI355X, from the repository root):", ""]
    lines += ["    " + c for c in command.split(" ;; ")]
    lines += ["", f"The first copy in each run moves {COPY_BYTES} bytes. FETCH_SIZE reads it as "
              f"{COPY_BYTES / ff / 1024:.0f} KiB (scale {ff:.3f}), WRITE_SIZE as "
              f"{COPY_BYTES / wf / 1024:.0f} KiB (scale {wf:.3f}).", "",
              "| per launch (mean over the run's launches) | bytes |", "|---|---:|",
              f"| scaled FETCH_SIZE | {fetch:.4g} |", f"| scaled WRITE_SIZE | {write:.4g} |",
              f"| traffic | {fetch + write:.4g} |", "",
              f"{len(fv)} launches with work. Kernel sources hash {res['kernel_hash']}."]
    open(out_md, "w").write("\n".join(lines) + "\n")


def loop_bytes(nsys=3, nelx=1024, nely=512, sub=32, k=6):
    """Algorithmic HBM bytes per launch of the PCG-loop kernels, FP64, 2-d Q4,
    every system running: each array the kernel must touch, read or written
    once (the stored moduli, flags and coarse basis included)."""
    nnodes = (nelx + 1) * (nely + 1)
    ndof, nel = 2 * nnodes, nelx * nely
    nsub = (nelx // sub) * (nely // sub)
    nloc = 2 * (sub + 1) ** 2
    nt = nsub * k
    ct = (nt + 63) // 64                      # tile rows of the packed K_c^-1
    v = 8 * nsys * ndof                      # one FP64 vector of every system
    zl = 8 * nsys * nsub * nloc              # local solutions
    phi = 8 * nsub * k * nloc                # coarse basis, shared by the systems
    return {
        "k_apply_q4": 4 * v + 8 * nsys * nel + ndof,          # z, p read; p', K p' written; moduli, flags
        "k_update_xr": 6 * v,                                  # u, p, r, q read; u, r written
        "k_extend": zl + phi + 2 * v + ndof,                   # zloc, Phi, r read; z written
        "k_restrict": phi + zl,                                # Phi and the boxes of r
        # lower 64 x 64 tiles of K_c^-1 read, tile partials written; the
        # partials summed
        "k_coarse_gemv_tiles": 8 * nsys * (ct * (ct + 1) // 2 * 64 * 64 + ct * ct * 64),
        "k_coarse_gemv_sum": 8 * nsys * (ct * ct * 64 + nt),
    }


def summarize_mfma(csv_path, command, out, title):
    """Matrix-core and vector FP64 work of the dense setup kernels from one
    rocprofv3 --pmc run (SQ_INSTS_VALU_MFMA_MOPS_F64: units of 512 flops;
    SQ_INSTS_VALU_FLOPS_FP64; SQ_VALU_MFMA_BUSY_CYCLES against GRBM_GUI_ACTIVE
    over the chip's 1024 SIMDs), durations from the same run's timestamps."""
    import csv
    per = {}
    for r in csv.DictReader(open(csv_path)):
        k = short_name(r["Kernel_Name"])
        d = per.setdefault(k, {})
        e = d.setdefault(int(r["Dispatch_Id"]), {"us": (int(r["End_Timestamp"]) -
                                                         int(r["Start_Timestamp"])) / 1e3})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    rows = []
    for k, d in per.items():
        ds = list(d.values())
        n = len(ds)
        us = sum(x["us"] for x in ds) / n
        mf = sum(x.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for x in ds) * 512 / n
        vf = sum(x.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) for x in ds) / n
        busy = sum(x.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for x in ds)
        act = sum(x.get("GRBM_GUI_ACTIVE", 0.0) for x in ds)
        # GRBM_GUI_ACTIVE comes summed over the 8 XCDs, each counting the
        # same active cycles: one XCD's count is the kernel's active time
        util = 100.0 * busy / (act / 8 * 1024) if act > 0 else 0.0
        if us * n < 200 and mf == 0:
            continue
        rows.append((us * n, k, n, us, mf, vf, util))
    rows.sort(reverse=True)
    lines = [f"# FP64 matrix-core use of the setup kernels: {title}", "",
             "Command (on one MI355X, from the repository root):", "", "    " + command, "",
             "Per dispatch (mean over the run's dispatches of the kernel). MFMA flops = "
             "SQ_INSTS_VALU_MFMA_MOPS_F64 x 512; achieved = MFMA flops / duration, against "
             "the 78.6 TFLOP/s FP64 matrix-core peak; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / "
             "(active cycles x 1024 SIMDs), active cycles = GRBM_GUI_ACTIVE / 8 (the counter "
             "comes summed over the 8 XCDs). The VALU column is SQ_INSTS_VALU_FLOPS_FP64 as "
             "the counter reports it. Durations come from the counter run (kernels "
             "serialised).", "",
             "| kernel | dispatches | avg us | MFMA GFLOP | MFMA TFLOP/s | % of 78.6 "
             "| MFMA busy % | VALU FP64 counter (G) |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for _, k, n, us, mf, vf, util in rows:
        tf = mf / (us * 1e-6) / 1e12 if us > 0 else 0.0
        lines.append(f"| {k} | {n} | {us:.1f} | {mf / 1e9:.3f} | {tf:.2f} | "
                     f"{100 * tf / 78.6:.1f} | {util:.1f} | {vf / 1e9:.3f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def summarize_loop(fetch_csv, write_csv, trace_csv, command, out):
    """Per-kernel HBM traffic and bandwidth of the PCG loop over the launches
    in which all three systems run: bytes from two rocprofv3 --pmc runs of one
    solve (scaled by the calibration copy), durations from a kernel trace of
    the same workload."""
    import csv

    def counters(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        copy = next(r for r in rows if "copyBuffer" in r["Kernel_Name"])
        scale = COPY_BYTES / (float(copy["Counter_Value"]) * 1024)
        per = {}
        for r in rows:
            per.setdefault(short_name(r["Kernel_Name"]), []).append(
                float(r["Counter_Value"]) * 1024 * scale)
        return per

    fetch, write = counters(fetch_csv, "FETCH_SIZE"), counters(write_csv, "WRITE_SIZE")
    dur = {}
    for r in sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"])):
        dur.setdefault(short_name(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    alg = loop_bytes()
    lines = ["# PCG-loop kernels: 1024x512 cantilever, 3 realisations, FP64", "",
             "Commands (on one MI355X, from the repository root):", ""]
    lines += ["    " + c for c in command.split(" ;; ")]
    lines += ["", "Launches in which all three systems run (the first iterations of each solve; "
              "the later ones carry one or two systems). Measured bytes: FETCH_SIZE + WRITE_SIZE, "
              "each scaled by what it reads for a copy of known size. Bandwidth against the "
              "8 TB/s HBM3E peak.", "",
              "| kernel | launches | avg us | measured MB | measured GB/s | % peak "
              "| algorithmic MB | algorithmic GB/s |",
              "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for name in ["k_apply_q4", "k_update_xr", "k_restrict", "k_local_solves",
                 "k_coarse_gemv_tiles", "k_coarse_gemv_sum", "k_extend"]:
        fv, wv, dv = fetch.get(name, []), write.get(name, []), dur.get(name, [])
        if not fv or not dv:
            continue
        tot = [a + b for a, b in zip(fv, wv)]
        top = max(tot)
        idx = [i for i, x in enumerate(tot) if x > 0.8 * top]   # all three systems running
        per_solve = len(tot)
        nsolve = len(dv) // per_solve
        ds = [dv[s * per_solve + i] for s in range(nsolve) for i in idx]
        mb = sum(tot[i] for i in idx) / len(idx)
        us = sum(ds) / len(ds)
        a = alg.get(name)
        if name == "k_local_solves":
            a = None
        lines.append(f"| {name} | {len(idx)} | {us:.1f} | {mb / 1e6:.1f} | {mb / us / 1e3:.0f} | "
                     f"{mb / us / 1e3 / 80:.0f} | " +
                     (f"{a / 1e6:.1f} | {a / us / 1e3:.0f} |" if a else "- | - |"))
    lines += ["", "The local solves' algorithmic bytes are in the bench line's roofline."]
    open(out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["cantilever2d", "cantilever3d", "serving"],
                    default="cantilever2d")
    ap.add_argument("--serving-requests", type=int, default=16)
    ap.add_argument("--serving-updates", type=int, default=10)
    ap.add_argument("--serving-budget-gb", type=float, default=160.0)
    ap.add_argument("--serving-slots", type=int, default=6)
    ap.add_argument("--serving-seed", type=int, default=1005)
    ap.add_argument("--serving-2d-only", action="store_true")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 10; 3 in 3D)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 2; 1 in 3D)")
    ap.add_argument("--ncoarse", type=int, default=0,
                    help="coarse vectors per subdomain, the cap under a threshold (0: 6 in 2D, 16 in 3D)")
    ap.add_argument("--lambda-thresh", type=float, default=None,
                    help="eigenvalue threshold of the coarse space (default 0 in 2D, 1e-6 in 3D)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--gmres-restart", type=int, default=50,
                    help="cycle length of the paper's GMRES solve reported beside the steps")
    ap.add_argument("--gmres-reps", type=int, default=None,
                    help="timed GMRES solves per preconditioner (0: none; default 3 in 2-d, 0 in 3-d)")
    ap.add_argument("--eig-iters", type=int, default=0, help="subspace iterations (0: library default)")
    ap.add_argument("--eig-extra", type=int, default=0, help="guard vectors (0: library default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device, the reference kernel for HBM counters")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="write a profile summary of a rocprofv3 --stats run and exit (no GPU)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic of the roofline kernel from two --pmc runs and exit")
    ap.add_argument("--summarize-loop", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "TRACE_CSV"),
                    help="write the per-kernel PCG-loop traffic table and exit")
    ap.add_argument("--summarize-mfma", metavar="COUNTER_CSV",
                    help="write the matrix-core table of a rocprofv3 --pmc run and exit")
    ap.add_argument("--command", default="", help="command recorded in a summary")
    ap.add_argument("--title", default="1024x512 cantilever, 3 realisations, FP64")
    ap.add_argument("--bench-json", default=None, help="bench line of the traced run")
    ap.add_argument("--out", default=None, help="summary file")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.command, args.out, args.title, args.bench_json)
        return
    if args.summarize_mfma:
        summarize_mfma(args.summarize_mfma, args.command, args.out, args.title)
        return
    if args.summarize_loop:
        summarize_loop(*args.summarize_loop, args.command, args.out)
        return
    three = args.workload == "cantilever3d"
    if args.steps is None:
        args.steps = 3 if three else 50
    if args.gmres_reps is None:
        args.gmres_reps = 0 if three else 3
    if args.warmup is None:
        args.warmup = 1 if three else 2
    if args.ncoarse <= 0:
        args.ncoarse = 16 if three else 6
    if args.lambda_thresh is None:
        args.lambda_thresh = 1e-6 if three else 0.0
    if args.summarize_traffic:
        tf = TRAFFIC_FILES[args.workload]
        summarize_traffic(*args.summarize_traffic, args.command, tf, tf.replace(".json", ".md"),
                          kernel=ROOFLINE_KERNEL[args.workload], workload=args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solve of one "
              "system does not span GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1411_3923_amd as T
    from paper_1411_3923_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    T.load_library()
    if args.workload == "serving":
        mixed = run_serving(args, T.MIXED)
        fp64 = None if args.no_mixed else run_serving(args, T.FP64)
        line = {
            "metric": "PCG solve time & DOF-iters/s to rel-res 1e-8 (FP64 vs mixed); p50/p99 latency",
            "value": mixed["dof_iters_per_s"], "unit": "DOF-iters/s", "n_gpus": 1,
            "steps": mixed["requests"], "warmup": 0,
            "ms_per_step": 1e3 * mixed["wall_s"] / max(mixed["requests"], 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 outer CG, f32 local solves and coarse-basis products", "data": "synthetic",
            "config": {"workload": "serving_stream_q4_h8_mixed",
                       "step": f"one request: admission, {args.serving_updates} warm-started robust "
                               "design updates (density pipeline, basis rule, batched PCG, "
                               "sensitivities)",
                       "rtol": args.rtol},
            "serving_mixed": mixed, "serving_fp64": fp64,
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(line), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if three:
        p = W.cantilever3d(192, 96, 96, 16, args.ncoarse)
    else:
        p = W.cantilever2d(1024, 512, 32, args.ncoarse)
    rho_h = W.design_field(p)
    f_h = W.load_vector(p)

    r64 = run_gpu(T.FP64, args, p, rho_h, f_h)
    rmx = None if args.no_mixed else run_gpu(T.MIXED, args, p, rho_h, f_h)

    prof = r64["block_solves"]
    achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else None
    traffic = None
    tf = TRAFFIC_FILES[args.workload]
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("kernel_hash") == kernel_hash(args.workload):
            traffic = t.get("bytes_per_launch")

    def summary(r):
        return {k: r[k] for k in ("ms_per_step", "dof_iters_per_s", "solve_only_dof_iters_per_s",
                                  "solve_ms_p50", "solve_ms_p99", "setup_ms_p50", "iters",
                                  "relres", "true_relres", "status", "compliance",
                                  "eig_max_ritz_residual", "coarse_vectors_per_subdomain",
                                  "paper_solver")}

    line = {
        "metric": "PCG solve time & DOF-iters/s to rel-res 1e-8 (FP64 vs mixed); p50/p99 latency",
        "value": r64["dof_iters_per_s"],
        "unit": "DOF-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": ({"workload": "cantilever3d_h8_192x96x96_layered", "elements": p.n_el,
                    "dofs_per_system": p.n_dof, "systems": p.nsys, "subdomain": p.sub,
                    "coarse_vectors_cap": p.k, "lambda_thresh": args.lambda_thresh,
                    "rtol": args.rtol,
                    "step": "basis+factor build, PCG, compliance+sensitivities"} if three else
                   {"workload": "cantilever2d_q4_1024x512_3realisations", "elements": p.n_el,
                    "dofs_per_system": p.n_dof, "systems": p.nsys, "subdomain": p.sub,
                    "coarse_vectors": p.k, "rtol": args.rtol,
                    "step": "filter+projection, basis+factor build, batched PCG, "
                            "compliance+sensitivities, chain rule"}),
        "fp64": summary(r64),
        "roofline": {"bound": "hbm", "kernel": ROOFLINE_KERNEL[args.workload],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic,
                     "launches": prof["launches"],
                     "avg_launch_ms": prof["ms"] / max(prof["launches"], 1),
                     "algorithmic_bytes_per_launch": prof["bytes"] / max(prof["launches"], 1)},
    }
    if rmx is not None:
        line["mixed"] = summary(rmx)
        line["mixed"]["dtype"] = "f64 outer CG, f32 local solves and coarse-basis products"
        u64, umx = r64["u"], rmx["u"]
        line["mixed"]["rel_diff_vs_fp64"] = {
            "u": [float(np.linalg.norm(umx[s] - u64[s]) / np.linalg.norm(u64[s]))
                  for s in range(p.nsys)],
            "compliance": [abs(a - b) / abs(b) for a, b in zip(rmx["compliance"], r64["compliance"])],
            "dc": [float(np.linalg.norm(rmx["dc"][s] - r64["dc"][s]) / np.linalg.norm(r64["dc"][s]))
                   for s in range(p.nsys)],
        }
        bmx = rmx["block_solves"]
        line["mixed"]["block_solves_GBs"] = (bmx["bytes"] / (bmx["ms"] * 1e-3) / 1e9
                                            if bmx["ms"] > 0 else None)
    line["roofline"]["hbm_measured"] = hbm_measured()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args)
        if not three:
            errs = section_errors(args)
            line["fp64"]["error_vs_oracle_section"] = errs["fp64"]
            if "mixed" in line:
                line["mixed"]["error_vs_oracle_section"] = errs["mixed"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

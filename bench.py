"""Benchmark of the IBDL hot path on one MI355X.

A step is one complete IBDL solve of a batch of right-hand sides (32 by
default: enough column tiles to give every compute unit eight blocks) on the 2-D
star workload (periodic unit square, 1024^2 grid, star r = 0.3 + 0.05 cos 5t
with 4096 boundary points, alpha = 1, Dirichlet, random-Fourier manufactured
data): the right-hand side, unpreconditioned GMRES on the device to tol 1e-8,
and the grid solution.  The geometry's plan (binning, sort, spread matrices) is
built once before timing.  Inputs are resident on the GPU.

value = operator applications per second over the timed steps (every GMRES
iteration of every right-hand side counts one application; the time includes
the right-hand side, the Krylov arithmetic and the grid solution).  The line
also reports solves/s, per-step latency percentiles, the FP64 path, the error
of both against the FP64 oracle, the roofline of the dominant kernel (timed with
HIP events on the library's stream) and the oracle's own throughput on the
host.

With --workload serve the line reports the served stream instead: 2000
requests (80% 2-D, 20% 3-D, sizes 256^2..2048^2 and 64^3..256^3, alpha
log-uniform in [1, 1000], mixed precision, grid solution included) cycling
through a set of materialised request templates; first the saturation
throughput with a bounded number of requests outstanding, then seeded Poisson
arrivals at 0.5x and 0.8x of it, with p50/p99 of submission-to-result latency.

With --workload batch512 a step is one batched solve of the 512-instance
ellipse batch (grid sizes 128..512, 2..8 right-hand sides each, Dirichlet and
Neumann, alpha log-uniform in [1, 1000], mixed precision) followed by the grid
solutions of every instance; the roofline is that of one batched operator
application over all instances.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs R]
                       [--workload star1024|sphere256|batch512|serve]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IBDL operator applies/s + batched solves/s at 1e-6 rel err; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def stage_bytes(st, dim, n, m, prec, nrhs):
    """Algorithmic bytes per call of each grid stage for this geometry: every
    necessary read and write counted once (see the design notes)."""
    bc = 16 if prec == 0 else 8      # complex
    br = 8 if prec == 0 else 4       # real
    W = n // 2 + 1
    S, G = st["n_spread_lines"], st["n_gather_lines"]
    gpp = 4 if dim == 2 else 16
    csr = st["dip_nnz"] * (4 + br) + st["dip_active_nodes"] * 8 + (st["nlines"] + 1) * 4 + S * 4
    pts = m * (12 + 12 * br + 4)
    out = {}
    out["spread+fft_x"] = nrhs * (S * W * bc + m * 8) + csr
    if dim == 2:
        out["fft_y+symbol"] = nrhs * (S + G) * W * bc
    else:
        Ps, Pg = st["n_spread_planes"], st["n_gather_planes"]
        out["fft_y"] = nrhs * (S + Ps * n) * W * bc
        out["fft_z+symbol"] = nrhs * (Ps + Pg) * n * W * bc
        out["ifft_y"] = nrhs * (Pg * n + G) * W * bc
    out["ifft_x+interp"] = nrhs * (G * W * bc + m * gpp * br) + pts
    out["finish"] = nrhs * (m * gpp * br + m * 16) + m * 4
    return out


def stage_flops(dim, n, nrhs):
    """Algorithmic floating-point operations per call of the 2-D column stage
    (every column k_x = 0..n/2 of every right-hand side: forward and inverse
    length-n complex FFT at the conventional 5 n log2 n each, and the real
    symbol scaling, 2 per element).  The row stages' FFTs run only over the
    lines that carry forcing or are read, and are not counted here."""
    if dim != 2:
        return {}
    W = n // 2 + 1
    return {"fft_y+symbol": nrhs * W * (10 * n * math.log2(n) + 2 * n)}


# FP32 vector peak of MI355X (256 CUs x 2.4 GHz x 128 lanes x 2 per FMA)
ALU_PEAK_TFLOPS = 157.3
ROOF_APPLIES = 50
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "star1024_nrhs32_traffic.md")
KERNEL_SOURCES = ["paper_2203_12126_amd/csrc/pipeline.h", "paper_2203_12126_amd/csrc/fft.h",
                  "paper_2203_12126_amd/csrc/common.h"]


def stage_kernel(stage, dim, n):
    """Kernel (FP32 instantiation) behind a stage name of a mixed 2-D apply."""
    if dim != 2:
        return stage
    return {"spread+fft_x": f"k_row_fwd<float, {n}, false>",
            "fft_y+symbol": f"k_col<float, {n}, 1, 1, false>",
            "ifft_x+interp": f"k_row_inv<float, {n}, 0, false>",
            "finish": "k_finish<float, false>"}.get(stage, stage)


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(workload, nrhs, kernel):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the summary
    is for another configuration or the kernel sources changed since."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if not ln.startswith("traffic:"):
            continue
        kv = dict(x.strip().split("=", 1) for x in ln[len("traffic:"):].split(";") if "=" in x)
        if (kv.get("workload") == workload and int(kv.get("nrhs", -1)) == nrhs and kv.get("kernel") == kernel
                and kv.get("sources_sha1") == kernel_sources_sha1()):
            return int(kv["bytes_per_launch"])
    return None


def full_grid_bytes_per_apply(dim, n, m, prec):
    """(4d-4) H + M (16 + 2 d b): the full-grid byte count of one apply."""
    b = 8 if prec == 0 else 4
    H = n ** (dim - 1) * (n // 2 + 1) * 2 * b
    return (4 * dim - 4) * H + m * (16 + 2 * dim * b)


def make_workload(name, nrhs):
    from paper_2203_12126_amd import workloads as W
    if name == "star1024":
        probs = [W.config_star1024(m=4096, alpha=1.0, bc=W.DIRICHLET, seed=2203 + r) for r in range(nrhs)]
        desc = ("2-D Dirichlet screened Poisson, periodic unit square, 1024^2 grid, star "
                "r=0.3+0.05cos(5t) with 4096 points, alpha=1, random-Fourier manufactured data")
        tol = 1e-8
    elif name == "sphere256":
        probs = [W.config_sphere256()]
        for r in range(1, nrhs):
            probs.append(W.config_sphere256())
        desc = ("3-D Dirichlet, periodic unit cube, 256^3 grid, sphere R=0.3 with 40000 Fibonacci "
                "points, alpha=10, u=exp(x+y)cos(sqrt2 z-0.3)")
        tol = 1e-8
    else:
        raise SystemExit(f"unknown workload {name}")
    return probs, desc, tol


def batch_stage_bytes(stats, metas):
    """Algorithmic bytes of one batched mixed apply, per stage, summed over instances."""
    tot = {}
    for st, mt in zip(stats, metas):
        for k, v in stage_bytes(st, mt["dim"], mt["n"], mt["m"], 1, mt["nrhs"]).items():
            tot[k] = tot.get(k, 0) + v
    return tot


def run_batch(args):
    import torch
    from paper_2203_12126_amd import ibdl
    from paper_2203_12126_amd import workloads as W

    t0 = time.perf_counter()
    specs = W.config_batch()
    items, data, g = [], [], []
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    for sp in specs:
        _, _, probs = W.batch_instance(sp)
        items.append((probs[0], len(probs)))
        data.append(t(np.stack([p.data for p in probs])))
        g.append(t(np.stack([p.g_tilde for p in probs])))
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = ibdl.Batch.from_problems(items, prec=ibdl.MIXED)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    R = batch.total_rhs
    tol = 1e-8

    # outputs allocated once, outside the timed steps
    sol_out, u_out = batch.empty(), batch.empty(grid=True)
    for _ in range(args.warmup):
        sol, u, info = batch.solve_grid(data, g, tol=tol, out=sol_out, u=u_out)
    torch.cuda.synchronize()
    lat, iters = [], 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        sol, u, info = batch.solve_grid(data, g, tol=tol, out=sol_out, u=u_out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        iters += int(info.field("iters").sum())
    el = time.perf_counter() - t0
    statuses = sorted({i["status"] for i in info})

    # roofline: one batched mixed operator application over every instance
    rng = np.random.default_rng(0)
    q = [t(rng.standard_normal(d.shape)) for d in data]
    out = batch.apply(q)
    torch.cuda.synchronize()
    batch.set_timing(True)
    napp = 20
    for _ in range(napp):
        batch.apply(q, out=out)
    stages = batch.stage_times()
    batch.set_timing(False)
    stats = [batch.stats(i) for i in range(batch.count)]
    sb = batch_stage_bytes(stats, batch.meta)
    per_apply = {nm: ms * calls / napp for nm, ms, calls in stages}
    dom = max(per_apply, key=per_apply.get)
    achieved = sb.get(dom, 0) / (per_apply[dom] * 1e-3) / 1e9
    apply_ms = sum(per_apply.values())
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": int(sb.get(dom, 0)), "ms_per_launch": round(per_apply[dom], 5),
            "note": "stage summed over the (grid size) groups of one batched apply"}

    # accuracy of a few instances against the FP64 oracle (outside the timed region)
    from oracle import ibdl_oracle as O
    errs = []
    cpu = None
    small = [i for i, sp in enumerate(specs) if sp["n"] == 128][:3]
    t_cpu, cpu_iters = 0.0, 0
    for i in small:
        p = items[i][0]
        st = O.setup_from_problem(p)
        c0 = time.perf_counter()
        res, _ = O.solve(st, p.data, p.g_tilde, bc=p.bc, tol=tol)
        t_cpu += time.perf_counter() - c0
        cpu_iters += res.iters
        ref, _ = O.solve(st, p.data, p.g_tilde, bc=p.bc, tol=1e-13)
        x = sol[i][0].cpu().numpy()
        errs.append(float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)))
    if not args.no_cpu:
        cpu = {"value": round(cpu_iters / t_cpu, 3), "unit": "applies/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle solves of {len(small)} n=128 instances of the batch "
                         f"({cpu_iters} applies) = {t_cpu:.1f} s"}
    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": METRIC, "value": round(iters / el, 2), "unit": "applies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 grid + f64 krylov", "data": "synthetic",
        "config": {"workload": "batch512", "description": "512 2-D ellipse instances, n in {128,192,256,384,512}, "
                   "2..8 rhs, Dirichlet/Neumann, alpha log-uniform [1,1000], tol 1e-8, mixed",
                   "instances": batch.count, "total_rhs": R, "tol": tol, "precision": "mixed",
                   "graphs": args.graphs == "on"},
        "solves_per_s": round(args.steps * R / el, 2),
        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "iters_per_solve": round(iters / (args.steps * R), 2),
        "statuses": statuses,
        "batched_apply_ms": round(apply_ms, 4),
        "stages_ms_per_apply": {k: round(v, 5) for k, v in per_apply.items()},
        "rel_err_vs_oracle_sampled": errs,
        "setup_s": {"inputs": round(t_gen, 2), "plans": round(t_plan, 2)},
        "autotune": ibdl.autotune_report().splitlines(),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    batch.close()
    print(json.dumps(line), flush=True)


def run_serve(args):
    import torch
    from paper_2203_12126_amd import ibdl
    from paper_2203_12126_amd import workloads as W

    count = args.serve_requests
    specs = W.config_serve(count=count)
    ntpl = min(args.serve_templates, count)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    tpl = []
    for sp in specs[:ntpl]:
        p = W.serve_instance(sp)
        g = p.grid
        tpl.append(dict(dim=g.dim, n=g.n, lo=tuple(g.lo), length=g.length, alpha=p.alpha, bc=p.bc,
                        X=t(p.geom.X), normal=t(p.geom.normal), weight=t(p.geom.weight),
                        data=t(p.data).reshape(1, -1), g=t(p.g_tilde).reshape(1, -1), m=p.geom.m))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    srv = ibdl.Server(max_slots=64, streams=4)

    def submit(i):
        q = tpl[i % ntpl]
        return srv.submit(q["dim"], q["n"], q["lo"], q["length"], q["alpha"], q["X"], q["normal"], q["weight"],
                          q["data"], q["g"], bc=q["bc"], prec=ibdl.MIXED, tol=1e-8, grid=True)

    # warm-up: every template once
    for tk in [submit(i) for i in range(ntpl)]:
        srv.wait(tk)

    def closed_loop(n, window):
        out, live, i = [], [], 0
        c0 = time.perf_counter()
        while i < n or live:
            while i < n and len(live) < window:
                live.append(submit(i))
                i += 1
            keep = []
            for tk in live:
                r = srv.poll(tk)
                if r is None:
                    keep.append(tk)
                else:
                    out.append(r)
            live = keep
            if live:
                time.sleep(0.0002)
        return out, time.perf_counter() - c0

    def open_loop(n, qps, cap=512):
        out, live = [], []
        arr = np.array([s["arrival"] for s in specs[:n]]) / qps
        c0 = time.perf_counter()
        i = 0
        while i < n or live:
            now = time.perf_counter() - c0
            while i < n and arr[i] <= now and len(live) < cap:
                live.append(submit(i))
                i += 1
            keep = []
            for tk in live:
                r = srv.poll(tk)
                if r is None:
                    keep.append(tk)
                else:
                    out.append(r)
            live = keep
            time.sleep(0.0002)
        return out, time.perf_counter() - c0

    sat_res, sat_el = closed_loop(count, args.serve_window)
    sat = count / sat_el
    runs = {}
    for f in (0.5, 0.8):
        res, el = open_loop(count, f * sat)
        lat = np.array([r["times"]["total_ms"] for r in res])
        runs[f"{f}x"] = {"qps": round(f * sat, 2), "solves_per_s": round(len(res) / el, 2),
                         "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                         "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                         "queue_ms_p50": round(float(np.percentile([r["times"]["queue_ms"] for r in res], 50)), 3),
                         "mean_cohort": round(float(np.mean([r["times"]["cohort_size"] for r in res])), 2),
                         "bad_status": int(sum(r["status"] != 0 for r in res))}
    st = srv.stats()
    srv.close()
    lat = np.array([r["times"]["total_ms"] for r in sat_res])
    iters = sum(r["info"][0]["iters"] for r in sat_res)
    line = {
        "metric": METRIC, "value": round(sat, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": count, "warmup": ntpl, "ms_per_step": round(sat_el / count * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 grid + f64 krylov", "data": "synthetic",
        "config": {"workload": "serve", "requests": count, "templates": ntpl, "window": args.serve_window,
                   "description": "served stream: 80% 2-D (256^2..2048^2, circle/star, 1k..16k points, D/N), "
                                  "20% 3-D (64^3..256^3, sphere/ellipsoid, 5k..40k points), alpha logU[1,1000], "
                                  "tol 1e-8, grid solution included", "precision": "mixed",
                   "graphs": args.graphs == "on"},
        "saturation": {"solves_per_s": round(sat, 2), "applies_per_s": round(iters / sat_el, 1),
                       "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                       "latency_ms_p99": round(float(np.percentile(lat, 99)), 3)},
        "open_loop": runs,
        "server": {"peak_active": st["peak_active"], "cohorts": st["cohorts"],
                   "peak_in_use_GB": round(st["peak_in_use_bytes"] / 1e9, 3),
                   "budget_GB": round(st["budget_bytes"] / 1e9, 1)},
        "setup_s": round(t_gen, 2),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--workload", default="star1024")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="length of the oracle CPU sample")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-templates", type=int, default=48)
    ap.add_argument("--serve-window", type=int, default=64)
    ap.add_argument("--graphs", choices=["on", "off"], default="off",
                    help="replay Arnoldi steps from recorded HIP graphs (on) or launch each kernel (off)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each solve fits one MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_12126_amd import ibdl

    torch.cuda.set_device(0)
    ibdl.set_graphs(args.graphs == "on")
    if args.workload == "batch512":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    probs, desc, tol = make_workload(args.workload, args.nrhs)
    p0 = probs[0]
    dim, n, m = p0.grid.dim, p0.grid.n, p0.geom.m
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    data = t(np.stack([p.data for p in probs]))
    g = t(np.stack([p.g_tilde for p in probs]))

    def run(prec, steps, warmup, timing):
        """Timed steps with stage timing off; then, if asked, a few more steps with
        the per-stage events on (their times feed the roofline)."""
        plan = ibdl.Plan.from_problem(p0, prec=prec)
        # outputs allocated once, outside the timed steps
        sol_out = torch.empty_like(data)
        u_out = torch.empty((data.shape[0],) + (n,) * dim, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            sol, u, info = plan.solve_grid(data, g, tol=tol, out=sol_out, u=u_out)
        torch.cuda.synchronize()
        lat, iters = [], 0
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            sol, u, info = plan.solve_grid(data, g, tol=tol, out=sol_out, u=u_out)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
            iters += int(info.field("iters").sum())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stages = []
        if timing:
            plan.set_timing(True)
            for _ in range(max(3, steps // 4)):
                plan.solve(data, g, tol=tol)
            stages = plan.stage_times()
            plan.set_timing(False)
        stats = plan.stats()
        out = dict(elapsed=el, lat=lat, iters=iters, sol=sol.cpu().numpy(), u=u.cpu().numpy(),
                   info=info, stages=stages, stats=stats)
        plan.close()
        return out

    mixed = run(ibdl.MIXED, args.steps, args.warmup, True)
    fp64 = run(ibdl.FP64, max(3, args.steps // 2), 1, False)

    if args.calib_copy_mib:
        nb = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # accuracy against the FP64 oracle (outside the timed region), and the
    # oracle's own throughput on a bounded sample of the same right-hand sides
    from oracle import ibdl_oracle as O
    from threadpoolctl import threadpool_limits
    st = O.setup_from_problem(p0)
    tight, _ = O.solve(st, p0.data, p0.g_tilde, tol=1e-13)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err_mixed = rel(mixed["sol"][0], tight.x)
    err_fp64 = rel(fp64["sol"][0], tight.x)
    err_u_mixed = rel(mixed["u"][0], O.eval_grid(st, tight.x, g_tilde=p0.g_tilde))
    cpu_iters, cpu_solves, t_cpu = 0, 0, 0.0
    if not args.no_cpu:
        with threadpool_limits(limits=1):
            for pr in probs:
                c0 = time.perf_counter()
                res, _ = O.solve(st, pr.data, pr.g_tilde, tol=tol)
                O.eval_grid(st, res.x, g_tilde=pr.g_tilde)
                t_cpu += time.perf_counter() - c0
                cpu_iters += res.iters
                cpu_solves += 1
                if t_cpu >= args.cpu_seconds:
                    break

    K = args.steps
    el = mixed["elapsed"]
    applies_s = mixed["iters"] / el
    solves_s = K * args.nrhs / el
    lat_ms = np.array(mixed["lat"]) * 1e3

    # roofline of the dominant kernel: a dedicated loop of mixed operator
    # applications with every right-hand side active and the stage events on
    rplan = ibdl.Plan.from_problem(p0, prec=ibdl.MIXED)
    gen = torch.Generator(device="cuda").manual_seed(7)
    q = torch.randn(args.nrhs, m, dtype=torch.float64, device="cuda", generator=gen)
    out = rplan.apply(q)
    for _ in range(5):
        rplan.apply(q, out=out)
    torch.cuda.synchronize()
    rplan.set_timing(True)
    for _ in range(ROOF_APPLIES):
        rplan.apply(q, out=out)
    stages = rplan.stage_times()
    rplan.set_timing(False)
    rstats = rplan.stats()
    rplan.close()
    sb = stage_bytes(rstats, dim, n, m, 1, args.nrhs)
    dom_ms = {nm: ms for nm, ms, _ in stages}
    dom = max(dom_ms, key=dom_ms.get)
    achieved = sb.get(dom, 0) / (dom_ms[dom] * 1e-3) / 1e9
    kname = stage_kernel(dom, dim, n)
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": int(sb.get(dom, 0))}
    flops = stage_flops(dim, n, args.nrhs).get(dom)
    if flops:
        # the column stage issues FFT arithmetic at a rate set by the vector ALUs
        # (instruction-issue bound in the counters), not by HBM bandwidth
        tf = flops / (dom_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kname, "stage": dom, "achieved": round(tf, 2),
                "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / ALU_PEAK_TFLOPS, 4),
                "traffic": read_traffic(args.workload, args.nrhs, kname), "flops_per_launch": int(flops),
                "ms_per_launch": round(dom_ms[dom], 5), "launches": ROOF_APPLIES, "hbm": hbm}
    else:
        roof = {"bound": "hbm", "kernel": kname, "stage": dom, "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": hbm["frac"], "traffic": read_traffic(args.workload, args.nrhs, kname),
                "bytes_per_launch": hbm["bytes_per_launch"], "ms_per_launch": round(dom_ms[dom], 5),
                "launches": ROOF_APPLIES}

    cpu = None
    if not args.no_cpu:
        cpu = {"value": round(cpu_iters / t_cpu, 3), "unit": "applies/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle solves (rhs, GMRES to tol {tol:g}, grid solution) of the first "
                         f"{cpu_solves} right-hand sides of the workload: {cpu_iters} applies in {t_cpu:.1f} s, "
                         f"one thread (numpy FFT; BLAS pools limited to 1)",
               "solves_per_s": round(cpu_solves / t_cpu, 4), "host_cpus": os.cpu_count()}

    line = {
        "metric": METRIC, "value": round(applies_s, 2), "unit": "applies/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(el / K * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 grid + f64 krylov", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "dim": dim, "M": m,
                   "alpha": p0.alpha, "bc": "dirichlet", "nrhs": args.nrhs, "tol": tol,
                   "precision": "mixed", "graphs": args.graphs == "on"},
        "solves_per_s": round(solves_s, 3),
        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 4),
        "iters_per_solve": round(mixed["iters"] / (K * args.nrhs), 2),
        "rel_err_vs_oracle": {"Q_mixed": err_mixed, "Q_fp64": err_fp64, "u_mixed": err_u_mixed},
        "fp64_path": {"applies_per_s": round(fp64["iters"] / fp64["elapsed"], 2),
                      "solves_per_s": round(len(fp64["lat"]) * args.nrhs / fp64["elapsed"], 3),
                      "latency_ms_p50": round(float(np.percentile(np.array(fp64["lat"]) * 1e3, 50)), 4)},
        "stages_ms_in_solves": {nm: round(ms, 5) for nm, ms, _ in mixed["stages"]},
        "stages_ms_apply": {nm: round(ms, 5) for nm, ms in dom_ms.items()},
        "full_grid_bytes_per_apply": full_grid_bytes_per_apply(dim, n, m, 1),
        "autotune": ibdl.autotune_report().splitlines(),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

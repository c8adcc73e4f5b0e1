"""Benchmark of the IBDL hot path on one MI355X.

Default workload (sphere256): the 3-D Dirichlet problem on a periodic unit cube
with a 256^3 grid, a sphere R = 0.3 with 40000 Fibonacci-lattice points, alpha =
10 and 32 distinct manufactured right-hand sides (harmonic u = exp(k.x)
cos(l.x + phase), forcing g = -alpha u inside the sphere).  A step is one
complete IBDL solve of all of them: the right-hand side, unpreconditioned GMRES
on the device to tol 1e-8, and the grid solution.  The geometry's plan
(binning, sort, spread matrices) is built once before timing.  Inputs are
resident on the GPU.

value = operator applications per second of the FP64 path (every GMRES
iteration of every right-hand side counts one application; the time includes
the right-hand side, the Krylov arithmetic and the grid solution).  Beside it
the line reports the mixed path (FP32 grid, FP64 Krylov with FP64 refinement):
applies/s, solves/s and latency percentiles; the error of both against FP64
oracle solves of the same right-hand sides; the HBM roofline of the dominant
kernel and of the whole operator (timed with HIP events on the library's
stream); and the oracle's own throughput on the host, on one thread and on all
cores.

--workload star1024: the 2-D star workload (1024^2 grid, star r = 0.3 + 0.05
cos 5t with 4096 points, alpha = 1, random-Fourier manufactured data) in the
same form.

--workload serve: the served stream: 2000 requests (80% 2-D, 20% 3-D, sizes
256^2..2048^2 and 64^3..256^3, alpha log-uniform in [1, 1000], mixed
precision, grid solution included) cycling through a set of materialised
request templates; first the saturation throughput with a bounded number of
requests outstanding, then seeded Poisson arrivals at 0.5x and 0.8x of it, with
p50/p99 of submission-to-result latency.

--workload batch512: a step is one batched solve of the 512-instance ellipse
batch (grid sizes 128..512, 2..8 right-hand sides each, Dirichlet and Neumann,
alpha log-uniform in [1, 1000], mixed precision) followed by the grid solutions
of every instance.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs R]
                       [--workload sphere256|star1024|batch512|serve]
"""
import argparse
import glob
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
ROOF_APPLIES = 20
KERNEL_SOURCES = ["paper_2203_12126_amd/csrc/pipeline.h", "paper_2203_12126_amd/csrc/fft.h",
                  "paper_2203_12126_amd/csrc/common.h"]
CPU_WORKERS_MAX = 16  # the host share of one GPU


def half_spectrum_bytes(dim, n, prec):
    """H = n^(d-1) (n/2+1) complex values of the pass's precision."""
    b = 8 if prec == 0 else 4
    return n ** (dim - 1) * (n // 2 + 1) * 2 * b


def operator_bytes(dim, n, m, prec):
    """Algorithmic bytes of one operator application (one right-hand side):
    B = (4d-4) H + M (16 + 2 d b): every axis pass reads and writes the half
    spectrum once, with the spread fused into the first pass and the
    interpolation into the last, plus the point data."""
    b = 8 if prec == 0 else 4
    return (4 * dim - 4) * half_spectrum_bytes(dim, n, prec) + m * (16 + 2 * dim * b)


def stage_share_bytes(dim, n, m, prec):
    """B split over the stages of a pass (one right-hand side): the first and last
    row passes write / read H, each column pass reads and writes H; the point
    terms go to the stages that move them.  The shares sum to B."""
    b = 8 if prec == 0 else 4
    H = half_spectrum_bytes(dim, n, prec)
    out = {"spread+fft_x": H + 8 * m}
    if dim == 2:
        out["fft_y+symbol"] = 2 * H
    else:
        out["fft_y"] = 2 * H
        out["fft_z+symbol"] = 2 * H
        out["ifft_y"] = 2 * H
    out["ifft_x+interp"] = H + 2 * dim * b * m
    out["finish"] = 8 * m
    return out


def stage_touched_bytes(st, dim, n, m, prec, nrhs):
    """Bytes each stage must move for this geometry, per call: only the lines
    that carry forcing or are read (the passes skip the rest)."""
    bc = 16 if prec == 0 else 8      # complex
    br = 8 if prec == 0 else 4       # real
    W = n // 2 + 1
    S, G = st["n_spread_lines"], st["n_gather_lines"]
    gpp = 4 if dim == 2 else 16
    csr = st["dip_nnz"] * (4 + br) + st["dip_active_nodes"] * 8 + (st["nlines"] + 1) * 4 + S * 4
    pts = m * (12 + 12 * br + 4)
    out = {"spread+fft_x": nrhs * (S * W * bc + m * 8) + csr}
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


def stage_kernel(stage, dim, n, prec, z_rows=1):
    """Kernel template behind a stage name (the row variants are tuned per shape;
    z_rows: the 3-D symbol pass's column rows per workgroup, from the plan)."""
    R = "double" if prec == 0 else "float"
    names = {"spread+fft_x": f"k_row_fwd<{R}, {n}>", "ifft_x+interp": f"k_row_inv<{R}, {n}, 0>",
             "finish": f"k_finish<{R}>"}
    if dim == 2:
        names["fft_y+symbol"] = f"k_col<{R}, {n}, 1, 1>"
    else:
        names["fft_y"] = f"k_col<{R}, {n}, 0, 1>"
        names["fft_z+symbol"] = f"k_col<{R}, {n}, 1, {z_rows}>"
        names["ifft_y"] = f"k_col<{R}, {n}, 2, 1>"
    return names.get(stage, stage)


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(workload, nrhs, kernel):
    """HBM bytes per launch of a kernel from the committed counter summaries
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when no summary covers
    this configuration or the kernel sources changed since the counters ran."""
    sha = kernel_sources_sha1()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        for ln in open(path).read().splitlines():
            if not ln.startswith("traffic:"):
                continue
            kv = dict(x.strip().split("=", 1) for x in ln[len("traffic:"):].split(";") if "=" in x)
            if (kv.get("workload") == workload and int(kv.get("nrhs", -1)) == nrhs and kv.get("kernel") == kernel
                    and kv.get("sources_sha1") == sha):
                return int(kv["bytes_per_launch"])
    return None


def make_workload(name, nrhs):
    from paper_2203_12126_amd import workloads as W
    if name == "star1024":
        probs = [W.config_star1024(m=4096, alpha=1.0, bc=W.DIRICHLET, seed=2203 + r) for r in range(nrhs)]
        desc = ("2-D Dirichlet screened Poisson, periodic unit square, 1024^2 grid, star "
                "r=0.3+0.05cos(5t) with 4096 points, alpha=1, random-Fourier manufactured data "
                "(one seed per right-hand side)")
    elif name == "sphere256":
        probs = [W.config_sphere256(seed=r) for r in range(nrhs)]
        desc = ("3-D Dirichlet screened Poisson, periodic unit cube, 256^3 grid, sphere R=0.3 with 40000 "
                "Fibonacci points, alpha=10, harmonic manufactured u=exp(k.x)cos(l.x+phase) "
                "(one seed per right-hand side)")
    else:
        raise SystemExit(f"unknown workload {name}")
    return probs, desc, 1e-8


def workload_problem(name, r):
    """Right-hand side r of a named workload (rebuilt in oracle worker processes)."""
    from paper_2203_12126_amd import workloads as W
    if name == "star1024":
        return W.config_star1024(m=4096, alpha=1.0, bc=W.DIRICHLET, seed=2203 + r)
    return W.config_sphere256(seed=r)


def _oracle_solve_worker(name, r, tol):
    """One FP64 oracle solve (right-hand side, GMRES, grid solution) on one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import ibdl_oracle as O
    p = workload_problem(name, r)
    st = O.setup_from_problem(p)
    with threadpool_limits(limits=1):
        c0 = time.perf_counter()
        res, _ = O.solve(st, p.data, p.g_tilde, tol=tol)
        u = O.eval_grid(st, res.x, g_tilde=p.g_tilde)
        el = time.perf_counter() - c0
    # applies: GMRES iterations, plus the right-hand side and the grid solution passes
    return r, res.iters, el, res.x, u


def _oracle_apply_worker(name, seconds):
    """Oracle operator applications on one thread for at least `seconds` (at least 2)."""
    from threadpoolctl import threadpool_limits
    from oracle import ibdl_oracle as O
    from paper_2203_12126_amd import workloads as W
    p = workload_problem(name, 0)
    st = O.setup_from_problem(p)
    q = W.random_density(p.geom.m, seed=1, nrhs=1)[0]
    k = 0
    with threadpool_limits(limits=1):
        c0 = time.perf_counter()
        while k < 2 or time.perf_counter() - c0 < seconds:
            O.apply_A(st, q)
            k += 1
        el = time.perf_counter() - c0
    return k, el


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(CPU_WORKERS_MAX, n))


def copy_rate_gbs(mib=1024, reps=5):
    """Device-to-device copy rate of the card: read plus write bytes over the best of
    `reps` timed copies of `mib` MiB (torch's copy kernel, events on its stream).
    It is the streaming rate a memory-bound kernel reaches in practice; `peak`
    stays the published figure."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (best * 1e-3) / 1e9


def batch_stage_bytes(metas):
    """Algorithmic bytes of one batched mixed apply, per stage, summed over instances."""
    tot = {}
    for mt in metas:
        for k, v in stage_share_bytes(mt["dim"], mt["n"], mt["m"], 1).items():
            tot[k] = tot.get(k, 0) + v * mt["nrhs"]
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
    sb = batch_stage_bytes(batch.meta)
    per_apply = {nm: ms * calls / napp for nm, ms, calls in stages}
    dom = max(per_apply, key=per_apply.get)
    achieved = sb.get(dom, 0) / (per_apply[dom] * 1e-3) / 1e9
    apply_ms = sum(per_apply.values())
    op_bytes = sum(operator_bytes(mt["dim"], mt["n"], mt["m"], 1) * mt["nrhs"] for mt in batch.meta)
    op_gbs = op_bytes / (apply_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": int(sb.get(dom, 0)), "ms_per_launch": round(per_apply[dom], 5),
            "note": "stage summed over the (grid size) groups of one batched apply",
            "copy_GBps": round(copy_rate_gbs(), 1),
            "operator": {"achieved": round(op_gbs, 1), "frac": round(op_gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_apply": int(op_bytes), "ms_per_apply": round(apply_ms, 5)}}

    # accuracy of a few instances against the FP64 oracle (outside the timed region)
    from oracle import ibdl_oracle as O
    # accuracy: the first instance of every grid size (its first right-hand side)
    # against the oracle's tight solve
    errs = {}
    for nn in sorted({sp["n"] for sp in specs}):
        i = next(j for j, sp in enumerate(specs) if sp["n"] == nn)
        p = items[i][0]
        st = O.setup_from_problem(p)
        ref, _ = O.solve(st, p.data, p.g_tilde, bc=p.bc, tol=1e-13)
        x = sol[i][0].cpu().numpy()
        errs[f"n{nn}"] = float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x))
    # the oracle's own rate: solves (tol of the batch) of the instances' first
    # right-hand sides in batch order, on one thread, for about --cpu-seconds
    cpu = None
    if not args.no_cpu:
        t_cpu, cpu_iters, ninst = 0.0, 0, 0
        for i in range(len(specs)):
            if t_cpu >= args.cpu_seconds:
                break
            p = items[i][0]
            st = O.setup_from_problem(p)
            c0 = time.perf_counter()
            res, _ = O.solve(st, p.data, p.g_tilde, bc=p.bc, tol=tol)
            t_cpu += time.perf_counter() - c0
            cpu_iters += res.iters
            ninst += 1
        cpu = {"value": round(cpu_iters / t_cpu, 3), "unit": "applies/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle solves of the first right-hand side of the first {ninst} instances "
                         f"of the batch ({cpu_iters} applies) in {t_cpu:.1f} s on one thread"}
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
    ap.add_argument("--workload", default="sphere256")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="length of the one-thread oracle sample (operator applications)")
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
    del probs[1:]
    nrhs = data.shape[0]

    def run(prec, steps, warmup):
        """Timed solve steps (ibdl_solve_grid of every right-hand side)."""
        plan = ibdl.Plan.from_problem(p0, prec=prec)
        # outputs allocated once, outside the timed steps
        sol_out = torch.empty_like(data)
        u_out = torch.empty((nrhs,) + (n,) * dim, dtype=torch.float64, device="cuda")
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
        el = time.perf_counter() - t0
        out = dict(elapsed=el, lat=lat, iters=iters, steps=steps, sol=sol.cpu().numpy(), u=u,
                   statuses=sorted({int(x) for x in info.field("status")}),
                   fp64_applies=int(info.field("fp64_applies").sum()), stats=plan.stats())
        plan.close()
        return out

    def roofline(prec):
        """A dedicated loop of operator applications with every right-hand side
        active and the stage events on (recorded in each stage kernel's own
        dispatch on the library's stream)."""
        rplan = ibdl.Plan.from_problem(p0, prec=prec)
        gen = torch.Generator(device="cuda").manual_seed(7)
        q = torch.randn(nrhs, m, dtype=torch.float64, device="cuda", generator=gen)
        out = rplan.apply(q)
        for _ in range(3):
            rplan.apply(q, out=out)
        torch.cuda.synchronize()
        rplan.set_timing(True)
        for _ in range(ROOF_APPLIES):
            rplan.apply(q, out=out)
        stages = rplan.stage_times()
        rplan.set_timing(False)
        rstats = rplan.stats()
        rplan.close()
        ms = {nm: v for nm, v, _ in stages}
        share = stage_share_bytes(dim, n, m, prec)
        touched = stage_touched_bytes(rstats, dim, n, m, prec, nrhs)
        dom = max(ms, key=ms.get)
        bpl = share[dom] * nrhs
        achieved = bpl / (ms[dom] * 1e-3) / 1e9
        apply_ms = sum(ms.values())
        opb = operator_bytes(dim, n, m, prec) * nrhs
        op_gbs = opb / (apply_ms * 1e-3) / 1e9
        kname = stage_kernel(dom, dim, n, prec, rstats["z_rows"])
        traffic = read_traffic(args.workload, nrhs, kname)
        return {
            "bound": "hbm", "kernel": kname, "stage": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": int(bpl), "ms_per_launch": round(ms[dom], 5), "launches": ROOF_APPLIES,
            "traffic_GBps": None if traffic is None else round(traffic / (ms[dom] * 1e-3) / 1e9, 1),
            "copy_GBps": copy_gbs,
            "touched_bytes_per_launch": int(touched[dom]),
            "operator": {"achieved": round(op_gbs, 1), "frac": round(op_gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_apply": int(opb), "ms_per_apply": round(apply_ms, 5),
                         "applies_per_s": round(nrhs / (apply_ms * 1e-3), 1)},
            "stages_ms": {k: round(v, 5) for k, v in ms.items()},
            "stages_frac": {k: round(share[k] * nrhs / (ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for k in ms
                            if k in share},
        }

    fp64 = run(ibdl.FP64, args.steps, args.warmup)
    mixed = run(ibdl.MIXED, args.steps, args.warmup)
    copy_gbs = round(copy_rate_gbs(), 1)
    roof64 = roofline(0)
    roof32 = roofline(1)

    if args.calib_copy_mib:
        nb = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # the oracle on the host: operator applications on one thread, and FP64 solves of
    # distinct right-hand sides in one process per core; the GPU solutions of the
    # same right-hand sides are compared with those solves
    cpu, errs = None, None
    if not args.no_cpu:
        import concurrent.futures as cf
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        cores = min(host_cores(), nrhs)
        with cf.ProcessPoolExecutor(max_workers=1, mp_context=ctx) as ex:
            k1, el1 = ex.submit(_oracle_apply_worker, args.workload, args.cpu_seconds).result()
        c0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
            futs = [ex.submit(_oracle_solve_worker, args.workload, r, tol) for r in range(cores)]
            res = [f.result() for f in futs]
        wall = time.perf_counter() - c0
        tot_iters = sum(x[1] for x in res)
        rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
        errs = {"rhs": [x[0] for x in res],
                "Q_fp64": [rel(fp64["sol"][x[0]], x[3]) for x in res],
                "Q_mixed": [rel(mixed["sol"][x[0]], x[3]) for x in res],
                "u_fp64": [rel(fp64["u"][x[0]].cpu().numpy(), x[4]) for x in res],
                "u_mixed": [rel(mixed["u"][x[0]].cpu().numpy(), x[4]) for x in res],
                "oracle_tol": tol}
        errs["max"] = {k: max(v) for k, v in errs.items() if k.startswith(("Q_", "u_"))}
        cpu = {"value": round(tot_iters / wall, 3), "unit": "applies/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 oracle solves (right-hand side, GMRES to tol {tol:g}, grid solution) of the first "
                         f"{cores} right-hand sides of the workload, one single-threaded process per core: "
                         f"{tot_iters} GMRES applies in {wall:.1f} s wall",
               "solves_per_s": round(cores / wall, 4), "host_cpus": os.cpu_count(),
               "one_thread": {"value": round(k1 / el1, 3), "unit": "applies/s", "cores": 1,
                              "sample": f"{k1} oracle operator applications in {el1:.1f} s on one thread "
                                        "(numpy FFT; BLAS pools limited to 1)"}}

    K = args.steps
    el = fp64["elapsed"]
    lat64 = np.array(fp64["lat"]) * 1e3
    lat32 = np.array(mixed["lat"]) * 1e3
    line = {
        "metric": METRIC, "value": round(fp64["iters"] / el, 2), "unit": "applies/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(el / K * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "dim": dim, "M": m,
                   "alpha": p0.alpha, "bc": "dirichlet", "nrhs": nrhs, "tol": tol, "precision": "fp64",
                   "graphs": args.graphs == "on"},
        "solves_per_s": round(K * nrhs / el, 3),
        "latency_ms_p50": round(float(np.percentile(lat64, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(lat64, 99)), 4),
        "iters_per_solve": round(fp64["iters"] / (K * nrhs), 2),
        "statuses": fp64["statuses"],
        "mixed_path": {"dtype": "f32 grid + f64 krylov", "applies_per_s": round(mixed["iters"] / mixed["elapsed"], 2),
                       "solves_per_s": round(K * nrhs / mixed["elapsed"], 3),
                       "ms_per_step": round(mixed["elapsed"] / K * 1e3, 4),
                       "latency_ms_p50": round(float(np.percentile(lat32, 50)), 4),
                       "latency_ms_p99": round(float(np.percentile(lat32, 99)), 4),
                       "iters_per_solve": round(mixed["iters"] / (K * nrhs), 2),
                       "fp64_residual_passes_per_solve": round(mixed["fp64_applies"] / nrhs, 2),
                       "statuses": mixed["statuses"], "roofline": roof32},
        "rel_err_vs_oracle": errs,
        "autotune": ibdl.autotune_report().splitlines(),
        "roofline": roof64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

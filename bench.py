#!/usr/bin/env python3
"""Benchmark of the AD-INLA hot path on one MI355X.

A step is one exact gradient of the INLA objective (forward sweeps of Qc and Qp with the
fused forward solve, then the upper solve, selected inversion with trace epilogues, Phase B
and gradient assembly) on the synthetic univariate SPDE model with a 32x32 grid (b = 1024),
50 time steps, 6 covariates, 200 observations per step and d = 4.  It is compared with the
GPU's own (2d+1)-point central-difference gradient (all 9 objective evaluations batched into
one pass of the same kernels).  Steps are captured once into a hipGraph and replayed.

Printed: one JSON line (value = AD gradients per second).  A separate, event-profiled pass
gives the roofline numbers of the dominant kernel; the dense CPU oracle is timed on a bounded
sample of the same workload as the CPU baseline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gradients/sec AD vs 2d+1 FD at rel 1e-8; FP64 MFMA % peak for BTA factor+selinv"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# profiler names of the library's kernel groups -> device kernel symbols (as rocprofv3 lists them)
KERNEL_SYMBOLS = {"gemm_f64": "gemm_f64_kernel", "potrf_panel": "potrf_panel_kernel",
                  "gemv": "gemv_t_kernel", "assemble": "assemble_blocks_kernel",
                  "trace": "trace_kernel", "tip": "tip_kernel", "panel_step": "panel_step_kernel",
                  "w_sparse": "w_from_gtg_kernel"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uni_32x32_nt50")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-nt", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--hessian", action="store_true",
                    help="time the posterior Hessian of Eq. 12 (2d+1 exact gradients) against "
                         "the 2d^2+1-point finite-difference Hessian instead")
    ap.add_argument("--sweep", choices=["time", "space"], default=None,
                    help="problem-size sweep of c_AD = T_AD / T_f and beta = t_bwd / t_fwd: "
                         "n = 2..256 steps on the 32x32 univariate grid (time), or three "
                         "coregionalised fields on ns = 72..1122 nodes, n = 16 (space)")
    ap.add_argument("--no-split", action="store_true",
                    help="time the gradient without the two-sided split of the block chain")
    ap.add_argument("--no-d15", action="store_true",
                    help="skip the nested d = 15 measurement (coreg3_30x30_nt48)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep every GEMM on 64 x 64 tiles instead of the autotuned table")
    ap.add_argument("--progress", action="store_true",
                    help="print a line to stderr after every timed step (long workloads)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the event-profiled gradient steps (the command rocprofv3 traces)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="with --roofline-only: also run one plain device copy of this many MiB, "
                         "the reference dispatch for scaling HBM byte counters")
    return ap.parse_args()


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs scaled by a plain copy of known size), or None when there is none or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


def timed(fn, steps, warmup, use_graph, torch):
    """Mean ms per call of fn() over `steps` calls (after `warmup`), timed with events on the
    current stream (the library launches on that stream)."""
    if use_graph:
        fn()  # allocations (workspaces) happen outside the capture
        torch.cuda.synchronize()
        if PROGRESS:
            print("first call done", file=sys.stderr, flush=True)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        run = g.replay
    else:
        run = fn
    for _ in range(warmup):
        run()
        if PROGRESS:
            torch.cuda.synchronize()
            print("warm-up step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for t in range(steps):
        run()
        ev[t + 1].record()
        if PROGRESS:  # long calls: a line per finished step
            ev[t + 1].synchronize()
            print(f"step {t + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    per_call = [ev[t].elapsed_time(ev[t + 1]) for t in range(steps)]
    TIMES[id(fn)] = per_call
    return ev[0].elapsed_time(ev[steps]) / steps


TIMES = {}
PROGRESS = False


def timed_backward(model, theta, f, g, info, steps, warmup, use_graph, torch):
    """Mean ms of the reverse pass alone: each step replays the forward pass that saves the
    factors (untimed) and then the gradient that reuses them (timed with its own events), since
    a reuse consumes the saved factors."""
    fwd = lambda: model.forward_saved(theta)  # noqa: E731
    bwd = lambda: model.grad(theta, reuse=True, f=f, g=g, info=info)  # noqa: E731
    fwd()
    bwd()
    torch.cuda.synchronize()
    if use_graph:
        ga = torch.cuda.CUDAGraph()
        with torch.cuda.graph(ga):
            fwd()
        gb = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gb):
            bwd()
        run_f, run_b = ga.replay, gb.replay
    else:
        run_f, run_b = fwd, bwd
    for _ in range(warmup):
        run_f()
        run_b()
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(steps):
        run_f()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run_b()
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
    return total / steps


def median_ci(xs):
    """Median and a distribution-free 95% confidence interval for it (order statistics of the
    binomial(n, 1/2) ranks, normal approximation)."""
    v = sorted(xs)
    n = len(v)
    if n == 0:
        return None
    med = v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])
    half = 0.98 * math.sqrt(n)
    lo = v[max(0, int(math.floor(n / 2 - half)))]
    hi = v[min(n - 1, int(math.ceil(n / 2 + half)) - 1)]
    return {"median": med, "ci95": [lo, hi], "n": n}


def algorithmic_flops(b, n, a):
    """Dense-block work of the method per block and matrix (flops, multiply-add = 2):
    forward (Alg. 1) POTRF b^3/3 + TRSM b^3 + SYRK b^3 per block (the last block: POTRF);
    selected inversion (14/3) b^3 per block."""
    fwd = 2 * ((n - 1) * (7.0 / 3.0) + 1.0 / 3.0) * b ** 3
    si = 2 * (14.0 / 3.0) * n * b ** 3
    return fwd, si


def event_gap_ms(torch, n=257):
    """Median gap between consecutive event records on the stream, with the device held busy
    so that all records are queued before the first is processed."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    torch.cuda.synchronize()
    torch.cuda._sleep(20_000_000)
    for e in evs:
        e.record()
    torch.cuda.synchronize()
    gaps = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(n - 1))
    return gaps[len(gaps) // 2]


def profiled_pass(args, ad_step, bta, torch):
    """Per-kernel time and algorithmic work of `profile_steps` gradient steps.  The device is
    first held busy (torch.cuda._sleep) so that every launch and event of the profiled steps is
    already queued when they run: the event intervals then bracket the kernels back to back
    instead of including host launch latency."""
    ad_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with bta.profile() as P0:
        ad_step()
    host_s = time.perf_counter() - t0  # host time to enqueue one step with its events
    # ~2.0e9 cycles/s: hold for twice the enqueue time of the profiled steps
    hold_cycles = int(2.0 * host_s * args.profile_steps * 2.0e9) + 50_000_000
    with bta.profile() as P:
        torch.cuda._sleep(hold_cycles)
        for _ in range(args.profile_steps):
            ad_step()
    stats = P.stats
    # An event interval around a launch also holds the processing of one event record; the gap
    # between back-to-back records (device held, nothing in between) measures it, and it is
    # taken off every launch interval of the dominant kernel.
    ovh_ms = event_gap_ms(torch)
    gemm_like = {k: v for k, v in stats.items() if ":" not in k}
    # the dominant kernel by kernel time: its event time less one record gap per launch (a
    # kernel launched often would otherwise be charged for its many gaps)
    name, st = max(gemm_like.items(), key=lambda kv: kv[1]["ms"] - kv[1]["launches"] * ovh_ms)
    launches = max(st["launches"], 1)
    raw_ms = st["ms"]
    kern_ms = max(raw_ms - launches * ovh_ms, 1e-9)
    per_launch_ms = kern_ms / launches
    if st["flops"] > 0 and name not in ("gemv", "assemble", "trace", "w_sparse"):
        achieved = st["flops"] / (kern_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
    else:
        achieved = st["bytes"] / (kern_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    if st["bytes"] > 0:
        roof["algorithmic_bytes_per_launch"] = st["bytes"] / launches
    roof.update({"kernel": name, "kernel_symbol": KERNEL_SYMBOLS.get(name, name),
                 "launches_per_step": st["launches"] / args.profile_steps,
                 "avg_launch_us": per_launch_ms * 1e3,
                 "avg_event_interval_us": raw_ms / launches * 1e3,
                 "event_record_gap_us": ovh_ms * 1e3,
                 "algorithmic_per_launch": (st["flops"] or st["bytes"]) / max(st["launches"], 1),
                 "host_enqueue_ms_per_step": host_s * 1e3})
    return stats, roof


def cpu_baseline(spec_name, seed, nt_sample):
    import numpy as np
    import oracle
    from workloads import NAMED_CONFIGS, make_model
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    k, nx, ny, nt, a, obs = NAMED_CONFIGS[spec_name]
    sample = make_model(k, nx, ny, nt_sample, a, obs, seed)
    t0 = time.perf_counter()
    oracle.gradient(sample, sample.theta)
    ts = time.perf_counter() - t0
    N_full = nt * k * nx * ny + a
    scale = (N_full / sample.N) ** 3
    return {
        "value": 1.0 / (ts * scale),
        "unit": "gradients/s",
        "extrapolated": True,
        "measured": {"N": int(sample.N), "nt": nt_sample, "seconds_per_gradient": ts,
                     "gradients_per_s": 1.0 / ts},
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"dense oracle f + exact gradient on the same grid and covariates with "
                   f"nt={nt_sample} (N={sample.N}) took {ts:.2f} s on {threads} BLAS threads; "
                   f"scaled by (N/N_sample)^3 = {scale:.4g} to the full N={N_full}"),
        "sample_seconds": ts,
        "cpu_count": os.cpu_count(),
        "single_thread": single_thread_oracle(k, nx, ny, nt, a, obs, seed, N_full),
    }


def single_thread_oracle(k, nx, ny, nt, a, obs, seed, N_full, nt_sample=2):
    """The same oracle gradient with the BLAS limited to one thread, on a smaller sample."""
    import oracle
    from workloads import make_model
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        return None
    sample = make_model(k, nx, ny, nt_sample, a, obs, seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.gradient(sample, sample.theta)
        ts = time.perf_counter() - t0
    scale = (N_full / sample.N) ** 3
    return {"value": 1.0 / (ts * scale), "unit": "gradients/s", "cores": 1,
            "sample": (f"nt={nt_sample} (N={sample.N}) took {ts:.2f} s on 1 BLAS thread; "
                       f"scaled by (N/N_sample)^3 = {scale:.4g}"),
            "sample_seconds": ts}


UNEVEN_COUNT = 64
# block size -> grid of the uneven batch's instances (b = nx * ny)
UNEVEN_GRIDS = {128: (16, 8), 256: (16, 16), 512: (32, 16), 1024: (32, 32)}


def uneven_shapes(seed, count=UNEVEN_COUNT):
    """An uneven batch: b in {128, 256, 512, 1024}, n in [8, 64], a in [2, 8], drawn from seed."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(8, 65)), int(rng.choice([128, 256, 512, 1024])),
             int(rng.integers(2, 9))) for _ in range(count)]


def bench_uneven(args, torch):
    """An uneven batch of 64 INLA instances (block sizes 128..1024 on 16x8..32x32 grids, 8..64
    time steps, 2..8 fixed effects, b/8 observations per step, each at its own theta drawn from
    the seed): objectives and exact gradients of all of them per call (inla_batch_objective /
    inla_batch_grad, instances of one block size sharing every launch), timed from graph
    replays.  Beside it, the batched BTA factorisation of random matrices of the same shapes."""
    import numpy as np
    from paper_2605_06392_amd import bta, inla
    from workloads import make_model

    dev = torch.device("cuda:0")
    shapes = uneven_shapes(args.seed)
    specs, models = [], []
    for i, (n, b, a) in enumerate(shapes):
        nx, ny = UNEVEN_GRIDS[b]
        spec = make_model(1, nx, ny, n, a, b // 8, args.seed * 1000 + i)
        specs.append(spec)
        models.append(inla.InlaModel(spec, device=dev))
        if PROGRESS:
            print(f"instance {i + 1}/{len(shapes)} created", file=sys.stderr, flush=True)
    B = inla.InlaBatch(models)
    theta = torch.tensor(np.stack([s.theta for s in specs]), dtype=torch.float64, device=dev)
    B.theta.copy_(theta)
    torch.cuda.reset_peak_memory_stats()

    def replay_times(kind, steps, warmup):
        B.capture(kind)
        for _ in range(warmup):
            B.replay(kind)
            if PROGRESS:
                torch.cuda.synchronize()
                print(f"{kind}: warm-up replay done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        out = []
        for t in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            B.replay(kind)
            e1.record()
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
            if PROGRESS:
                print(f"{kind}: replay {t + 1}/{steps} done", file=sys.stderr, flush=True)
        return out

    # first with every product on 64 x 64 tiles, then with the tiles the autotuner picks per block
    # size and role (coordinate search over timed gradient calls of each block-size group)
    inla.clear_tiles()
    t_obj64 = replay_times("objective", args.steps, args.warmup)
    t_grad64 = replay_times("grad", args.steps, args.warmup)
    t0 = time.perf_counter()
    changed = B.autotune("grad", reps=2)
    tune_s = time.perf_counter() - t0
    table = inla.tile_table(sorted(UNEVEN_GRIDS))
    if PROGRESS:
        print(f"autotune: {changed} choices changed in {tune_s:.1f} s", file=sys.stderr, flush=True)
    t_obj = replay_times("objective", args.steps, args.warmup)
    f_obj = B.f.clone()
    t_grad = replay_times("grad", args.steps, args.warmup)
    torch.cuda.synchronize()
    f_b, g_b, info_b = B.f.cpu().numpy(), B.g.cpu().numpy(), B.info.cpu().numpy()
    infos_ok = bool((info_b == 0).all())
    peak = torch.cuda.max_memory_allocated()
    # consistency: instances evaluated one at a time (smallest, largest, and one of each block
    # size) give the same f and gradient
    pick = sorted(range(len(shapes)), key=lambda i: shapes[i][0] * shapes[i][1] ** 2)
    check_idx = {pick[0], pick[-1]}
    for bb in UNEVEN_GRIDS:
        members = [i for i in range(len(shapes)) if shapes[i][1] == bb]
        if members:
            check_idx.add(members[0])
    rel_f = rel_g = 0.0
    for i in sorted(check_idx):
        f1, g1, inf1 = models[i].grad(theta[i])
        torch.cuda.synchronize()
        rel_f = max(rel_f, abs(f1.item() - f_b[i]) / abs(f1.item()))
        rel_g = max(rel_g, float(np.abs(g1.cpu().numpy() - g_b[i]).max() /
                                 np.abs(g1.cpu().numpy()).max()))
        infos_ok = infos_ok and int(inf1.item()) == 0
    obj_vs_grad_f = float((f_obj.cpu().numpy() - f_b).__abs__().max() / np.abs(f_b).max())

    # App. B work of the instances: forward per matrix, selected inversion per block
    fwd_fl = sum(2 * ((n - 1) * 7.0 / 3.0 + 1.0 / 3.0) * b ** 3 for n, b, _ in shapes)
    si_fl = sum(2 * (14.0 / 3.0) * n * b ** 3 for n, b, _ in shapes)
    ms_obj = sum(t_obj) / len(t_obj)
    ms_grad = sum(t_grad) / len(t_grad)
    d = B.d
    count = len(shapes)
    line = {
        "metric": "INLA gradients/s and objectives/s, uneven batch of instances in one call",
        "value": count * 1000.0 / ms_grad,
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_grad,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uneven64", "count": count, "seed": args.seed, "d": d,
                   "b_counts": {str(bb): sum(1 for _, b, _ in shapes if b == bb)
                                for bb in UNEVEN_GRIDS},
                   "n_range": [min(n for n, _, _ in shapes), max(n for n, _, _ in shapes)],
                   "a_range": [min(a for _, _, a in shapes), max(a for _, _, a in shapes)],
                   "obs_per_step": "b/8", "groups": B.groups, "graph": True},
        "objectives_per_s": count * 1000.0 / ms_obj,
        "ms_per_objective_batch": median_ci(t_obj),
        "ms_per_gradient_batch": median_ci(t_grad),
        "autotune": {"changed": changed, "seconds": tune_s,
                     "tiles_not_64": {str(bb): [r for r, t in roles.items() if t != 64]
                                      for bb, roles in table.items()},
                     "untuned_64x64": {"ms_per_objective_batch": median_ci(t_obj64),
                                       "ms_per_gradient_batch": median_ci(t_grad64)}},
        "fd_gradients_per_s_from_objective_batches": count * 1000.0 / ((2 * d + 1) * ms_obj),
        "ad_over_fd_speedup": (2 * d + 1) * ms_obj / ms_grad,
        "tflops_paper_flop_model": {"objective": fwd_fl / (ms_obj * 1e-3) / 1e12,
                                    "gradient": (fwd_fl + si_fl) / (ms_grad * 1e-3) / 1e12},
        "check": {"info_ok": infos_ok, "instances_vs_single_model": sorted(check_idx),
                  "f_rel_vs_single": rel_f, "grad_rel_vs_single": rel_g,
                  "objective_vs_gradient_call_f_rel": obj_vs_grad_f},
        "peak_device_memory_gb": peak / 1e9,
    }
    del B, models
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    line["bta_factor_batched"] = bench_uneven_factor(args, torch, shapes)
    print(json.dumps(line), flush=True)


def bench_uneven_factor(args, torch, shapes):
    """Batched factorisation (with the fused lower solve) of random BTA matrices of the uneven
    batch's shapes in one bta_factor_batched call."""
    from paper_2605_06392_amd import bta
    from workloads.bta import random_bta_device

    dev = torch.device("cuda:0")
    keys = ("D", "B", "C", "T")
    pristine, work = [], []
    for i, (n, b, a) in enumerate(shapes):
        blk = random_bta_device(n, b, a, args.seed * 1000 + i, dev)
        m = {"D": bta.to_cm(blk["D"]), "B": bta.to_cm(blk["B"]) if n > 1 else None,
             "C": bta.to_cm(blk["C"]), "T": bta.to_cm(blk["T"][None])[0], "rhs": blk["rhs"]}
        del blk
        pristine.append(m)
        work.append({k: (v.clone() if v is not None else None) for k, v in m.items()})

    def restore():
        for w, p in zip(work, pristine):
            for k in keys + ("rhs",):
                if p[k] is not None:
                    w[k].copy_(p[k])

    # the factorisation's algorithmic work (App. B, one matrix): POTRF b^3/3 per block, TRSM and
    # the Schur update b^3 each for every block but the last
    flops = sum(((n - 1) * 7.0 / 3.0 + 1.0 / 3.0) * b ** 3 for n, b, _ in shapes)
    for _ in range(max(1, args.warmup)):
        restore()
        bta.bta_factor_batched(work, with_rhs=True)
    torch.cuda.synchronize()
    per_call = []
    infos_ok = True
    for _ in range(max(3, args.steps // 2)):
        restore()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, logdet, info = bta.bta_factor_batched(work, with_rhs=True)
        e1.record()
        torch.cuda.synchronize()
        per_call.append(e0.elapsed_time(e1))
        infos_ok = infos_ok and bool((info == 0).all().item())
    # consistency: the smallest matrices factorised one at a time give the same log-determinants
    order = sorted(range(len(shapes)), key=lambda i: shapes[i][0] * shapes[i][1] ** 2)[:3]
    rel = 0.0
    for i in order:
        m = {k: (v.clone() if v is not None else None) for k, v in pristine[i].items()}
        _, ld1, inf1 = bta.bta_factor(m["D"], m["B"], m["C"], m["T"], m["rhs"])
        rel = max(rel, abs(ld1.item() - logdet[i].item()) / abs(ld1.item()))
        infos_ok = infos_ok and int(inf1.item()) == 0
    mean = sum(per_call) / len(per_call)
    return {"matrices_per_s": len(shapes) * 1000.0 / mean, "ms_per_call": median_ci(per_call),
            "tflops_paper_flop_model": flops / (mean * 1e-3) / 1e12,
            "check": {"info_ok": infos_ok, "logdet_vs_single_rel": rel}}


def bench_d15(args, torch, np, workload="coreg3_30x30_nt48"):
    """AD gradient against the GPU's 31-point FD gradient on the three-field d = 15 model
    (b = 2700, n = 48, a = 6): a few graph replays of each, the FD batch in one pass."""
    from paper_2605_06392_amd import inla
    from workloads import named_config
    dev = torch.device("cuda:0")
    spec = named_config(workload, seed=args.seed)
    model = inla.InlaModel(spec, device=dev)
    d = model.d
    npts = 2 * d + 1
    theta = torch.tensor(spec.theta, dtype=torch.float64, device=dev)
    f_ad = torch.empty(1, dtype=torch.float64, device=dev)
    g_ad = torch.empty(d, dtype=torch.float64, device=dev)
    i_ad = torch.empty(1, dtype=torch.int32, device=dev)
    f_fd = torch.empty(1, dtype=torch.float64, device=dev)
    g_fd = torch.empty(d, dtype=torch.float64, device=dev)
    i_fd = torch.empty(npts, dtype=torch.int32, device=dev)
    print(f"d15: model {workload} on the device", file=sys.stderr, flush=True)
    model.grad(theta, f=f_ad, g=g_ad, info=i_ad)
    model.fd_grad(theta, h=1e-4, max_batch=npts, f=f_fd, g=g_fd, info=i_fd)
    torch.cuda.synchronize()
    gad, gfd = g_ad.cpu().numpy(), g_fd.cpu().numpy()
    rel = float(np.abs(gad - gfd).max() / np.abs(gad).max())
    ok = int(i_ad.item()) == 0 and bool((i_fd.cpu().numpy() == 0).all())
    print("d15: accuracy check done", file=sys.stderr, flush=True)
    fd_step = lambda: model.fd_grad(theta, h=1e-3, max_batch=npts, f=f_fd, g=g_fd, info=i_fd)  # noqa: E731
    plain = lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad)  # noqa: E731
    ms_plain = timed(plain, 3, 1, True, torch)
    ad_step = lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad, split=True)  # noqa: E731
    ms_ad = timed(ad_step, 3, 1, True, torch)
    torch.cuda.synchronize()
    split_rel = float(np.abs(g_ad.cpu().numpy() - gad).max() / np.abs(gad).max())
    print(f"d15: AD {ms_ad:.1f} ms (plain sweep {ms_plain:.1f} ms)", file=sys.stderr, flush=True)
    ms_fd = timed(fd_step, 2, 1, True, torch)
    print(f"d15: FD {ms_fd:.1f} ms", file=sys.stderr, flush=True)
    k, nx, ny, nt, a, obs = NAMED_CONFIGS_REF[workload]
    b = k * nx * ny
    fwd_fl, si_fl = algorithmic_flops(b, nt, a)
    out = {"workload": workload, "b": b, "n": nt, "a": a, "d": d, "N": nt * b + a,
           "ms_ad_gradient": ms_ad, "ms_fd_gradient": ms_fd, "ad_over_fd_speedup": ms_fd / ms_ad,
           "ad_gradients_per_s": 1000.0 / ms_ad, "fd_gradients_per_s": 1000.0 / ms_fd,
           "ad_tflops_paper_flop_model": (fwd_fl + si_fl) / (ms_ad * 1e-3) / 1e12,
           "fd_points": npts,
           "check": {"ad_vs_gpu_fd_rel_inf_h1e-4": rel, "info_ok": ok,
                     "split_vs_plain_grad_rel": split_rel},
           "split": True, "ms_ad_plain_sweep": ms_plain,
           "ms_ad_per_call": median_ci(TIMES.get(id(ad_step), [])),
           "ms_fd_per_call": median_ci(TIMES.get(id(fd_step), []))}
    del model
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def bench_hessian(args, model, theta, spec, torch, np):
    """Posterior Hessian at theta: Eq. 12 (2d+1 exact gradients, one graph) against the
    second-order FD Hessian (2d^2+1 objectives: the faster of one batched call and sub-batches
    of 2d+1 points)."""
    d = model.d
    dev = theta.device
    f = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(d, dtype=torch.float64, device=dev)
    H = torch.empty((d, d), dtype=torch.float64, device=dev)
    info = torch.empty(2 * d + 1, dtype=torch.int32, device=dev)
    nfd = 2 * d * d + 1
    Hf = torch.empty((d, d), dtype=torch.float64, device=dev)
    ff = torch.empty(1, dtype=torch.float64, device=dev)
    info_f = torch.empty(nfd, dtype=torch.int32, device=dev)
    use_graph = not args.no_graph
    # Eq. 12: the 2d+1 gradients in as few passes as the memory allows (and one at a time)
    total = torch.cuda.get_device_properties(dev).total_memory
    ad_batches = sorted({1, model.fitting_batch(2 * d + 1, 1)})
    ad_ms, ad_calls = {}, {}
    for mb in ad_batches:
        ad = lambda: model.hessian(theta, h=5e-3, max_batch=mb, f=f, g=g, H=H, info=info)  # noqa: E731,B023
        ad_ms[mb] = timed(ad, args.steps, args.warmup, use_graph, torch)
        ad_calls[mb] = TIMES[id(ad)]
    best_ad = min(ad_ms, key=ad_ms.get)
    ms_ad = ad_ms[best_ad]
    torch.cuda.synchronize()
    peak_ad = torch.cuda.max_memory_allocated()
    fd_ms = {}
    fd_calls = {}
    # batch sizes whose objective workspace fits in half of the device memory
    sizes = [mb for mb in sorted({nfd, 2 * d + 1})
             if model.workspace_bytes(mb, 0) <= total // 2] or [2 * d + 1]
    for mb in sizes:
        fd = lambda: model.fd_hessian(theta, h=5e-3, max_batch=mb, f=ff, H=Hf, info=info_f)  # noqa: E731,B023
        # an FD Hessian in several passes is timed eagerly: capturing one (about 2e5 launches at
        # b = 2700, d = 15) ended the process during capture or replay
        fd_ms[mb] = timed(fd, max(1, args.steps // 2), min(1, args.warmup),
                          use_graph and mb >= nfd, torch)
        fd_calls[mb] = TIMES[id(fd)]
    best = min(fd_ms, key=fd_ms.get)
    torch.cuda.synchronize()
    Hn, Hfn = H.cpu().numpy(), Hf.cpu().numpy()
    scale = np.abs(Hn).max()
    k, nx, ny, nt, a, obs = NAMED_CONFIGS_REF[args.workload]
    line = {
        "metric": "posterior Hessians/s: Eq. 12 (2d+1 exact gradients) vs 2d^2+1-point FD",
        "value": 1000.0 / ms_ad,
        "unit": "hessians/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_ad,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "b": k * nx * ny, "n": nt, "a": a, "d": d,
                   "h": 5e-3, "seed": args.seed, "graph": use_graph},
        "ad_hessian_max_batch": best_ad,
        "ms_ad_hessian_by_batch": {str(mb_): v for mb_, v in ad_ms.items()},
        "ms_per_fd_hessian": fd_ms[best],
        "fd_hessian_max_batch": best,
        "ms_fd_hessian_by_batch": {str(mb_): v for mb_, v in fd_ms.items()},
        "ad_over_fd_speedup": fd_ms[best] / ms_ad,
        "ms_ad_per_call": median_ci(ad_calls[best_ad]),
        "ms_fd_per_call": median_ci(fd_calls[best]),
        "check": {"info_ok": bool((info == 0).all().item()) and bool((info_f == 0).all().item()),
                  "asymmetry_rel": float(np.abs(Hn - Hn.T).max() / scale),
                  "ad_vs_fd_hessian_rel": float(np.abs(Hn - Hfn).max() / scale)},
        "peak_device_memory_gb": {"ad": peak_ad / 1e9,
                                  "with_fd_batch": torch.cuda.max_memory_allocated() / 1e9},
    }
    print(json.dumps(line), flush=True)


NAMED_CONFIGS_REF = {}

SWEEPS = {
    # (k, nx, ny, nt, a, obs per step and field)
    "time": [(1, 32, 32, n, 6, 200) for n in (2, 4, 8, 16, 32, 64, 128, 256)],
    "space": [(3, nx, ny, 16, 6, max(nx * ny // 4, 8))
              for nx, ny in ((9, 8), (12, 12), (18, 16), (24, 24), (30, 30), (34, 33))],
}


def bench_sweep(args, torch, np):
    """c_AD = T_AD / T_f (one exact gradient against one objective evaluation), beta =
    t_bwd / t_fwd, and the AD speed-up over the batched (2d+1)-point FD gradient, over a family
    of problem sizes; one JSON line per size, then a summary line."""
    from paper_2605_06392_amd import inla
    from workloads import make_model
    dev = torch.device("cuda:0")
    use_graph = not args.no_graph
    rows = []
    for k, nx, ny, nt, a, obs in SWEEPS[args.sweep]:
        spec = make_model(k, nx, ny, nt, a, obs, args.seed)
        model = inla.InlaModel(spec, device=dev)
        d = model.d
        npts = 2 * d + 1
        theta = torch.tensor(spec.theta, dtype=torch.float64, device=dev)
        f1 = torch.empty(1, dtype=torch.float64, device=dev)
        i1 = torch.empty(1, dtype=torch.int32, device=dev)
        g = torch.empty(d, dtype=torch.float64, device=dev)
        gf = torch.empty(d, dtype=torch.float64, device=dev)
        ifd = torch.empty(npts, dtype=torch.int32, device=dev)
        th1 = theta[None].contiguous()
        steps, warm = args.steps, args.warmup
        ms_f = timed(lambda: model.objective(th1, out=f1, info=i1), steps, warm, use_graph, torch)
        ms_ad = timed(lambda: model.grad(theta, f=f1, g=g, info=i1), steps, warm, use_graph, torch)
        ms_fwd = timed(lambda: model.forward_saved(theta), steps, warm, use_graph, torch)
        ms_bwd = timed_backward(model, theta, f1, g, i1, steps, warm, use_graph, torch)
        mb = model.fitting_batch(npts, 0)
        ms_fd = timed(lambda: model.fd_grad(theta, h=1e-3, max_batch=mb, f=f1, g=gf, info=ifd),
                      steps, warm, use_graph, torch)
        torch.cuda.synchronize()
        ok = bool((i1 == 0).all().item()) and bool((ifd == 0).all().item())
        row = {"k": k, "nx": nx, "ny": ny, "ns": nx * ny, "b": k * nx * ny, "n": nt, "a": a,
               "d": d, "ms_f": ms_f, "ms_ad": ms_ad, "ms_fwd": ms_fwd, "ms_bwd": ms_bwd,
               "ms_fd_gradient": ms_fd, "fd_max_batch": mb, "c_AD": ms_ad / ms_f,
               "beta": ms_bwd / ms_fwd, "ad_over_fd": ms_fd / ms_ad,
               "ad_over_sequential_fd": npts * ms_f / ms_ad, "info_ok": ok}
        rows.append(row)
        print(json.dumps({"sweep": args.sweep, **row}), flush=True)
        del model
        torch.cuda.empty_cache()
    print(json.dumps({"metric": f"problem-size sweep ({args.sweep})", "unit": "c_AD, beta",
                      "c_AD": [r["c_AD"] for r in rows], "beta": [r["beta"] for r in rows],
                      "ad_over_fd": [r["ad_over_fd"] for r in rows],
                      "sizes": [(r["b"], r["n"]) for r in rows], "dtype": "f64",
                      "data": "synthetic", "graph": use_graph, "seed": args.seed}), flush=True)


def main():
    args = parse()
    global PROGRESS
    PROGRESS = args.progress
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path; "
              "the stencil points or the time axis would be split across GPUs", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.sweep:
        torch.cuda.set_device(0)
        bench_sweep(args, torch, np)
        return
    if args.workload == "uneven64":
        torch.cuda.set_device(0)
        bench_uneven(args, torch)
        return
    from workloads import NAMED_CONFIGS, named_config
    NAMED_CONFIGS_REF.update(NAMED_CONFIGS)
    from paper_2605_06392_amd import bta, inla

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = named_config(args.workload, seed=args.seed)
    model = inla.InlaModel(spec, device=dev)
    d = model.d
    npts = 2 * d + 1
    theta = torch.tensor(spec.theta, dtype=torch.float64, device=dev)
    f_ad = torch.empty(1, dtype=torch.float64, device=dev)
    g_ad = torch.empty(d, dtype=torch.float64, device=dev)
    i_ad = torch.empty(1, dtype=torch.int32, device=dev)
    f_fd = torch.empty(1, dtype=torch.float64, device=dev)
    g_fd = torch.empty(d, dtype=torch.float64, device=dev)
    i_fd = torch.empty(npts, dtype=torch.int32, device=dev)

    if args.hessian:
        bench_hessian(args, model, theta, spec, torch, np)
        return

    if args.roofline_only:
        # the headline gradient (the two-sided split when the model has one)
        sp = (not args.no_split) and model.workspace_bytes(1, inla.MODE_GRAD_SPLIT) > 0
        ad_only = lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad, split=sp)  # noqa: E731
        for _ in range(args.warmup):
            ad_only()
        stats, roof = profiled_pass(args, ad_only, bta, torch)
        if args.calibration_copy_mib > 0:
            n = args.calibration_copy_mib * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            roof["calibration_copy_bytes_each_way"] = n * 8
        roof["traffic"] = measured_traffic(roof["kernel_symbol"], args.workload)
        print(json.dumps({"roofline": roof, "kernels": stats}), flush=True)
        return

    # accuracy at full size: AD vs GPU central differences with h = 1e-4
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    model.grad(theta, f=f_ad, g=g_ad, info=i_ad)
    torch.cuda.synchronize()
    peak_ad = torch.cuda.max_memory_allocated()
    model.fd_grad(theta, h=1e-4, f=f_fd, g=g_fd, info=i_fd)
    torch.cuda.synchronize()
    gad = g_ad.cpu().numpy()
    gfd = g_fd.cpu().numpy()
    ad_fd_rel = float(np.abs(gad - gfd).max() / np.abs(gad).max())
    ok = int(i_ad.item()) == 0 and bool((i_fd.cpu().numpy() == 0).all())

    use_graph = not args.no_graph
    # the headline gradient: the two-sided split of the block chain (both halves swept at once,
    # then the separator and the tip) when the model has one, else the plain sweep
    split = (not args.no_split) and model.workspace_bytes(1, inla.MODE_GRAD_SPLIT) > 0
    g_sp = torch.empty(d, dtype=torch.float64, device=dev)
    if split:
        model.grad(theta, f=f_ad, g=g_sp, info=i_ad, split=True)
        torch.cuda.synchronize()
        split_rel = float(np.abs(g_sp.cpu().numpy() - gad).max() / np.abs(gad).max())
        ok = ok and int(i_ad.item()) == 0
    plain_step = lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad)  # noqa: E731
    ad_step = ((lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad, split=True))  # noqa: E731
               if split else plain_step)
    fd_step = lambda: model.fd_grad(theta, h=1e-3, max_batch=npts, f=f_fd, g=g_fd, info=i_fd)  # noqa: E731
    fwd_step = lambda: model.forward_saved(theta)  # noqa: E731
    # GEMM tiles: every product on 64 x 64 tiles first, then (unless disabled) the autotuner's
    # choice per role at this block size, timed on the gradient itself; FD is timed with the
    # same table
    inla.clear_tiles()
    tune = None
    if not args.no_autotune:
        ms_ad64 = timed(lambda: model.grad(theta, f=f_ad, g=g_ad, info=i_ad),
                        max(3, args.steps // 2), args.warmup, use_graph, torch)
        t0 = time.perf_counter()
        changed = model.autotune(theta[None], kind="grad", reps=3)
        tune = {"changed": changed, "seconds": time.perf_counter() - t0,
                "tiles": inla.tile_table([model.b])[model.b], "ms_ad_all_64x64": ms_ad64}
    ms_ad = timed(ad_step, args.steps, args.warmup, use_graph, torch)
    ms_ad_plain = (timed(plain_step, max(3, args.steps // 2), 1, use_graph, torch)
                   if split else ms_ad)
    g_ref = g_ad.clone()  # every replay of the full gradient recomputes it
    ms_fd = timed(fd_step, args.steps, args.warmup, use_graph, torch)
    ms_fwd = timed(fwd_step, max(3, args.steps // 2), 1, use_graph, torch)
    f_one = torch.empty(1, dtype=torch.float64, device=dev)
    i_one = torch.empty(1, dtype=torch.int32, device=dev)
    obj_ws = model.new_workspace(1, inla.MODE_OBJECTIVE)
    obj_step = lambda: model.objective(theta[None], out=f_one, info=i_one, ws=obj_ws)  # noqa: E731
    ms_obj_plain = timed(obj_step, max(3, args.steps // 2), 1, use_graph, torch)
    ms_obj = ms_obj_plain
    if split:
        obj_ws2 = model.new_workspace(1, inla.MODE_OBJECTIVE_SPLIT)
        obj_split = lambda: model.objective(theta[None], out=f_one, info=i_one, ws=obj_ws2,  # noqa: E731
                                            split=True)
        ms_obj = timed(obj_split, max(3, args.steps // 2), 1, use_graph, torch)
    ms_bwd = timed_backward(model, theta, f_ad, g_ad, i_ad, max(3, args.steps // 2), 1, use_graph,
                            torch)

    # the carry-only memory mode (factors rebuilt in the backward pass)
    g_c = torch.empty(d, dtype=torch.float64, device=dev)
    ms_carry = timed(lambda: model.grad(theta, f=f_ad, g=g_c, info=i_ad, carry=True),
                     max(3, args.steps // 2), 1, use_graph, torch)
    torch.cuda.synchronize()
    carry_rel = float((g_c - g_ref).abs().max().item() / g_ref.abs().max().item())

    stats, roof = profiled_pass(args, ad_step, bta, torch)
    roof["traffic"] = measured_traffic(roof["kernel_symbol"], args.workload)

    k, nx, ny, nt, a, obs = NAMED_CONFIGS[args.workload]
    b = k * nx * ny
    fwd_fl, si_fl = algorithmic_flops(b, nt, a)
    # FP64-MFMA utilisation of the block Cholesky and the selected inversion: App. B flops of
    # both (both matrices) over the summed kernel time of the kernels that do them (panel
    # steps and panels, every GEMM role, and the sparse W_j product that replaces the dense
    # L_B G), against the 78.6 TFLOP/s peak; rocprof's MFMA counters cross-check it
    fac_si_kernels = ("panel_step", "potrf_panel", "gemm_f64", "w_sparse")
    fac_si_ms = sum(stats[kk]["ms"] for kk in fac_si_kernels if kk in stats) / args.profile_steps
    mfma_pct = 100.0 * (fwd_fl + si_fl) / (fac_si_ms * 1e-3) / (PEAK_FP64_TFLOPS * 1e12)
    hbm_kernels = {}
    for kk in ("w_sparse", "gemv", "assemble", "trace"):
        if kk in stats and stats[kk]["ms"] > 0 and stats[kk]["bytes"] > 0:
            gbs = stats[kk]["bytes"] / (stats[kk]["ms"] * 1e-3) / 1e9
            hbm_kernels[kk] = {"GB/s": gbs, "frac_of_8TB/s": gbs / PEAK_HBM_GBS,
                               "algorithmic_bytes_per_launch":
                                   stats[kk]["bytes"] / max(1, stats[kk]["launches"]),
                               "launches_per_step": stats[kk]["launches"] / args.profile_steps}
    # HBM traffic over the compulsory bytes of the dominant kernel (both per launch)
    gb = roof.get("algorithmic_bytes_per_launch")
    roof["traffic_over_algorithmic_bytes"] = (roof["traffic"] / gb) if (gb and roof.get("traffic")) else None
    line = {
        "metric": METRIC,
        "value": 1000.0 / ms_ad,
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_ad,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "b": b, "n": nt, "a": a, "d": d,
                   "N": nt * b + a, "obs_per_step": obs * k, "seed": args.seed,
                   "graph": use_graph},
        "fd_gradients_per_s": 1000.0 / ms_fd,
        "ms_per_fd_gradient": ms_fd,
        "ad_over_fd_speedup": ms_fd / ms_ad,
        "ms_forward": ms_fwd,
        "ms_backward": ms_bwd,
        "beta_bwd_over_fwd": ms_bwd / ms_fwd,
        # c_AD = T_AD / t_eval, t_eval one objective evaluation on its own (Sec. IV-D), both by
        # the same sweep (split or plain)
        "c_AD": ms_ad / ms_obj,
        "ms_objective": ms_obj,
        "ad_over_batched_fd_point": ms_ad / (ms_fd / npts),
        # the paper's stage split (Sec. IV-I), of the plain sweep: Chol + L-solve of both
        # matrices is the forward sweep; U-solve + selected inversion + traces of both matrices
        # the reverse pass.  Qc and Qp share every launch, so Phase C (the Qp part) is not timed
        # apart: its chain does the same selected-inversion work as Qc's, about half of the
        # reverse pass.
        "stage_split_ms": {"chol_lsolve_both": ms_fwd, "usolve_selinv_traces_both": ms_bwd,
                           "phase_c_share_of_reverse": 0.5},
        "ad_tflops_paper_flop_model": (fwd_fl + si_fl) / (ms_ad * 1e-3) / 1e12,
        "fp64_mfma_pct_factor_selinv": {"pct_of_78.6": mfma_pct,
                                        "app_b_gflop": (fwd_fl + si_fl) / 1e9,
                                        "kernel_ms": fac_si_ms, "kernels": list(fac_si_kernels)},
        "hbm_kernels": hbm_kernels,
        "objectives_per_s_fd_batch": npts * 1000.0 / ms_fd,
        "check": {"ad_vs_gpu_fd_rel_inf_h1e-4": ad_fd_rel, "info_ok": ok},
        "ms_ad_per_call": median_ci(TIMES.get(id(ad_step), [])),
        "split": {"used": split, "separator_block": (nt - 1) // 2 if split else None,
                  "ms_ad_plain_sweep": ms_ad_plain, "ms_objective_plain_sweep": ms_obj_plain,
                  "grad_rel_vs_plain": split_rel if split else None},
        "autotune": tune,
        "ms_fd_per_call": median_ci(TIMES.get(id(fd_step), [])),
        "carry_only": {"ms_per_gradient": ms_carry,
                       "workspace_gb": model.workspace_bytes(1, 2) / 1e9,
                       "stored_factor_workspace_gb": model.workspace_bytes(1, 1) / 1e9,
                       "grad_rel_vs_stored": carry_rel},
        # torch-owned device memory (every workspace; the model's own upload is a few MB)
        "peak_device_memory_gb": {"ad": peak_ad / 1e9,
                                  "with_fd_batch": torch.cuda.max_memory_allocated() / 1e9},
        "kernels": {kname: {"launches_per_step": v["launches"] / args.profile_steps,
                            "ms_per_step": v["ms"] / args.profile_steps,
                            "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None}
                    for kname, v in stats.items()},
        "roofline": roof,
    }
    if not args.no_d15 and args.workload == "uni_32x32_nt50":
        line["d15"] = bench_d15(args, torch, np)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.seed, args.cpu_sample_nt)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

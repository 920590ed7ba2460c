#!/usr/bin/env python3
"""Benchmark of the Faster Mean Shift hot path on one MI355X.

A step is one whole ms_fit (Algorithm 2: seed draws, batched iterations with
early stopping, merge, pool coverage, seed-count control, labelling) on the
200,000-point, 3-D, 50-blob anisotropic Gaussian mixture with h = 15
(synthetic stand-in for the paper's 200K-point simulation, Section III),
with X already resident in HBM.

Printed (one JSON line):
  value            pair evaluations per second over the whole step
                   (sum over iterations of active seeds x n, divided by the
                   measured step time);
  time_to_cluster  the step time itself;
  roofline         the fused step kernel at its largest launch of the
                   workload (512 seeds x 200,000 points), timed with HIP
                   events on the stream the library launches on;
  cpu_baseline     the FP64 oracle on the host's cores, on the same fit.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VEC_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS_MD = os.path.join(ROOT, "profiles", "counters_fused_step_aniso3d_512x200000.md")


def source_digest():
    """Digest of the HIP sources, recorded next to the counter figures so that
    stale figures are never reported."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2112_13891_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_figures(prec):
    """HBM bytes per fused-step iteration (step + reduction and finalize) at the
    512 x 200,000 launch, from the committed FETCH_SIZE / WRITE_SIZE summary
    (scaled by a copy kernel of known size), and the MFMA flops the step
    kernel executed (K padded to 16); both None when the sources changed since
    the counters were taken."""
    try:
        text = open(COUNTERS_MD).read()
    except OSError:
        return None, None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != source_digest():
        return None, None
    tb = vals.get(f"{prec}_traffic_bytes_per_iteration")
    mb = vals.get(f"{prec}_mfma_flops_per_iteration")
    return (float(tb) if tb else None), (float(mb) if mb else None)


def flops_per_pair(d):
    # distance 2D+3, weight 2 (+1 exp, not counted), accumulate 2D+1
    return 4 * d + 6


def algorithmic_bytes(prec, m, n):
    """Bytes one iteration must move at m seeds x n points, D = 3, with every
    block live: the points once per 64-seed tile (16 B per point; the BF16 form
    also reads its 64 B of per-point operands), plus each seed's partial sums
    once written and once read (16 B per seed and point chunk of at least two
    256-point blocks).  Culled blocks are not read, so the measured traffic can
    be lower."""
    tiles = -(-m // 64)
    cmax = -(-n // 512)
    grid = min(2048, tiles * cmax)
    chunks = min(max(1, grid // tiles), cmax) if tiles < grid else 1
    per_point = 16 + 64 if prec == "bf16" else 16
    return tiles * n * per_point + 2 * m * chunks * 16


def time_kernel(api, torch, X, seeds, h, kernel, precision, iters, plain=False):
    """Average duration of one fused-step iteration with every seed active:
    (t(2k iterations) - t(k)) / k, HIP events on the library's stream, so that
    the call's set-up (packing, sorting, workspace) cancels out.  A few
    milliseconds of fill kernels are queued ahead of each timed call, so the
    host has enqueued the whole call before the GPU reaches it and the events
    see GPU time only (a slow host, e.g. under a tracer, cannot hide the first
    iterations behind its own set-up)."""
    pad = torch.empty(1 << 28, dtype=torch.float32, device=X.device)

    def run(k):
        st = torch.cuda.current_stream()
        for _ in range(16):
            pad.fill_(0.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        api.step(X, seeds, h, kernel=kernel, precision=precision, tol=1e-30, n_iter=k, plain=plain)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    run(iters)  # warm
    base = min(run(iters) for _ in range(3))
    full = min(run(2 * iters) for _ in range(3))
    del pad
    return (full - base) / iters


def other_configs(api, torch, workloads):
    """Secondary workloads of the method, each timed briefly: the 2-D blob fit,
    the 32-D embedding fit (Gaussian, both precisions), 512 uneven clouds in one
    batched step, and the differentiable form
    (64 clouds x 16,384 points x 16, T = 10 unrolled steps, forward + adjoint)."""
    import numpy as np
    from paper_2112_13891_amd.autograd import MeanShiftT
    out = {}

    def fit_rate(w, steps, **kw):
        X = torch.from_numpy(w.X).cuda()
        api.fit(X, w.h, kernel=w.kernel, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = api.fit(X, w.h, kernel=w.kernel, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        return {"time_to_cluster_ms": dt * 1e3, "pair_evals_per_s": r.pairs / dt, "K": r.k,
                "rounds": [int(b) for b in r.round_B], "pairs_per_fit": r.pairs}

    w = workloads.blobs2d(seed=0)
    out["blobs2d_fp32"] = fit_rate(w, 10)
    out["blobs2d_fp32"]["workload"] = "blobs2d: 2,000 points, D=2, 5 blobs, Gaussian h=5, pool seeding"
    out["blobs2d_bf16"] = fit_rate(w, 10, precision="bf16")
    w = workloads.embed32(seed=0)
    out["embed32_gaussian_fp32"] = fit_rate(w, 2)
    out["embed32_gaussian_fp32"]["workload"] = ("embed32: 262,144 points, D=32, 100 clusters + 5% "
                                                "outliers, Gaussian h=1.5, pool seeding")
    out["embed32_gaussian_bf16"] = fit_rate(w, 2, precision="bf16")
    out["embed32_gaussian_bf16"]["speedup_vs_fp32"] = (
        out["embed32_gaussian_fp32"]["time_to_cluster_ms"] / out["embed32_gaussian_bf16"]["time_to_cluster_ms"])
    # the flat window on the same embeddings: no two points share a window, so
    # every point founds its own mode (K = n) and merge and labels are n^2
    # problems; a throughput case (one fit per precision after one warm-up)
    w = workloads.embed32(seed=0, kernel="flat")
    for prec in ("fp32", "bf16"):
        r = fit_rate(w, 1, precision=prec)
        out[f"embed32_flat_{prec}"] = r
    out["embed32_flat_fp32"]["workload"] = ("embed32: 262,144 points, D=32, 100 clusters + 5% outliers, "
                                            "flat h=1.5 (every window a singleton: K = n)")
    # cosine metric on 32-D embeddings (unit directions, chord bandwidth 0.3)
    w = workloads.embed_cos(seed=0)
    for prec in ("fp32", "bf16"):
        out[f"embed32_cosine_{prec}"] = fit_rate(w, 2, precision=prec, metric="cosine")
    out["embed32_cosine_fp32"]["workload"] = ("embed_cos: 262,144 rows, D=32, 100 directions (angular "
                                              "spread 0.2) + 5% uniform directions, cosine metric, "
                                              "Gaussian chord h=0.3")
    # RGB images (the segmentation shape of Section I): 512^2 and 1024^2 pixels
    for side in (512, 1024):
        w = workloads.image_rgb(seed=0, side=side)
        for prec in ("fp32", "bf16"):
            key = f"image_rgb{side}_{prec}"
            out[key] = fit_rate(w, 5, precision=prec)
            if prec == "fp32":
                out[key]["workload"] = (f"image_rgb: {side}x{side} RGB pixels ({side * side:,} points, "
                                        "D=3), 24 Voronoi colour regions + N(0, 6^2) noise, Gaussian h=12")
    # frame sequence with seed-count adaptation (Section II-D): 6 frames
    frames = workloads.frames2d(seed=0, n=200_000)
    Xf = [torch.from_numpy(f.X).cuda() for f in frames]
    for prec in ("fp32", "bf16"):
        api.fit_sequence(Xf, 5.0, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, starts = api.fit_sequence(Xf, 5.0, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"frames2d_sequence_{prec}"] = {
            "ms_per_frame": dt / len(Xf) * 1e3, "start_N": starts,
            "rounds_per_frame": [len(r.round_N) for r in res], "K": [r.k for r in res]}
    out["frames2d_sequence_fp32"]["workload"] = (
        "frames2d: 6 frames x 200,000 points, D=2, 40 drifting blobs then 4 from frame 3, Gaussian h=5, "
        "each frame warm-started from the previous seed count (H=32)")
    # many uneven clouds in one batched call (FP32): 512 clouds of 1,000..65,536
    # points, D = 16, up to 256 seeds each, 10 iterations with every seed active
    clouds = workloads.clouds16(seed=0)
    Xs = [c[0] for c in clouds]
    rng = np.random.default_rng(0)
    Ss = [X[rng.choice(len(X), min(len(X), 256), replace=False)] for X in Xs]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    Xa = torch.from_numpy(np.concatenate(Xs)).cuda()
    Sa = torch.from_numpy(np.concatenate(Ss)).cuda()
    pairs = sum(len(s) * len(x) for s, x in zip(Ss, Xs))

    def batched(k, graph=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=k, graph=graph)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    batched(2)
    batched(2, True)
    t_it = (min(batched(20) for _ in range(2)) - min(batched(10) for _ in range(2))) / 10
    t_itg = (min(batched(20, True) for _ in range(2)) - min(batched(10, True) for _ in range(2))) / 10
    Xc = [torch.from_numpy(x).cuda() for x in Xs]
    Sc = [torch.from_numpy(s).cuda() for s in Ss]

    def per_cloud(k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for x, s_ in zip(Xc, Sc):
            api.step(x, s_, 1.0, tol=1e-30, n_iter=k)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    per_cloud(1)
    t_pc = (per_cloud(4) - per_cloud(2)) / 2
    out["clouds16_batched_fp32"] = {
        "workload": "512 clouds, sizes log-uniform in [1000, 65536] (%d points), D=16, 2..40 "
                    "clusters each, Gaussian h=1, min(n, 256) seeds per cloud" % int(xo[-1]),
        "ms_per_iteration": t_it * 1e3, "ms_per_iteration_graph": t_itg * 1e3,
        "pair_evals_per_iteration": pairs, "pair_evals_per_s": pairs / t_it,
        "per_cloud_calls_ms_per_iteration": t_pc * 1e3,
        "speedup_vs_per_cloud_calls": t_pc / t_it}
    # the whole method on the 512 clouds in one call, beside one ms_fit per cloud
    def fit_all():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per, lab, k_off, rounds = api.fit_batched(Xa, xo, 1.0)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, k_off, rounds

    fit_all()
    t_fb, k_off, rounds = min((fit_all() for _ in range(2)), key=lambda r: r[0])
    Xc = [torch.from_numpy(x).cuda() for x in Xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, x in enumerate(Xc):
        api.fit(x, 1.0, rng_seed=c)
    torch.cuda.synchronize()
    t_pf = time.perf_counter() - t0
    out["clouds16_fit_batched_fp32"] = {
        "workload": "the 512 clouds above, whole method per cloud (pool seeding N0=128, L=8, merge/cover "
                    "radius h, labels) in one ms_fit_batched call",
        "ms_per_call": t_fb * 1e3, "rounds": rounds, "modes_total": int(k_off[-1]),
        "per_cloud_fit_calls_ms": t_pf * 1e3, "speedup_vs_per_cloud_fits": t_pf / t_fb}
    # many small clouds, where the launches rather than the arithmetic set the
    # pace: whole-call time of 30 iterations launched eagerly and as one graph
    rng = np.random.default_rng(1)
    Xs = [workloads.cloud16(rng, int(n), 2)[0] for n in rng.integers(200, 2000, 256)]
    Ss = [X[rng.choice(len(X), 32, replace=False)] for X in Xs]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    Xa = torch.from_numpy(np.concatenate(Xs)).cuda()
    Sa = torch.from_numpy(np.concatenate(Ss)).cuda()
    batched(2)
    batched(2, True)
    t_e = min(batched(30) for _ in range(5))
    t_g = min(batched(30, True) for _ in range(5))
    best_R, ms_R = api.tune_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, trials=8)
    t_t = min(batched(30) for _ in range(5))   # the tuned shape from here on
    out["small_clouds2_batched_fp32"] = {
        "workload": "256 clouds of 200..2000 points (%d points), D=2, 32 seeds each, Gaussian h=1, "
                    "30 iterations per call" % int(xo[-1]),
        "ms_per_call_eager": t_e * 1e3, "ms_per_call_graph": t_g * 1e3,
        "graph_speedup": t_e / t_g, "tuned_R": best_R,
        "tuner_ms_per_iteration_by_R": {str(r): v for r, v in ms_R.items()},
        "ms_per_call_tuned": t_t * 1e3}

    # differentiable form
    clouds = workloads.diffclouds(seed=0)
    X = torch.from_numpy(np.stack([c[0] for c in clouds])).cuda()
    C = torch.from_numpy(np.stack([c[2][c[1]] for c in clouds]).astype(np.float32)).cuda()

    def fwd_bwd():
        Xr = X.detach().requires_grad_(True)
        S = MeanShiftT.apply(Xr, 1.0, 10)
        loss = ((S - C) ** 2).sum()
        loss.backward()
        return Xr.grad

    fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 2
    for _ in range(steps):
        fwd_bwd()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    B, n, d = X.shape
    fwd_pairs = B * n * n * 10
    out["diffclouds_fp32"] = {"workload": "64 clouds x 16,384 points, D=16, T=10 Gaussian steps, h=1, "
                                          "loss vs generating centres; forward + adjoint",
                              "ms_per_step": dt * 1e3, "forward_pair_evals_per_step": fwd_pairs,
                              "forward_pair_evals_per_s_over_step": fwd_pairs / dt}
    return out


def cpu_baseline(w, args):
    import oracle
    oracle.lib()
    th = oracle.threads()
    t0 = time.perf_counter()
    r = oracle.fit(w.X, w.h, kernel=w.kernel)
    dt = time.perf_counter() - t0
    return {"value": r.pairs / dt, "unit": "pair evals/s", "cores": th, "kind": "oracle",
            "sample": f"one whole FP64 fit of the same workload ({len(r.round_B)} rounds, "
                      f"{r.pairs:.3e} pairs, K={r.k}) in {dt:.2f} s",
            "time_to_cluster_ms": dt * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"],
                    help="precision of the headline value; the other form is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the secondary workloads (2-D blobs, 32-D embedding, adjoint)")
    ap.add_argument("--kernel-iters", type=int, default=20)
    ap.add_argument("--phase", default="all", choices=["all", "kernel", "fit", "batched"],
                    help="kernel: only the dominant-kernel launch shape (both precisions) and a "
                         "256 MiB copy that calibrates the traffic counters; fit: only --steps "
                         "fits per precision; batched: only --steps whole-method calls on the "
                         "512 uneven clouds (D = 16); all for profilers")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2112_13891_amd import api, workloads

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    api.lib()
    if args.phase == "batched":
        clouds = workloads.clouds16(seed=0)
        xo = np.concatenate([[0], np.cumsum([len(c[0]) for c in clouds])]).astype(np.int64)
        Xa = torch.from_numpy(np.concatenate([c[0] for c in clouds])).cuda()
        log(f"workload clouds16: {len(clouds)} clouds, {int(xo[-1])} points, D=16")
        for _ in range(args.warmup):
            api.fit_batched(Xa, xo, 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, k_off, rounds = api.fit_batched(Xa, xo, 1.0)
        torch.cuda.synchronize()
        print(json.dumps({"phase": "batched", "ms_per_call": (time.perf_counter() - t0) / args.steps * 1e3,
                          "rounds": rounds, "modes_total": int(k_off[-1])}), flush=True)
        return
    w = workloads.aniso3d(seed=0)
    X = torch.from_numpy(w.X).cuda()
    n, d = w.X.shape
    log(f"workload aniso3d n={n} d={d} h={w.h} kernel={w.kernel}")

    if args.phase == "kernel":
        # the largest launch of the fit: 512 seeds (third round) x all points
        rng = np.random.default_rng(0)
        seeds = torch.from_numpy(w.X[rng.choice(n, 512, replace=False)]).cuda()
        out = {"phase": "kernel", "launch": f"512 seeds x {n} points"}
        for prec in ("fp32", "bf16"):
            t = time_kernel(api, torch, X, seeds, w.h, w.kernel, prec, args.kernel_iters)
            out[prec + "_iteration_ms"] = t
            out[prec + "_pair_evals_per_s"] = 512 * n / (t * 1e-3)
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)   # 256 MiB read + 256 MiB written per launch
        torch.cuda.synchronize()
        out["copy_bytes_each_way"] = src.numel() * 4
        print(json.dumps(out), flush=True)
        return

    def one(prec, plain=False):
        return api.fit(X, w.h, kernel=w.kernel, precision=prec, plain=plain)

    if args.phase == "fit":
        out = {"phase": "fit"}
        for prec in ("fp32", "bf16"):
            for _ in range(args.warmup):
                one(prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                r = one(prec)
            torch.cuda.synchronize()
            out[prec + "_ms_per_fit"] = (time.perf_counter() - t0) / args.steps * 1e3
            out[prec + "_breakdown_ms"] = {"iterate": r.iterate_ms, "merge_and_pool": r.merge_ms,
                                           "assign": r.assign_ms, "host_total": r.total_ms}
        print(json.dumps(out), flush=True)
        return

    results = {}
    for prec in ["fp32", "bf16"]:
        for _ in range(args.warmup):
            one(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for _ in range(args.steps):
            last = one(prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        results[prec] = (dt, last)
        log(f"{prec}: {dt / args.steps * 1e3:.3f} ms/fit, K={last.k}, pairs={last.pairs}, "
            f"iterate_ms={last.iterate_ms:.3f} merge_ms={last.merge_ms:.3f} "
            f"assign_ms={last.assign_ms:.3f} total_ms={last.total_ms:.3f}")

    # the plain FP32 form (every pair, input order) for comparison
    for _ in range(args.warmup):
        one("fp32", plain=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plast = one("fp32", plain=True)
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    log(f"plain fp32: {plain_dt / args.steps * 1e3:.3f} ms/fit, K={plast.k}")

    dt, last = results[args.precision]
    ms_per_step = dt / args.steps * 1e3
    value = last.pairs * args.steps / dt

    # dominant kernel: the fused step at the workload's largest launch
    rng = np.random.default_rng(0)
    m = int(max(last.round_B)) if last.rounds else 512
    seeds = torch.from_numpy(w.X[rng.choice(n, m, replace=False)]).cuda()
    t_it = time_kernel(api, torch, X, seeds, w.h, w.kernel, args.precision, args.kernel_iters)
    pairs = m * n
    achieved_tflops = pairs * flops_per_pair(d) / (t_it * 1e-3) / 1e12
    traffic, mfma_flops = counter_figures(args.precision)
    step_name = "step_bf16_kernel" if args.precision == "bf16" else "step_cull_kernel"
    roof = {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VEC_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VEC_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": f"one fused-step iteration: {step_name} + finalize_fused_kernel "
                      "(chunk reduction and finalize in one launch)",
            "launch": f"{m} seeds x {n} points", "avg_ms": t_it,
            "flops_per_pair": flops_per_pair(d),
            "algorithmic_bytes": algorithmic_bytes(args.precision, m, n),
            "pair_evals_per_s": pairs / (t_it * 1e-3)}
    if mfma_flops:
        # matrix cores: executed (padded) bf16 MFMA work against the dense bf16 peak
        roof["mfma_tflops_executed"] = mfma_flops / (t_it * 1e-3) / 1e12
        roof["mfma_frac_of_bf16_peak"] = roof["mfma_tflops_executed"] / BF16_MFMA_PEAK_TFLOPS
    log(f"kernel: {t_it * 1e3:.1f} us/iteration at {m}x{n}: {pairs / (t_it * 1e-3):.3e} pairs/s, "
        f"{achieved_tflops:.2f} TFLOP/s")

    # throughput stress: every point a seed (Algorithm 1 shape), one iteration
    t_all = time_kernel(api, torch, X, X, w.h, w.kernel, args.precision, 2)
    stress = n * n / (t_all * 1e-3)
    log(f"all-seeds iteration: {t_all:.2f} ms -> {stress:.3e} pairs/s")

    out = {
        "metric": "seed-point pair evals/s + time-to-cluster 200K pts, BF16-refined vs FP32",
        "value": value,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16 products, f32 refine/accumulate",
        "data": "synthetic",
        "config": {"workload": "aniso3d: 200,000 points, D=3, 50 anisotropic Gaussian blobs "
                               "(centres U[0,1000]^3, per-axis sigma U[3,8], Dirichlet(2) weights), "
                               "Gaussian kernel h=15, pool seeding N0=128, L=8, tol=1e-3, "
                               "max_iter=100, merge/cover radius h",
                   "n": n, "d": d, "precision": args.precision, "K": last.k,
                   "rounds": [int(b) for b in last.round_B], "pairs_per_fit": last.pairs},
        "time_to_cluster_ms": ms_per_step,
        "breakdown_ms": {"iterate": last.iterate_ms, "merge_and_pool": last.merge_ms,
                         "assign": last.assign_ms, "host_total": last.total_ms},
        "kernel_pair_evals_per_s": pairs / (t_it * 1e-3),
        "all_seeds_iteration_pair_evals_per_s": stress,
        "roofline": roof,
    }
    other = "fp32" if args.precision == "bf16" else "bf16"
    odt, olast = results[other]
    out[f"{other}_time_to_cluster_ms"] = odt / args.steps * 1e3
    out[f"{other}_pair_evals_per_s"] = olast.pairs * args.steps / odt
    if args.precision == "bf16":
        out["bf16_refined_pair_fraction"] = last.refined_pairs / max(1, last.pairs)
        out["speedup_time_to_cluster_vs_fp32"] = odt / dt
    t_other = time_kernel(api, torch, X, seeds, w.h, w.kernel, other, args.kernel_iters)
    out[f"{other}_kernel_pair_evals_per_s"] = pairs / (t_other * 1e-3)
    out["kernel_speedup_vs_" + other] = t_other / t_it
    log(f"{other} kernel: {t_other * 1e3:.1f} us/iteration -> {pairs / (t_other * 1e-3):.3e} pairs/s")
    t_plain = time_kernel(api, torch, X, seeds, w.h, w.kernel, "fp32", args.kernel_iters, plain=True)
    out["plain_fp32_time_to_cluster_ms"] = plain_dt / args.steps * 1e3
    out["plain_fp32_K"] = plast.k
    out["speedup_time_to_cluster_vs_plain_fp32"] = plain_dt / dt
    out["plain_fp32_kernel_pair_evals_per_s"] = pairs / (t_plain * 1e-3)
    out["kernel_speedup_vs_plain_fp32"] = t_plain / t_it
    log(f"plain fp32 kernel: {t_plain * 1e3:.1f} us/iteration")
    if not args.no_other_configs:
        out["other_configs"] = other_configs(api, torch, workloads)
        log("other configs:", json.dumps(out["other_configs"]))
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, args)
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']:.3e} pairs/s on {cb['cores']} threads")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Faster Mean Shift hot path on one MI355X.

A step is one whole ms_fit (Algorithm 2: seed draws, batched iterations with
early stopping, merge, pool coverage, seed-count control, labelling) on the
200,000-point, 3-D, 50-blob anisotropic Gaussian mixture with h = 15
(synthetic stand-in for the paper's 200K-point simulation, Section III),
with X already resident in HBM.

Printed (one JSON line):
  value            pair evaluations per second over the whole step, counted
                   as the method defines them: every active seed against all
                   n points at every iteration (Section II-B), divided by the
                   measured step time; the pairs the kernels actually
                   evaluated (culled blocks skipped) are reported beside it;
  time_to_cluster  the step time itself;
  roofline         the fused step (step kernel and its reduction/finalize
                   launch) at the workload's largest launch (512 seeds x
                   200,000 points), timed with HIP events on the stream the
                   library launches on;
  configs          the same figures for every workload of the method: the
                   2-D blobs, the 200K mixture, the 32-D embedding mixture
                   (largest launch 8,192 seeds x 262,144 points), the 512
                   uneven clouds and the differentiable form;
  cpu_baseline     the FP64 oracle on the host's cores (all threads and one),
                   medians of three runs, with each workload's error against
                   that oracle.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VEC_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "embed32_gauss_fit.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _plain(o):
    """JSON form of numpy scalars and arrays."""
    if hasattr(o, "tolist"):
        return o.tolist()
    raise TypeError(f"not JSON serializable: {type(o).__name__}")


COUNTERS = {
    "c2": os.path.join(ROOT, "profiles", "counters_fused_step_aniso3d_512x200000.md"),
    "c3": os.path.join(ROOT, "profiles", "counters_fused_step_embed32_8192x262144.md"),
}


# The sources each counted launch runs (its step kernels, their reduction and
# finalize, and the spatial order that decides which blocks they skip).
COUNTER_SOURCES = {
    "c2": ["k_step.hip", "k_step_cull.hip", "k_step_bf16.hip", "k_sort.hip", "step_common.h"],
    "c3": ["k_step_cull.hip", "k_step_bf16f.hip", "k_sort.hip", "step_common.h"],
}


def source_digest(which):
    """Digest of the HIP sources of one counted launch, recorded next to its
    counter figures so that stale figures are never reported."""
    h = hashlib.sha256()
    for f in COUNTER_SOURCES[which]:
        with open(os.path.join(ROOT, "paper_2112_13891_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_figures(which, prec):
    """Figures of one fused-step iteration read from a committed counter
    summary ("- key: value" lines): HBM bytes (FETCH_SIZE and WRITE_SIZE,
    scaled by a copy kernel of known size), the executed MFMA flops and the
    fraction of pairs the kernels evaluated.  Empty when the launch's HIP
    sources changed since the counters were taken."""
    try:
        text = open(COUNTERS[which]).read()
    except OSError:
        return {}
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != source_digest(which):
        return {}
    out = {}
    for key in ("traffic_bytes_per_iteration", "mfma_flops_per_iteration", "evaluated_pair_fraction"):
        v = vals.get(f"{prec}_{key}")
        if v not in (None, "", "None"):
            out[key] = float(v)
    return out


def flops_per_pair(d):
    # distance 2D+3, weight 2 (+1 exp, not counted), accumulate 2D+1
    return 4 * d + 6


def contraction_flops_per_pair(d):
    # the contraction-shaped part: products of the distance and the accumulation
    return 4 * d + 2


def adjoint_flops_per_pair(d):
    """One unrolled step of the differentiable form, forward and adjoint, per
    seed-point pair: the forward update (4D+6), then the adjoint's recomputed
    forward (4D+6), its dS pass (weight 2D+5, g.(x - s') 2D, beta 3,
    beta (x - s) 2D) and its dX pass (weight 2D+5, g.(x - s') 2D, beta 3,
    (w/W) g + beta (s - x) 4D)."""
    return (4 * d + 6) + (4 * d + 6) + (6 * d + 8) + (8 * d + 8)


def algorithmic_bytes(m, n, d, tile=64):
    """Bytes one iteration must stream at m active seeds x n points: every
    seed tile of `tile` seeds reads the n x d points once, 4 bytes per
    coordinate (FP32, or the hi and lo bf16 planes of the BF16 form)."""
    tiles = -(-m // tile)
    return tiles * n * d * 4


def roofline_entry(pairs, d, t_ms, m, n, prec, launch, kernel, counters=None):
    """Algorithmic flops over the measured iteration against the FP32 vector
    peak (the path is bound by plain ALU arithmetic); for the BF16 form also
    the contraction flops against the dense bf16 MFMA peak."""
    t = t_ms * 1e-3
    tf = pairs * flops_per_pair(d) / t / 1e12
    ab = algorithmic_bytes(m, n, d, 128 if (prec == "bf16" and d > 4) else 64)
    e = {"bound": "alu", "achieved": tf, "peak": FP32_VEC_PEAK_TFLOPS, "unit": "TFLOP/s",
         "frac": tf / FP32_VEC_PEAK_TFLOPS, "kernel": kernel, "launch": launch, "avg_ms": t_ms,
         "flops_per_pair": flops_per_pair(d), "algorithmic_pair_evals_per_s": pairs / t,
         "algorithmic_bytes": ab, "algorithmic_hbm_frac": ab / t / 1e9 / HBM_PEAK_GBS}
    if prec == "bf16":
        ctf = pairs * contraction_flops_per_pair(d) / t / 1e12
        e["contraction_tflops_on_mfma_form"] = ctf
        e["contraction_frac_of_bf16_mfma_peak"] = ctf / BF16_MFMA_PEAK_TFLOPS
    c = counters or {}
    e["traffic"] = c.get("traffic_bytes_per_iteration")
    if c.get("mfma_flops_per_iteration"):
        e["mfma_tflops_executed"] = c["mfma_flops_per_iteration"] / t / 1e12
        e["mfma_executed_frac_of_bf16_peak"] = e["mfma_tflops_executed"] / BF16_MFMA_PEAK_TFLOPS
    if c.get("evaluated_pair_fraction") is not None:
        e["evaluated_pair_fraction"] = c["evaluated_pair_fraction"]
        e["evaluated_pair_evals_per_s"] = pairs * c["evaluated_pair_fraction"] / t
    return e


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


def fit_timing(api, torch, X, h, kernel, steps, **kw):
    """Seconds per whole fit (after one warm-up) and the last result."""
    api.fit(X, h, kernel=kernel, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = None
    for _ in range(steps):
        r = api.fit(X, h, kernel=kernel, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, r


def fit_summary(dt, r):
    return {"time_to_cluster_ms": dt * 1e3, "pair_evals_per_s": r.pairs / dt, "K": r.k,
            "rounds": [int(b) for b in r.round_B], "pairs_per_fit": r.pairs,
            "exact_pair_fraction": r.refined_pairs / max(1, r.pairs)}


def config_c1(api, torch, workloads, gpu_fits):
    w = workloads.blobs2d(seed=0)
    X = torch.from_numpy(w.X).cuda()
    out = {"workload": "blobs2d: 2,000 points, D=2, 5 isotropic blobs (centres U[0,100]^2, sigma 2), "
                       "Gaussian h=5, pool seeding N0=128, L=8"}
    for prec in ("fp32", "bf16"):
        dt, r = fit_timing(api, torch, X, w.h, w.kernel, 20, precision=prec)
        gpu_fits[("c1", prec)] = r
        s = fit_summary(dt, r)
        s["roofline"] = roofline_entry(r.pairs, w.d, dt * 1e3, max(r.round_B), w.n, prec,
                                       "whole fit", "whole fit (latency-bound: a few launches of "
                                       "microseconds each, every kernel far from its roofline)")
        out[prec] = s
    return out


def config_c3(api, torch, workloads, gpu_fits, iters):
    import numpy as np
    w = workloads.embed32(seed=0)
    X = torch.from_numpy(w.X).cuda()
    out = {"workload": "embed32: 262,144 points, D=32, 100 Gaussian clusters (centres N(0,16 I), sigma 0.5) "
                       "+ 5% uniform outliers in [-12,12]^32, Gaussian h=1.5, pool seeding"}
    for prec in ("fp32", "bf16"):
        dt, r = fit_timing(api, torch, X, w.h, w.kernel, 3, precision=prec)
        gpu_fits[("c3", prec)] = r
        out[prec] = fit_summary(dt, r)
    out["bf16_speedup_time_to_cluster_vs_fp32"] = (out["fp32"]["time_to_cluster_ms"]
                                                   / out["bf16"]["time_to_cluster_ms"])
    # the fit's largest launch: 8,192 seeds over all points
    m = 8192
    rng = np.random.default_rng(8192)
    seeds = torch.from_numpy(w.X[rng.choice(w.n, m, replace=False)]).cuda()
    for prec in ("fp32", "bf16"):
        t = time_kernel(api, torch, X, seeds, w.h, w.kernel, prec, iters)
        name = ("step_cull_kernel<32, 1, 1> + reduce_kernel + finalize_kernel" if prec == "fp32"
                else "step_bf16f_kernel<32, false> + reduce_kernel + finalize_kernel")
        out[prec]["roofline"] = roofline_entry(m * w.n, w.d, t, m, w.n, prec, f"{m} seeds x {w.n} points",
                                               name, counter_figures("c3", prec))
    out["bf16_kernel_speedup_vs_fp32"] = out["fp32"]["roofline"]["avg_ms"] / out["bf16"]["roofline"]["avg_ms"]
    log(f"c3: fp32 {out['fp32']['time_to_cluster_ms']:.2f} ms, bf16 {out['bf16']['time_to_cluster_ms']:.2f} ms; "
        f"8192-seed iteration fp32 {out['fp32']['roofline']['avg_ms']:.3f} ms, "
        f"bf16 {out['bf16']['roofline']['avg_ms']:.3f} ms")
    return out


def config_c4(api, torch, workloads, gpu_fits):
    import numpy as np
    clouds = workloads.clouds16(seed=0)
    Xs = [c[0] for c in clouds]
    rng = np.random.default_rng(0)
    Ss = [X[rng.choice(len(X), min(len(X), 256), replace=False)] for X in Xs]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    Xa = torch.from_numpy(np.concatenate(Xs)).cuda()
    Sa = torch.from_numpy(np.concatenate(Ss)).cuda()
    pairs = sum(len(s) * len(x) for s, x in zip(Ss, Xs))

    def batched(k, graph=False, precision="fp32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=k, graph=graph, precision=precision)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def per_iteration(graph=False, precision="fp32"):
        # the difference of 20 and 10 iterations: a call's set-up (the BF16
        # form's per-cloud sort and block features) cancels
        batched(2, graph, precision)
        return (min(batched(20, graph, precision) for _ in range(2))
                - min(batched(10, graph, precision) for _ in range(2))) / 10

    t_it = per_iteration()
    t_itg = per_iteration(graph=True)
    t_bf = per_iteration(precision="bf16")
    t_bfg = per_iteration(graph=True, precision="bf16")
    t_bf_setup = min(batched(1, precision="bf16") for _ in range(2)) - t_bf
    S32 = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=5)[0]
    S16 = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=5, precision="bf16")[0]
    torch.cuda.synchronize()
    bf_diff = float((S32 - S16).abs().max())
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
    out = {"workload": "512 clouds, sizes log-uniform in [1000, 65536] (%d points), D=16, 2..40 clusters "
                       "each, Gaussian h=1, min(n, 256) seeds per cloud" % int(xo[-1]),
           "ms_per_iteration": t_it * 1e3, "ms_per_iteration_graph": t_itg * 1e3,
           "pair_evals_per_iteration": pairs, "pair_evals_per_s": pairs / t_it,
           "per_cloud_calls_ms_per_iteration": t_pc * 1e3, "speedup_vs_per_cloud_calls": t_pc / t_it,
           "bf16": {"ms_per_iteration": t_bf * 1e3, "ms_per_iteration_graph": t_bfg * 1e3,
                    "pair_evals_per_s": pairs / t_bf, "speedup_vs_fp32": t_it / t_bf,
                    "call_setup_ms": t_bf_setup * 1e3,
                    "max_seed_difference_to_fp32_after_5_iterations_over_h": bf_diff}}
    e = roofline_entry(pairs, 16, t_it * 1e3, 0, 0, "fp32", "one batched iteration, every seed active",
                       "bstep_kernel<16, 16, 1> + bfinal_kernel + bplan_kernel")
    e["algorithmic_bytes"] = sum(-(-len(s) // 64) * len(x) * 16 * 4 for s, x in zip(Ss, Xs))
    e["algorithmic_hbm_frac"] = e["algorithmic_bytes"] / t_it / 1e9 / HBM_PEAK_GBS
    out["roofline"] = e

    def fit_all(precision="fp32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per, lab, k_off, rounds = api.fit_batched(Xa, xo, 1.0, precision=precision)
        torch.cuda.synchronize()
        gpu_fits[("c4", precision)] = (per, lab, k_off, xo, Xs)
        return time.perf_counter() - t0, k_off, rounds

    fit_all()
    t_fb, k_off, rounds = min((fit_all() for _ in range(3)), key=lambda r: r[0])
    fit_all("bf16")
    t_fb16, k_off16, rounds16 = min((fit_all("bf16") for _ in range(3)), key=lambda r: r[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, x in enumerate(Xc):
        api.fit(x, 1.0, rng_seed=c)
    torch.cuda.synchronize()
    t_pf = time.perf_counter() - t0
    out["fit_batched"] = {"ms_per_call": t_fb * 1e3, "rounds": rounds, "modes_total": int(k_off[-1]),
                          "per_cloud_fit_calls_ms": t_pf * 1e3, "speedup_vs_per_cloud_fits": t_pf / t_fb,
                          "bf16": {"ms_per_call": t_fb16 * 1e3, "rounds": rounds16,
                                   "modes_total": int(k_off16[-1]),
                                   "clouds_with_fp32_mode_count": int((np.diff(k_off16) == np.diff(k_off)).sum()),
                                   "speedup_vs_fp32": t_fb / t_fb16}}
    return out


def config_c5(api, torch, workloads):
    import numpy as np
    from paper_2112_13891_amd.autograd import MeanShiftT
    clouds = workloads.diffclouds(seed=0)
    X = torch.from_numpy(np.stack([c[0] for c in clouds])).cuda()
    C = torch.from_numpy(np.stack([c[2][c[1]] for c in clouds]).astype(np.float32)).cuda()

    def fwd_bwd():
        Xr = X.detach().requires_grad_(True)
        S = MeanShiftT.apply(Xr, 1.0, 10)
        ((S - C) ** 2).sum().backward()
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
    pairs = B * n * n * 10
    tf = pairs * adjoint_flops_per_pair(d) / dt / 1e12
    return {"workload": "64 clouds x 16,384 points, D=16, T=10 Gaussian steps, h=1, loss vs generating "
                        "centres; forward + adjoint with recompute",
            "ms_per_step": dt * 1e3, "forward_pair_evals_per_step": pairs,
            "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_VEC_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / FP32_VEC_PEAK_TFLOPS, "flops_per_pair": adjoint_flops_per_pair(d),
                         "kernel": "10 forward updates + 10 adjoint steps (fwd_partial, ds_partial, "
                                   "dx_partial and their reductions)", "avg_ms": dt * 1e3}}


def other_configs(api, torch, workloads):
    """Further shapes of the method, timed briefly: the flat window and the
    cosine metric on the 32-D embeddings, RGB images, a frame sequence, and
    many small clouds in one batched call (eager, as one graph, tuned)."""
    import numpy as np
    out = {}
    w = workloads.embed32(seed=0, kernel="flat")
    X = torch.from_numpy(w.X).cuda()
    for prec in ("fp32", "bf16"):
        out[f"embed32_flat_{prec}"] = fit_summary(*fit_timing(api, torch, X, w.h, w.kernel, 1, precision=prec))
    out["embed32_flat_fp32"]["workload"] = ("embed32: 262,144 points, D=32, 100 clusters + 5% outliers, "
                                            "flat h=1.5 (every window a singleton: K = n)")
    w = workloads.embed_cos(seed=0)
    X = torch.from_numpy(w.X).cuda()
    for prec in ("fp32", "bf16"):
        out[f"embed32_cosine_{prec}"] = fit_summary(*fit_timing(api, torch, X, w.h, w.kernel, 2, precision=prec,
                                                                metric="cosine"))
    out["embed32_cosine_fp32"]["workload"] = ("embed_cos: 262,144 rows, D=32, 100 directions (angular "
                                              "spread 0.2) + 5% uniform directions, cosine metric, "
                                              "Gaussian chord h=0.3")
    for side in (512, 1024):
        w = workloads.image_rgb(seed=0, side=side)
        X = torch.from_numpy(w.X).cuda()
        for prec in ("fp32", "bf16"):
            key = f"image_rgb{side}_{prec}"
            out[key] = fit_summary(*fit_timing(api, torch, X, w.h, w.kernel, 5, precision=prec))
            if prec == "fp32":
                out[key]["workload"] = (f"image_rgb: {side}x{side} RGB pixels ({side * side:,} points, "
                                        "D=3), 24 Voronoi colour regions + N(0, 6^2) noise, Gaussian h=12")
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
    rng = np.random.default_rng(1)
    Xs = [workloads.cloud16(rng, int(n), 2)[0] for n in rng.integers(200, 2000, 256)]
    Ss = [X[rng.choice(len(X), 32, replace=False)] for X in Xs]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    Xa = torch.from_numpy(np.concatenate(Xs)).cuda()
    Sa = torch.from_numpy(np.concatenate(Ss)).cuda()

    def batched(k, graph=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=k, graph=graph)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    batched(2)
    batched(2, True)
    t_e = min(batched(30) for _ in range(5))
    t_g = min(batched(30, True) for _ in range(5))
    best_R, ms_R, best_chunk, best_grid = api.tune_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, trials=8)
    t_t = min(batched(30) for _ in range(5))   # the tuned shape from here on
    out["small_clouds2_batched_fp32"] = {
        "workload": "256 clouds of 200..2000 points (%d points), D=2, 32 seeds each, Gaussian h=1, "
                    "30 iterations per call" % int(xo[-1]),
        "ms_per_call_eager": t_e * 1e3, "ms_per_call_graph": t_g * 1e3,
        "graph_speedup": t_e / t_g, "tuned_R": best_R, "tuned_chunk": best_chunk, "tuned_grid": best_grid,
        "tuner_ms_per_iteration_by_R": {str(r): v for r, v in ms_R.items()},
        "ms_per_call_tuned": t_t * 1e3}
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, and each workload's error against it
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def fit_error(gpu, modes_ref, labels_ref, margin_ref, k_ref, h):
    """The library's fit against the oracle's: K, the largest distance of a
    mode to its nearest oracle mode (over h), and the labels that differ after
    mapping the modes, in total and away from near-ties (two-mode margin of at
    least 1e-5 h)."""
    import numpy as np
    from scipy.spatial import cKDTree
    gm = gpu.modes.detach().cpu().numpy().astype(np.float64)
    om = np.asarray(modes_ref, np.float64)[:k_ref]
    out = {"K": gpu.k, "K_oracle": int(k_ref), "K_equal": gpu.k == int(k_ref)}
    if gpu.k == 0 or len(om) == 0:
        return out
    dist, match = cKDTree(om).query(gm, k=1)
    out["max_mode_err_over_h"] = float(dist.max() / h)
    if gpu.labels is not None and gpu.k == int(k_ref) and len(set(match.tolist())) == gpu.k:
        inv = np.empty(gpu.k, np.int64)
        inv[match] = np.arange(gpu.k)
        gl = gpu.labels.detach().cpu().numpy()
        diff = gl != inv[np.asarray(labels_ref)]
        out["labels_differ"] = int(diff.sum())
        out["labels_differ_away_from_ties"] = int((diff & (np.asarray(margin_ref) >= 1e-5 * h)).sum())
    return out


def median_time(f, reps=3):
    ts, r = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        r = f()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), r


def cpu_baseline(workloads, gpu_fits):
    """The oracle as it stands, on the host: medians of three runs on all
    threads and on one, for the 2-D blobs and the 200K mixture (whole fits)
    and a seed sample of the 32-D embeddings (64 seeds over all 262,144
    points, to convergence); each workload's GPU fit checked against it (the
    32-D one against the stored oracle fit)."""
    import numpy as np
    import oracle
    oracle.lib()
    nt = oracle.threads()
    res = {"cores": nt, "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    errors = {}
    w1 = workloads.blobs2d(seed=0)
    w2 = workloads.aniso3d(seed=0)
    w3 = workloads.embed32(seed=0)
    for name, w in (("c1", w1), ("c2", w2)):
        for th in (nt, 1):
            dt, r = median_time(lambda: oracle.fit(w.X, w.h, kernel=w.kernel, nthreads=th))
            res[f"{name}_fit_s_{'all' if th == nt else 'one'}_thread{'s' if th == nt else ''}"] = dt
            res[f"{name}_pair_evals_per_s_{'all' if th == nt else 'one'}"] = r.pairs / dt
            log(f"oracle {name} on {th} thread(s): {dt:.3f} s per fit")
        for prec in ("fp32", "bf16"):
            g = gpu_fits.get((name, prec))
            if g is not None:
                errors.setdefault(name, {})[prec] = fit_error(g, r.modes, r.labels, r.margin, r.k, w.h)
    rng = np.random.default_rng(64)
    S0 = w3.X[rng.choice(w3.n, 64, replace=False)].astype(np.float64)
    for th in (nt, 1):
        dt, o = median_time(lambda: oracle.step(w3.X, S0, w3.h, "gaussian", tol=1e-3, n_iter=100, nthreads=th))
        pairs = int(o[2].sum()) * w3.n
        res[f"c3_sample_s_{'all' if th == nt else 'one'}"] = dt
        res[f"c3_sample_pair_evals_per_s_{'all' if th == nt else 'one'}"] = pairs / dt
        log(f"oracle c3 sample on {th} thread(s): {dt:.3f} s")
    if os.path.exists(GOLDEN_C3):
        z = np.load(GOLDEN_C3, allow_pickle=False)
        margin = np.full(w3.n, np.inf)
        margin[z["near_idx"]] = z["near_margin"]
        for prec in ("fp32", "bf16"):
            g = gpu_fits.get(("c3", prec))
            if g is not None:
                errors.setdefault("c3", {})[prec] = fit_error(g, z["modes"], z["labels"].astype(np.int64), margin,
                                                              int(z["k"]), w3.h)
    # the 512 clouds' whole-method call: the smallest, the largest and two
    # other clouds against the oracle's fit of each cloud alone (cloud c
    # draws with state c), every sampled cloud's figures combined
    for prec in ("fp32", "bf16"):
        fb = gpu_fits.get(("c4", prec))
        if fb is None:
            continue
        per, lab, k_off, xo, Xs = fb
        sizes = np.diff(xo)
        pick = sorted({int(sizes.argmin()), int(sizes.argmax()), 100, 400})
        agg = {"clouds_checked": pick, "K_equal": True, "max_mode_err_over_h": 0.0, "labels_differ": 0,
               "labels_differ_away_from_ties": 0}
        for c in pick:
            ref = oracle.fit(Xs[c], 1.0, rng_seed=c, nthreads=nt)
            g = types.SimpleNamespace(modes=per[c], k=int(k_off[c + 1] - k_off[c]),
                                      labels=lab[int(xo[c]):int(xo[c + 1])])
            e = fit_error(g, ref.modes, ref.labels, ref.margin, ref.k, 1.0)
            agg["K_equal"] = agg["K_equal"] and e["K_equal"]
            agg["max_mode_err_over_h"] = max(agg["max_mode_err_over_h"], e.get("max_mode_err_over_h", float("inf")))
            agg["labels_differ"] += e.get("labels_differ", 0)
            agg["labels_differ_away_from_ties"] += e.get("labels_differ_away_from_ties", 0)
        errors.setdefault("c4", {})[prec] = agg
    value = res["c2_pair_evals_per_s_all"]
    return {"value": value, "unit": "pair evals/s", "cores": nt, "kind": "oracle",
            "sample": "the FP64 oracle's whole fit of the 200K mixture (median of 3 on all host threads); "
                      "also one thread, the 2-D blobs and a 64-seed sample of the 32-D embeddings; "
                      "four of the 512 clouds fitted once each for their errors",
            "time_to_cluster_ms": res["c2_fit_s_all_threads"] * 1e3, "detail": res,
            "error_vs_fp64": errors}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"],
                    help="precision of the headline value; the other form is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the secondary shapes (flat window, cosine metric, images, frames, small clouds)")
    ap.add_argument("--kernel-iters", type=int, default=20)
    ap.add_argument("--phase", default="all",
                    choices=["all", "kernel", "fit", "c3", "c3flat", "c3kernel", "batched", "batched_bf16", "c4kernel",
                             "c5"],
                    help="kernel: the 200K mixture's largest launch (both precisions) and a 256 MiB copy "
                         "that calibrates the traffic counters; fit: --steps fits per precision of the 200K "
                         "mixture; c3: --steps fits per precision of the 32-D embeddings; c3flat: the same "
                         "with the flat window (every window a singleton); c3kernel: their "
                         "largest launch (8,192 seeds) and the copy; batched: --steps whole-method calls on "
                         "the 512 uneven clouds (FP32; batched_bf16: the BF16 form); c4kernel: one batched-step call of --kernel-iters iterations "
                         "per precision on those clouds (every seed active) and the copy; c5: --steps steps of "
                         "the differentiable form; all: the benchmark")
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

    def copy_calibration(out):
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)   # 256 MiB read + 256 MiB written per launch
        torch.cuda.synchronize()
        out["copy_bytes_each_way"] = src.numel() * 4

    if args.phase in ("batched", "batched_bf16"):
        prec = "bf16" if args.phase == "batched_bf16" else "fp32"
        clouds = workloads.clouds16(seed=0)
        xo = np.concatenate([[0], np.cumsum([len(c[0]) for c in clouds])]).astype(np.int64)
        Xa = torch.from_numpy(np.concatenate([c[0] for c in clouds])).cuda()
        log(f"workload clouds16: {len(clouds)} clouds, {int(xo[-1])} points, D=16")
        for _ in range(args.warmup):
            api.fit_batched(Xa, xo, 1.0, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, k_off, rounds = api.fit_batched(Xa, xo, 1.0, precision=prec)
        torch.cuda.synchronize()
        print(json.dumps({"phase": "batched", "precision": prec,
                          "ms_per_call": (time.perf_counter() - t0) / args.steps * 1e3,
                          "rounds": rounds, "modes_total": int(k_off[-1])}), flush=True)
        return
    if args.phase == "c4kernel":
        clouds = workloads.clouds16(seed=0)
        Xs = [c[0] for c in clouds]
        rng = np.random.default_rng(0)
        Ss = [X[rng.choice(len(X), min(len(X), 256), replace=False)] for X in Xs]
        xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
        so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
        Xa = torch.from_numpy(np.concatenate(Xs)).cuda()
        Sa = torch.from_numpy(np.concatenate(Ss)).cuda()
        out = {"phase": "c4kernel", "launch": f"{len(Xs)} clouds, {int(xo[-1])} points, {int(so[-1])} seeds"}
        for prec in ("fp32", "bf16"):
            api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=2, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=args.kernel_iters, precision=prec)
            torch.cuda.synchronize()
            out[prec + "_call_ms"] = (time.perf_counter() - t0) * 1e3
        copy_calibration(out)
        print(json.dumps(out, default=_plain), flush=True)
        return
    if args.phase == "c5":
        out = config_c5(api, torch, workloads)
        out["phase"] = "c5"
        print(json.dumps(out, default=_plain), flush=True)
        return
    if args.phase in ("c3", "c3flat", "c3kernel"):
        w = workloads.embed32(seed=0)
        X = torch.from_numpy(w.X).cuda()
        out = {"phase": args.phase}
        if args.phase in ("c3", "c3flat"):
            kern = "flat" if args.phase == "c3flat" else w.kernel
            for prec in ("fp32", "bf16"):
                dt, r = fit_timing(api, torch, X, w.h, kern, args.steps, precision=prec)
                out[prec] = fit_summary(dt, r)
                out[prec]["breakdown_ms"] = {"iterate": r.iterate_ms, "merge_and_pool": r.merge_ms,
                                             "assign": r.assign_ms, "host_total": r.total_ms}
        else:
            rng = np.random.default_rng(8192)
            seeds = torch.from_numpy(w.X[rng.choice(w.n, 8192, replace=False)]).cuda()
            out["launch"] = f"8192 seeds x {w.n} points"
            for prec in ("fp32", "bf16"):
                t = time_kernel(api, torch, X, seeds, w.h, w.kernel, prec, args.kernel_iters)
                out[prec + "_iteration_ms"] = t
                out[prec + "_pair_evals_per_s"] = 8192 * w.n / (t * 1e-3)
            copy_calibration(out)
        print(json.dumps(out, default=_plain), flush=True)
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
        copy_calibration(out)
        print(json.dumps(out, default=_plain), flush=True)
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
        print(json.dumps(out, default=_plain), flush=True)
        return

    gpu_fits = {}
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
        gpu_fits[("c2", prec)] = last
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
    step_name = "step_bf16_kernel<3, 1, 1>" if args.precision == "bf16" else "step_cull_kernel<3, 1, 1>"
    roof = roofline_entry(pairs, d, t_it, m, n, args.precision, f"{m} seeds x {n} points",
                          f"one fused-step iteration: {step_name} + finalize_fused_kernel<3, 4, 1> "
                          "(chunk reduction and finalize in one launch)"
                          + (" + ordered_compact_kernel<3> (the active list in list order)"
                             if args.precision == "bf16" else ""),
                          counter_figures("c2", args.precision))
    log(f"kernel: {t_it * 1e3:.1f} us/iteration at {m}x{n}: {pairs / (t_it * 1e-3):.3e} pairs/s, "
        f"{roof['achieved']:.2f} TFLOP/s")

    # throughput stress: every point a seed (Algorithm 1 shape), one iteration
    t_all = time_kernel(api, torch, X, X, w.h, w.kernel, args.precision, 2)
    log(f"all-seeds iteration: {t_all:.2f} ms -> {n * n / (t_all * 1e-3):.3e} algorithmic pairs/s")

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
        "kernel_algorithmic_pair_evals_per_s": pairs / (t_it * 1e-3),
        "all_seeds_iteration_algorithmic_pair_evals_per_s": n * n / (t_all * 1e-3),
        "roofline": roof,
    }
    if roof.get("evaluated_pair_fraction") is not None:
        out["kernel_evaluated_pair_evals_per_s"] = roof["evaluated_pair_evals_per_s"]
    other = "fp32" if args.precision == "bf16" else "bf16"
    odt, olast = results[other]
    out[f"{other}_time_to_cluster_ms"] = odt / args.steps * 1e3
    out[f"{other}_pair_evals_per_s"] = olast.pairs * args.steps / odt
    if args.precision == "bf16":
        out["bf16_exact_pair_fraction"] = last.refined_pairs / max(1, last.pairs)
        out["speedup_time_to_cluster_vs_fp32"] = odt / dt
    t_other = time_kernel(api, torch, X, seeds, w.h, w.kernel, other, args.kernel_iters)
    out[f"{other}_kernel_algorithmic_pair_evals_per_s"] = pairs / (t_other * 1e-3)
    out["kernel_speedup_vs_" + other] = t_other / t_it
    log(f"{other} kernel: {t_other * 1e3:.1f} us/iteration -> {pairs / (t_other * 1e-3):.3e} pairs/s")
    t_plain = time_kernel(api, torch, X, seeds, w.h, w.kernel, "fp32", args.kernel_iters, plain=True)
    out["plain_fp32_time_to_cluster_ms"] = plain_dt / args.steps * 1e3
    out["plain_fp32_K"] = plast.k
    out["speedup_time_to_cluster_vs_plain_fp32"] = plain_dt / dt
    out["plain_fp32_kernel_algorithmic_pair_evals_per_s"] = pairs / (t_plain * 1e-3)
    out["kernel_speedup_vs_plain_fp32"] = t_plain / t_it
    log(f"plain fp32 kernel: {t_plain * 1e3:.1f} us/iteration")

    # every workload of the method, each with its roofline entry
    c2 = {"workload": out["config"]["workload"], args.precision: {"roofline": roof},
          other: {"roofline": roofline_entry(pairs, d, t_other, m, n, other, f"{m} seeds x {n} points",
                                             "one fused-step iteration", counter_figures("c2", other))}}
    for p_, (dt_, r_) in results.items():
        c2[p_].update(fit_summary(dt_ / args.steps, r_))
    out["configs"] = {"C1": config_c1(api, torch, workloads, gpu_fits), "C2": c2,
                      "C3": config_c3(api, torch, workloads, gpu_fits, max(3, args.kernel_iters // 4)),
                      "C4": config_c4(api, torch, workloads, gpu_fits), "C5": config_c5(api, torch, workloads)}
    if not args.no_other_configs:
        out["other_configs"] = other_configs(api, torch, workloads)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(workloads, gpu_fits)
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']:.3e} pairs/s on {cb['cores']} threads; errors {json.dumps(cb['error_vs_fp64'], default=_plain)}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out, default=_plain), flush=True)


if __name__ == "__main__":
    main()

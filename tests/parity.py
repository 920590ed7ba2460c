"""Comparison helpers between the HIP library and the FP64 oracle.

Contract (FP32 path):
  * ms_step: per seed, the iteration count equals the oracle's unless the
    oracle's shift at the deciding update lies within TIE_BAND of tol*h
    (FP32 computes that shift with ~1e-3 relative error); positions then
    agree within MODE_TOL * h at the same iteration count.
  * ms_fit: identical drawn-id lists per round, identical K, modes matched
    one-to-one within MODE_TOL * h, identical labels except where the
    oracle's two-mode margin is below MARGIN_TOL * h.
"""
import numpy as np

MODE_TOL = 1e-4
MARGIN_TOL = 1e-5
TIE_BAND = 1e-2


def step_parity(orc, X, seeds0, h, kernel, tol, gpu_S, gpu_iters, gpu_status, nthreads=None,
                metric="euclidean"):
    """Returns a report dict; raises AssertionError on a real mismatch."""
    S0 = np.asarray(seeds0, np.float64)
    oS, ost, oit, osh = orc.step(X, S0, h, kernel, tol=tol, n_iter=10_000, nthreads=nthreads,
                                 metric=metric)
    gS = np.asarray(gpu_S, np.float64)
    git = np.asarray(gpu_iters)
    gst = np.asarray(gpu_status)
    ties = 0
    worst = 0.0
    mism = np.nonzero(git != oit)[0]
    for j in mism:
        k = int(min(git[j], oit[j]))
        _, _, _, sh = orc.step(X, S0[j:j + 1], h, kernel, tol=1e-30, n_iter=k, nthreads=1, metric=metric)
        delta = float(np.sqrt(sh[0]))
        assert abs(delta - tol * h) <= TIE_BAND * tol * h, (
            f"seed {j}: iterations gpu {git[j]} vs oracle {oit[j]}, shift {delta} vs {tol * h}")
        ties += 1
        ref, _, _, _ = orc.step(X, S0[j:j + 1], h, kernel, tol=1e-30, n_iter=int(git[j]), nthreads=1,
                                metric=metric)
        err = float(np.abs(ref[0] - gS[j]).max())
        worst = max(worst, err)
        assert err <= MODE_TOL * h, (j, err)
    same = np.setdiff1d(np.arange(len(git)), mism)
    if same.size:
        err = np.abs(oS[same] - gS[same]).max(axis=1)
        worst = max(worst, float(err.max()))
        bad = np.nonzero(err > MODE_TOL * h)[0]
        assert bad.size == 0, f"{bad.size} seeds off by up to {err.max()} (h={h})"
        assert np.array_equal(gst[same], ost[same])
    return {"ties": ties, "max_err_over_h": worst / h, "seeds": len(git)}


def iteration_ties(orc, X, h, kernel, tol, drawn, g_iters, o_iters, g_status, o_status):
    """Seeds whose iteration count (or converged status) differs must sit at a
    convergence-threshold tie in the oracle.  Returns the number of ties."""
    ties = 0
    for j in np.nonzero((g_iters != o_iters) | (g_status != o_status))[0]:
        k = int(min(g_iters[j], o_iters[j]))
        s0 = X[drawn[j]:drawn[j] + 1].astype(np.float64)
        _, _, _, sh = orc.step(X, s0, h, kernel, tol=1e-30, n_iter=k, nthreads=1)
        delta = float(np.sqrt(sh[0]))
        assert abs(delta - tol * h) <= TIE_BAND * tol * h, (
            f"drawn seed {j} (id {drawn[j]}): iterations {g_iters[j]} vs {o_iters[j]}, "
            f"shift {delta} vs threshold {tol * h}")
        ties += 1
    return ties


def fit_parity(gpu, ref, X, h, margin_tol=MARGIN_TOL, mode_tol=MODE_TOL, orc=None,
               kernel="gaussian", tol=1e-3):
    """Compare a traced api.fit result with oracle.fit.  Returns a report."""
    rep = {}
    g_rounds = gpu.drawn_rounds()
    o_rounds = ref.rounds()
    assert len(g_rounds) == len(o_rounds), (gpu.round_N, ref.round_N)
    for r, (a, b) in enumerate(zip(g_rounds, o_rounds)):
        assert np.array_equal(a, b), f"round {r}: drawn ids differ"
    if orc is not None:
        rep["iteration_ties"] = iteration_ties(orc, X, h, kernel, tol, ref.drawn, gpu.drawn_iters,
                                               ref.drawn_iters, gpu.drawn_status, ref.drawn_status)
        if rep["iteration_ties"] == 0:
            assert gpu.pairs == ref.pairs
    assert gpu.k == ref.k, (gpu.k, ref.k)
    gm = gpu.modes.detach().cpu().numpy().astype(np.float64)
    # one-to-one nearest matching
    D = np.linalg.norm(gm[:, None, :] - ref.modes[None, :, :], axis=2) if gm.size else np.zeros((0, 0))
    match = D.argmin(axis=1)
    assert len(set(match.tolist())) == gpu.k, "mode matching is not one-to-one"
    err = D[np.arange(gpu.k), match].max() if gpu.k else 0.0
    rep["max_mode_err_over_h"] = float(err / h)
    assert err <= mode_tol * h, f"mode error {err / h:.3e} h"
    # modes are created in the same (draw) order, so the matching is the identity
    rep["identity_order"] = bool(np.array_equal(match, np.arange(gpu.k)))
    if gpu.labels is not None:
        gl = gpu.labels.detach().cpu().numpy()
        ol = match.argsort()[ref.labels] if not rep["identity_order"] else ref.labels
        diff = gl != ol
        near = ref.margin < margin_tol * h
        rep["label_mismatch"] = int(diff.sum())
        rep["label_mismatch_near_tie"] = int((diff & near).sum())
        assert not (diff & ~near).any(), f"{int((diff & ~near).sum())} labels differ away from ties"
    return rep


def flat_boundary_tie(X, s0, h, n_iter, rel=1e-5):
    """True when, along the FP64 trajectory of the flat-window update from
    s0, some point lies within rel*h of the window boundary: a place where
    any finite-precision evaluation may legitimately take the other side."""
    Xd = np.asarray(X, np.float64)
    s = np.asarray(s0, np.float64).copy()
    for _ in range(n_iter):
        dist = np.sqrt(((Xd - s) ** 2).sum(1))
        if np.min(np.abs(dist - h)) <= rel * h:
            return True
        win = dist <= h
        s = Xd[win].mean(0)
    return False


def ragged_check(X, S0, h, kernel, n_iter, gpu_S, gpu_iters, ref_S, ref_iters):
    """Per-seed comparison for a fixed number of updates; seeds that differ
    must sit at a flat-window boundary tie.  Returns the number of ties."""
    same = gpu_iters == ref_iters
    assert same.mean() > 0.98
    err = np.abs(gpu_S - ref_S).max(axis=1)
    bad = np.nonzero(same & (err > MODE_TOL * h))[0]
    ties = 0
    for j in bad:
        assert kernel == "flat" and flat_boundary_tie(X, S0[j], h, n_iter), (
            f"seed {j}: error {err[j]} > {MODE_TOL * h}")
        ties += 1
    return ties

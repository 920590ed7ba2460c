"""GPU parity of the HIP library against the FP64 oracle (through the C ABI).

Inputs are the seeded synthetic workloads of paper_2112_13891_amd.workloads
at the paper-shaped sizes (2-D blobs, 200K-point 3-D mixture, 262K-point
32-D embedding mixture), plus small ragged and degenerate cases.
"""
import sys

import numpy as np
import pytest

from parity import MARGIN_TOL, MODE_TOL, fit_parity, ragged_check, step_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def blobs():
    return workloads.blobs2d(seed=0)


@pytest.fixture(scope="module")
def aniso():
    return workloads.aniso3d(seed=0)


@pytest.fixture(scope="module")
def embed():
    return workloads.embed32(seed=0)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# ---------------------------------------------------------------------------
# ms_step trajectories
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_step_blobs2d_all_seeds(orc, blobs, kernel):
    say("step blobs2d", kernel)
    X = _gpu(blobs.X)
    S, conv, it, sh = api.step(X, X, blobs.h, kernel=kernel, tol=1e-3, n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, blobs.X, blobs.X, blobs.h, kernel, 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)
    assert (conv.cpu().numpy() == 1).all()


def test_step_aniso3d_sample(orc, aniso):
    say("step aniso3d sample")
    rng = np.random.default_rng(1)
    idx = rng.choice(aniso.n, 2000, replace=False)
    X = _gpu(aniso.X)
    S0 = aniso.X[idx]
    S, conv, it, sh = api.step(X, _gpu(S0), aniso.h, n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, aniso.X, S0, aniso.h, "gaussian", 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_step_embed32_sample(orc, embed, kernel):
    say("step embed32 sample", kernel)
    rng = np.random.default_rng(2)
    idx = rng.choice(embed.n, 96, replace=False)
    X = _gpu(embed.X)
    S0 = embed.X[idx]
    S, conv, it, sh = api.step(X, _gpu(S0), embed.h, kernel=kernel, n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, embed.X, S0, embed.h, kernel, 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)


@pytest.mark.parametrize("n,d", [(1, 1), (2, 3), (3, 2), (255, 4), (257, 5), (1000, 7),
                                 (1031, 8), (777, 13), (513, 16), (300, 33), (129, 64),
                                 (4099, 3)])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_step_ragged_shapes(orc, n, d, kernel):
    say("step ragged", n, d, kernel)
    rng = np.random.default_rng(n * 100 + d)
    X = (rng.standard_normal((n, d)) * 2.0).astype(np.float32)
    m = min(n, 300)
    S0 = X[rng.choice(n, m, replace=False)]
    h = 1.5 * np.sqrt(d)
    for n_iter in (1, 3):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter)
        ties = ragged_check(orc, X, S0, h, kernel, n_iter, S.cpu().numpy(), it.cpu().numpy(),
                            conv.cpu().numpy(), ref, oit, ost)
        if ties:
            say("flat boundary ties", ties)


@pytest.mark.parametrize("n,d", [(300, 65), (1031, 100), (513, 128), (200, 129), (777, 200),
                                 (300, 256), (70, 256)])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_step_wide_rows(orc, n, d, kernel):
    """Rows of 65..256 coordinates (padded to 128 or 256): the four waves of a
    workgroup split the coordinates, one wave per seed finalizes."""
    say("step wide", n, d, kernel)
    rng = np.random.default_rng(n * 1000 + d)
    C = 4.0 * rng.standard_normal((5, d))
    X = (C[rng.integers(0, 5, n)] + 0.5 * rng.standard_normal((n, d))).astype(np.float32)
    m = min(n, 150)
    S0 = X[rng.choice(n, m, replace=False)]
    h = 0.5 * np.sqrt(d) * (1.0 if kernel == "gaussian" else 1.6)
    for n_iter in (1, 4):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter)
        ties = ragged_check(orc, X, S0, h, kernel, n_iter, S.cpu().numpy(), it.cpu().numpy(),
                            conv.cpu().numpy(), ref, oit, ost)
        if ties:
            say("ties", ties)
    S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, n_iter=100)
    torch.cuda.synchronize()
    say(step_parity(orc, X, S0, h, kernel, 1e-3, S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy()))


@pytest.mark.parametrize("d", [65, 128, 256])
@pytest.mark.parametrize("all_points", [False, True])
def test_fit_wide_rows(orc, d, all_points):
    rng = np.random.default_rng(d)
    C = 4.0 * rng.standard_normal((6, d))
    n = 2500
    X = (C[rng.integers(0, 6, n)] + 0.5 * rng.standard_normal((n, d))).astype(np.float32)
    h = 0.5 * np.sqrt(d)
    g = api.fit(_gpu(X), h, all_points=all_points, trace=True)
    ref = orc.fit(X, h, all_points=all_points)
    rep = fit_parity(g, ref, X, h, orc=orc)
    say("fit wide", d, all_points, rep, "K", g.k)


def test_step_respects_converged_flags(orc, blobs):
    X = _gpu(blobs.X)
    S0 = blobs.X[:64]
    conv0 = np.zeros(64, np.uint8)
    conv0[::3] = 1
    S, conv, it, sh = api.step(X, _gpu(S0), blobs.h, n_iter=5, converged=_gpu(conv0))
    torch.cuda.synchronize()
    g = S.cpu().numpy()
    assert np.array_equal(g[::3], S0[::3]) and (it.cpu().numpy()[::3] == 0).all()
    assert (it.cpu().numpy()[1::3] > 0).all()


# ---------------------------------------------------------------------------
# ms_fit end to end
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("all_points", [False, True])
def test_fit_blobs2d(orc, blobs, all_points):
    say("fit blobs2d all_points", all_points)
    g = api.fit(_gpu(blobs.X), blobs.h, all_points=all_points, trace=True)
    ref = orc.fit(blobs.X, blobs.h, all_points=all_points)
    rep = fit_parity(g, ref, blobs.X, blobs.h, orc=orc)
    say(rep, "K", g.k, "rounds", g.round_N)
    assert g.k == 5


def test_fit_aniso3d_pool(orc, aniso):
    say("fit aniso3d pool")
    g = api.fit(_gpu(aniso.X), aniso.h, trace=True)
    ref = orc.fit(aniso.X, aniso.h)
    rep = fit_parity(g, ref, aniso.X, aniso.h, orc=orc)
    say(rep, "K", g.k, "rounds", g.round_N.tolist(), "pairs", g.pairs, "ms", g.total_ms)


def test_fit_flat_kernel_small(orc):
    rng = np.random.default_rng(7)
    C = rng.uniform(0, 50, (6, 3))
    y = rng.integers(0, 6, 3000)
    X = (C[y] + 0.8 * rng.standard_normal((3000, 3))).astype(np.float32)
    for all_points in (False, True):
        g = api.fit(_gpu(X), 2.5, kernel="flat", all_points=all_points, trace=True)
        ref = orc.fit(X, 2.5, kernel="flat", all_points=all_points)
        say(fit_parity(g, ref, X, 2.5, orc=orc, kernel="flat"))


@pytest.mark.parametrize("all_points", [False, True])
def test_fit_merge_chain(orc, all_points):
    """Isolated points on a line 5h apart with merge radius 6h: each seed stays
    on its point, and every merge decision waits on the previous link of a
    chain far deeper than the device decision passes resolve, so the host
    finishes the merge (and redoes the pool coverage) -- the same greedy
    result as the sequential rule."""
    n = 300
    X = np.zeros((n, 2), np.float32)
    X[:, 0] = 5.0 * np.arange(n, dtype=np.float32)
    g = api.fit(_gpu(X), 1.0, kernel="flat", merge_radius=6.0, all_points=all_points, trace=True)
    ref = orc.fit(X, 1.0, kernel="flat", merge_radius=6.0, all_points=all_points)
    say(fit_parity(g, ref, X, 1.0, orc=orc, kernel="flat"), "K", g.k)


def test_fit_gamma_early_stop(orc, aniso):
    X = aniso.X[:20000]
    g = api.fit(_gpu(X), aniso.h, gamma=0.75, trace=True)
    ref = orc.fit(X, aniso.h, gamma=0.75)
    assert np.array_equal(g.round_T, ref.round_T)
    say(fit_parity(g, ref, X, aniso.h, orc=orc))


def test_fit_deterministic(aniso):
    X = _gpu(aniso.X)
    a = api.fit(X, aniso.h, trace=True)
    b = api.fit(X, aniso.h, trace=True)
    assert torch.equal(a.modes, b.modes) and torch.equal(a.labels, b.labels)
    assert np.array_equal(a.drawn_final, b.drawn_final)


def test_fit_capacity_and_no_modes(blobs):
    X = _gpu(blobs.X)
    with pytest.raises(api.MeanShiftError) as e:
        api.fit(X, blobs.h, max_modes=3)
    assert e.value.code == api.MS_E_CAPACITY and e.value.k == 5
    with pytest.raises(api.MeanShiftError) as e:
        api.fit(X, blobs.h, max_iter=1, tol=1e-9)
    assert e.value.code == api.MS_E_NO_MODES


def test_fit_nonfinite(blobs):
    Xh = blobs.X.copy()
    Xh[17, 1] = np.nan
    with pytest.raises(api.MeanShiftError) as e:
        api.fit(_gpu(Xh), blobs.h, check_finite=True)
    assert e.value.code == api.MS_E_NONFINITE


def test_fit_single_point_and_tiny():
    X = _gpu(np.array([[1.5, -2.0, 3.0]], np.float32))
    g = api.fit(X, 1.0, trace=True)
    assert g.k == 1 and g.labels.cpu().tolist() == [0]
    assert np.allclose(g.modes.cpu().numpy(), [[1.5, -2.0, 3.0]])


# ---------------------------------------------------------------------------
# ms_assign
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,k", [(200_000, 3, 50), (5000, 32, 300), (1001, 2, 1),
                                   (3000, 64, 1500), (70_000, 16, 37), (4000, 65, 70),
                                   (3001, 128, 257), (2000, 256, 40)])
def test_assign_parity(orc, n, d, k):
    rng = np.random.default_rng(n + d + k)
    X = (rng.standard_normal((n, d)) * 10).astype(np.float32)
    M = X[rng.choice(n, k, replace=False)] + np.float32(0.01)
    lab, mg = api.assign(_gpu(X), _gpu(M), margin=True)
    torch.cuda.synchronize()
    ol, om = orc.assign(X, M.astype(np.float64))
    gl = lab.cpu().numpy()
    diff = gl != ol
    assert not (diff & (om >= 1e-5)).any()
    gm = mg.cpu().numpy()
    fin = np.isfinite(om)
    assert np.allclose(gm[fin], om[fin], atol=1e-3 * 10) and (~np.isfinite(gm) == ~fin).all()


def test_assign_ties_to_lowest_index():
    X = _gpu(np.array([[0.0], [1.0], [2.0]], np.float32))
    M = _gpu(np.array([[0.5], [1.5], [0.5]], np.float32))
    assert api.assign(X, M).cpu().tolist() == [0, 0, 1]


# ---------------------------------------------------------------------------
# BF16+refine form (D <= 4): same contract as the FP32 form
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_bf16_step_blobs2d_all_seeds(orc, blobs, kernel):
    say("bf16 step blobs2d", kernel)
    X = _gpu(blobs.X)
    S, conv, it, sh = api.step(X, X, blobs.h, kernel=kernel, precision="bf16", n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, blobs.X, blobs.X, blobs.h, kernel, 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)


def test_bf16_step_aniso3d_sample(orc, aniso):
    say("bf16 step aniso3d sample")
    rng = np.random.default_rng(1)
    idx = rng.choice(aniso.n, 2000, replace=False)
    S0 = aniso.X[idx]
    S, conv, it, sh = api.step(_gpu(aniso.X), _gpu(S0), aniso.h, precision="bf16", n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, aniso.X, S0, aniso.h, "gaussian", 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)


@pytest.mark.parametrize("n,d", [(1, 1), (2, 3), (3, 2), (255, 4), (257, 3), (1000, 1),
                                 (4099, 3), (20000, 2)])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_bf16_step_ragged_shapes(orc, n, d, kernel):
    rng = np.random.default_rng(n * 100 + d + 7)
    X = (rng.standard_normal((n, d)) * 2.0 + 50.0).astype(np.float32)
    m = min(n, 300)
    S0 = X[rng.choice(n, m, replace=False)]
    h = 1.5 * np.sqrt(d)
    for n_iter in (1, 3):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, precision="bf16",
                                   n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter)
        ties = ragged_check(orc, X, S0, h, kernel, n_iter, S.cpu().numpy(), it.cpu().numpy(),
                            conv.cpu().numpy(), ref, oit, ost)
        if ties:
            say("flat boundary ties", ties)


@pytest.mark.parametrize("all_points", [False, True])
def test_bf16_fit_blobs2d(orc, blobs, all_points):
    g = api.fit(_gpu(blobs.X), blobs.h, precision="bf16", all_points=all_points, trace=True)
    ref = orc.fit(blobs.X, blobs.h, all_points=all_points)
    rep = fit_parity(g, ref, blobs.X, blobs.h, orc=orc)
    say("bf16 fit blobs2d", all_points, rep, "refined", g.refined_pairs, "of", g.pairs)
    assert 0 < g.refined_pairs < g.pairs


def test_bf16_fit_aniso3d_pool(orc, aniso):
    g = api.fit(_gpu(aniso.X), aniso.h, precision="bf16", trace=True)
    ref = orc.fit(aniso.X, aniso.h)
    rep = fit_parity(g, ref, aniso.X, aniso.h, orc=orc)
    say("bf16 fit aniso3d", rep, "refined", g.refined_pairs, "of", g.pairs, "ms", g.total_ms)


def test_bf16_fit_flat_small(orc):
    rng = np.random.default_rng(7)
    C = rng.uniform(0, 50, (6, 3))
    y = rng.integers(0, 6, 3000)
    X = (C[y] + 0.8 * rng.standard_normal((3000, 3))).astype(np.float32)
    for all_points in (False, True):
        g = api.fit(_gpu(X), 2.5, kernel="flat", precision="bf16", all_points=all_points, trace=True)
        ref = orc.fit(X, 2.5, kernel="flat", all_points=all_points)
        say(fit_parity(g, ref, X, 2.5, orc=orc, kernel="flat"))


def _mixture2d(seed, n):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 100, (8, 2))
    y = rng.integers(0, 8, n)
    return (C[y] + 2.0 * rng.standard_normal((n, 2))).astype(np.float32)


def test_bf16_step_many_seeds_repeatable(orc):
    """More than 4,096 active seeds (the ordered compaction places more than
    64 runs): every point of a 12,000-point 2-D mixture as a seed, 1 and 3
    iterations against the oracle, and a second call gives the same bits."""
    X = _mixture2d(21, 12000)
    h = 4.0
    for n_iter in (1, 3):
        say("bf16 step, 12000 seeds, n_iter", n_iter)
        S, conv, it, sh = api.step(_gpu(X), _gpu(X), h, precision="bf16", n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, X.astype(np.float64), h, "gaussian", tol=1e-3, n_iter=n_iter)
        ragged_check(orc, X, X, h, "gaussian", n_iter, S.cpu().numpy(), it.cpu().numpy(),
                     conv.cpu().numpy(), ref, oit, ost)
    again = api.step(_gpu(X), _gpu(X), h, precision="bf16", n_iter=3)
    torch.cuda.synchronize()
    for a, b in zip((S, conv, it, sh), again):
        torch.testing.assert_close(b.cpu(), a.cpu(), rtol=0, atol=0, equal_nan=True)


@pytest.mark.parametrize("n,d", [(300_000, 3), (230_000, 4)])
def test_bf16_step_reduced_partials_ordered(orc, n, d):
    """Enough points that a tile's chunk partials exceed the one-launch
    reduce-and-finalize (more than 2,048 floats per slot): the reduction,
    the finalize and the ordered placement of the active list run as three
    launches, the finalize reading the reduced sums from the rows it then
    fills with each run's kept seeds.  256 seeds, 1 and 3 iterations
    against the oracle; a second call gives the same bits."""
    rng = np.random.default_rng(n + d)
    C = rng.uniform(0, 400, (30, d))
    y = rng.integers(0, 30, n)
    X = (C[y] + 6.0 * rng.standard_normal((n, d))).astype(np.float32)
    S0 = X[rng.choice(n, 256, replace=False)]
    h = 10.0
    for n_iter in (1, 3):
        say("bf16 step, reduced partials", n, d, "n_iter", n_iter)
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, precision="bf16", n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, "gaussian", tol=1e-3, n_iter=n_iter)
        ragged_check(orc, X, S0, h, "gaussian", n_iter, S.cpu().numpy(), it.cpu().numpy(),
                     conv.cpu().numpy(), ref, oit, ost)
    again = api.step(_gpu(X), _gpu(S0), h, precision="bf16", n_iter=3)
    torch.cuda.synchronize()
    for a, b in zip((S, conv, it, sh), again):
        torch.testing.assert_close(b.cpu(), a.cpu(), rtol=0, atol=0, equal_nan=True)


def test_bf16_fit_all_points_many_seeds(orc):
    """Algorithm 1 with 12,000 seeds in the BF16 form against the oracle."""
    X = _mixture2d(22, 12000)
    g = api.fit(_gpu(X), 4.0, precision="bf16", all_points=True, trace=True)
    ref = orc.fit(X, 4.0, all_points=True)
    say("bf16 fit, all 12000 points as seeds", fit_parity(g, ref, X, 4.0, orc=orc))


def test_bf16_deterministic(aniso):
    X = _gpu(aniso.X)
    a = api.fit(X, aniso.h, precision="bf16", trace=True)
    b = api.fit(X, aniso.h, precision="bf16", trace=True)
    assert torch.equal(a.modes, b.modes) and torch.equal(a.labels, b.labels)
    assert np.array_equal(a.drawn_final, b.drawn_final)


def test_bf16_rejects_large_d():
    X = _gpu(np.zeros((10, 33), np.float32))
    with pytest.raises(api.MeanShiftError) as e:
        api.fit(X, 1.0, precision="bf16")
    assert e.value.code == api.MS_E_INVALID


# ---------------------------------------------------------------------------
# BF16 screen form (8 <= D <= 32): products on MFMA screen the pairs, every
# pair above the screen is exact -- same contract as the FP32 form
# ---------------------------------------------------------------------------

def _clustered(seed, n, d, k, sigma=0.5, spread=4.0, outliers=0.03):
    rng = np.random.default_rng(seed)
    C = spread * rng.standard_normal((k, d))
    n_out = int(round(outliers * n))
    y = rng.integers(0, k, n - n_out)
    X = np.concatenate([C[y] + sigma * rng.standard_normal((n - n_out, d)),
                        rng.uniform(-3 * spread, 3 * spread, (n_out, d))])
    return X[rng.permutation(n)].astype(np.float32)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_bf16_step_embed32_sample(orc, embed, kernel):
    say("bf16 step embed32 sample", kernel)
    rng = np.random.default_rng(2)
    idx = rng.choice(embed.n, 96, replace=False)
    S0 = embed.X[idx]
    S, conv, it, sh = api.step(_gpu(embed.X), _gpu(S0), embed.h, kernel=kernel, precision="bf16",
                               n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, embed.X, S0, embed.h, kernel, 1e-3, S.cpu().numpy(),
                      it.cpu().numpy(), conv.cpu().numpy())
    say(rep)


@pytest.mark.parametrize("n,d", [(1, 5), (2, 8), (257, 5), (1000, 7), (1031, 8), (777, 13),
                                 (513, 16), (300, 17), (2049, 32), (4099, 24)])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
@pytest.mark.parametrize("layout", ["noise", "clusters"])
def test_bf16_step_ragged_wide(orc, n, d, kernel, layout):
    rng = np.random.default_rng(n * 100 + d + 11)
    if layout == "noise":   # every pair near: the exact path everywhere
        X = (rng.standard_normal((n, d)) * 2.0 + 50.0).astype(np.float32)
        h = 1.5 * np.sqrt(d)
    else:                   # separated clusters: most tiles below the screen
        X = _clustered(n + d, n, d, 6) + np.float32(20.0)
        h = 1.5
    m = min(n, 300)
    S0 = X[rng.choice(n, m, replace=False)]
    for n_iter in (1, 3):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, precision="bf16",
                                   n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter)
        ties = ragged_check(orc, X, S0, h, kernel, n_iter, S.cpu().numpy(), it.cpu().numpy(),
                            conv.cpu().numpy(), ref, oit, ost)
        if ties:
            say("flat boundary ties", ties)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
@pytest.mark.parametrize("all_points", [False, True])
def test_bf16_fit_wide(orc, kernel, all_points):
    X = _clustered(5, 4000, 32, 10)
    h = 1.5 if kernel == "gaussian" else 4.0   # a flat window of h = 1.5 holds one point in 32-D
    g = api.fit(_gpu(X), h, kernel=kernel, precision="bf16", all_points=all_points, trace=True)
    ref = orc.fit(X, h, kernel=kernel, all_points=all_points)
    rep = fit_parity(g, ref, X, h, orc=orc, kernel=kernel)
    say("bf16 fit wide", kernel, all_points, rep, "K", g.k, "exact pairs", g.refined_pairs,
        "of", g.pairs)
    assert g.refined_pairs < g.pairs


def test_bf16_deterministic_wide():
    X = _gpu(_clustered(9, 6000, 16, 12))
    a = api.fit(X, 1.0, precision="bf16", trace=True)
    b = api.fit(X, 1.0, precision="bf16", trace=True)
    assert torch.equal(a.modes, b.modes) and torch.equal(a.labels, b.labels)
    assert np.array_equal(a.drawn_final, b.drawn_final)

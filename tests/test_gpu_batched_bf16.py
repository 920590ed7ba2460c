"""GPU parity of the BF16 form of ms_step_batched (Gaussian kernel, 5 <= d <=
32): each cloud's points in the spatial order of the one-cloud BF16 form
(its own pivots and 256-point blocks), the seed-point products and W.X on
MFMA with the compensated three-part operands, the pairs the expanded form
cannot resolve computed in FP32 -- against the FP64 oracle run on each cloud
alone (Section II-B update, per-seed convergence of Algorithms 1-2)."""
import sys

import numpy as np
import pytest

from parity import MODE_TOL, ragged_check, step_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _batch(seed, sizes, d, max_seeds=150):
    """Clouds of the batched recipe (2..40 clusters, sigma 0.4 around centres
    N(0, 9 I)) with the given sizes; seeds drawn from each cloud's points."""
    rng = np.random.default_rng(seed)
    Xs, Ss = [], []
    for n in sizes:
        if n == 0:
            Xs.append(np.zeros((0, d), np.float32))
            Ss.append(np.zeros((0, d), np.float32))
            continue
        X, _, _ = workloads.cloud16(rng, n, d)
        m = int(min(n, rng.integers(0, max_seeds + 1)))
        Xs.append(X)
        Ss.append(X[rng.choice(n, m, replace=False)] if m else np.zeros((0, d), np.float32))
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    return Xs, Ss, xo, so


def _tensors(Xs, Ss):
    return (torch.from_numpy(np.concatenate(Xs)).to(DEV), torch.from_numpy(np.concatenate(Ss)).to(DEV))


# ragged clouds: empty, single points, sizes around the 256-point block and
# the 1,024-point chunk, and one with several pivots and many blocks
SIZES = [1, 2, 300, 0, 1500, 64, 2047, 4100, 17, 1025, 9000, 255, 257]


@pytest.mark.parametrize("d", [5, 8, 16, 29, 32])
def test_bf16_batched_fixed_iterations(orc, d):
    Xs, Ss, xo, so = _batch(300 + d, SIZES, d)
    Xa, Sa = _tensors(Xs, Ss)
    h = 1.0
    for n_iter in (1, 3):
        say("bf16 batched d", d, "n_iter", n_iter)
        S, conv, it, sh = api.step_batched(Xa, xo, Sa, so, h, n_iter=n_iter, precision="bf16")
        torch.cuda.synchronize()
        S, it, conv = S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy()
        for c in range(len(Xs)):
            a, b = so[c], so[c + 1]
            if a == b:
                continue
            ref, ost, oit, osh = orc.step(Xs[c], Ss[c].astype(np.float64), h, "gaussian", tol=1e-3,
                                          n_iter=n_iter)
            ragged_check(orc, Xs[c], Ss[c], h, "gaussian", n_iter, S[a:b], it[a:b], conv[a:b], ref, oit, ost)


def test_bf16_batched_to_convergence(orc):
    Xs, Ss, xo, so = _batch(377, SIZES, 16, max_seeds=300)
    Xa, Sa = _tensors(Xs, Ss)
    S, conv, it, sh = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=100, precision="bf16")
    torch.cuda.synchronize()
    S, conv, it = S.cpu().numpy(), conv.cpu().numpy(), it.cpu().numpy()
    for c in range(len(Xs)):
        a, b = so[c], so[c + 1]
        if a == b:
            continue
        rep = step_parity(orc, Xs[c], Ss[c], 1.0, "gaussian", 1e-3, S[a:b], it[a:b], conv[a:b])
        say("cloud", c, "n", len(Xs[c]), rep)


def test_bf16_batched_close_to_fp32_and_keeps_converged_seeds():
    """Seeds flagged converged are passed through untouched; the others agree
    with the FP32 batched step to within the parity bar."""
    Xs, Ss, xo, so = _batch(5, [500, 3000, 40, 9000], 16, max_seeds=300)
    Xa, Sa = _tensors(Xs, Ss)
    M = int(so[-1])
    rng = np.random.default_rng(1)
    conv0 = torch.from_numpy((rng.random(M) < 0.3).astype(np.uint8)).to(DEV)
    S, conv, it, _ = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=4, converged=conv0, precision="bf16")
    S32, conv32, it32, _ = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=4, converged=conv0)
    torch.cuda.synchronize()
    kept = conv0.cpu().numpy() == 1
    S, S32 = S.cpu().numpy(), S32.cpu().numpy()
    S0 = np.concatenate(Ss)
    assert np.array_equal(S[kept], S0[kept]) and (it.cpu().numpy()[kept] == 0).all()
    same = (it.cpu().numpy() == it32.cpu().numpy()) & (conv.cpu().numpy() == conv32.cpu().numpy())
    assert same.mean() > 0.99
    err = np.abs(S[same].astype(np.float64) - S32[same]).max()
    say("BF16 vs FP32 batched: largest difference", err, "seeds", int(same.sum()), "of", M)
    assert err < MODE_TOL * 1.0


def test_bf16_batched_graph_grid_and_repeat_bitwise():
    """The graph launch, another step grid and a second identical call give
    bitwise the same outputs (the chunking depends only on the counts and the
    chunk size, and no floating-point atomics)."""
    Xs, Ss, xo, so = _batch(91, SIZES, 16, max_seeds=300)
    Xa, Sa = _tensors(Xs, Ss)
    ref = [t.cpu() for t in api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=6, precision="bf16")]
    for kw in ({"graph": True}, {"tile_grid": 37}, {}, {"graph": True}):
        say("bf16 batched repeat", kw)
        got = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=6, precision="bf16", **kw)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            torch.testing.assert_close(b.cpu(), a, rtol=0, atol=0, equal_nan=True)


@pytest.mark.parametrize("chunk", [256, 700, 4096, 65536])
def test_bf16_batched_chunk_size_changes_rounding_only(chunk):
    """Chunks of whole blocks (a size is rounded up to a multiple of 256):
    after a few iterations with no convergence decisions (tol 1e-30) the seeds
    agree with the default chunking to within the FP32 rounding of the sums."""
    Xs, Ss, xo, so = _batch(70, SIZES, 8, max_seeds=200)
    Xa, Sa = _tensors(Xs, Ss)
    ref = api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=3, tile_chunk=1024,
                           precision="bf16")[0].cpu().numpy()
    got = api.step_batched(Xa, xo, Sa, so, 1.0, tol=1e-30, n_iter=3, tile_chunk=chunk,
                           precision="bf16")[0].cpu().numpy()
    err = float(np.abs(got.astype(np.float64) - ref).max())
    say("chunk", chunk, "largest difference to 1024-point chunks", err)
    assert err <= 1e-4


def test_bf16_batched_rejects_what_is_not_built():
    Xs, Ss, xo, so = _batch(3, [300, 500], 3)
    Xa, Sa = _tensors(Xs, Ss)
    with pytest.raises(api.MeanShiftError, match="Gaussian kernel at 5 <= d <= 32"):
        api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=1, precision="bf16")
    Xs, Ss, xo, so = _batch(3, [300, 500], 16)
    Xa, Sa = _tensors(Xs, Ss)
    with pytest.raises(api.MeanShiftError, match="Gaussian kernel at 5 <= d <= 32"):
        api.step_batched(Xa, xo, Sa, so, 1.0, kernel="flat", n_iter=1, precision="bf16")


def test_bf16_batched_full_size_sampled(orc):
    """The batched workload at full size (512 clouds of 1,000..65,536 points,
    D = 16, min(n, 256) seeds per cloud) in the BF16 form: after 3
    iterations, the seeds of sampled clouds (the smallest, the largest and two
    others) against the oracle run on each cloud alone."""
    clouds = workloads.clouds16(seed=0)
    Xs = [c[0] for c in clouds]
    rng = np.random.default_rng(0)
    Ss = [X[rng.choice(len(X), min(len(X), 256), replace=False)] for X in Xs]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum([len(s) for s in Ss])]).astype(np.int64)
    say("full-size batched bf16", len(Xs), "clouds", int(xo[-1]), "points")
    Xa, Sa = _tensors(Xs, Ss)
    S, conv, it, sh = api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=3, precision="bf16")
    torch.cuda.synchronize()
    S, it, conv = S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy()
    sizes = np.array([len(x) for x in Xs])
    for c in sorted({int(sizes.argmin()), int(sizes.argmax()), 100, 400}):
        a, b = so[c], so[c + 1]
        ref, ost, oit, osh = orc.step(Xs[c], Ss[c].astype(np.float64), 1.0, "gaussian", tol=1e-3, n_iter=3)
        say("cloud", c, "n", len(Xs[c]))
        ragged_check(orc, Xs[c], Ss[c], 1.0, "gaussian", 3, S[a:b], it[a:b], conv[a:b], ref, oit, ost)


def test_bf16_batched_tuner_keeps_tiles_of_128():
    """The tuner searches the BF16 form's chunk sizes and grids with tiles of
    128 seeds only, records the shape under the BF16 precision, and later
    default calls take it: the same bits as the explicit shape."""
    Xs, Ss, xo, so = _batch(52, SIZES, 16, max_seeds=300)
    Xa, Sa = _tensors(Xs, Ss)
    S_before = Sa.cpu().clone()
    best, ms, chunk, grid = api.tune_batched(Xa, xo, Sa, so, 1.0, trials=2, precision="bf16")
    say("bf16 tuned R", best, ms, "chunk", chunk, "grid", grid)
    assert best == 2 and set(ms) == {2} and ms[2] > 0
    assert chunk in (512, 1024, 2048, 4096) and grid in (1024, 2048, 4096)
    assert torch.equal(Sa.cpu(), S_before)
    got = [t.cpu() for t in api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=4, precision="bf16")]
    explicit = [t.cpu() for t in api.step_batched(Xa, xo, Sa, so, 1.0, n_iter=4, precision="bf16",
                                                  tile_chunk=chunk, tile_grid=grid)]
    for a, b in zip(explicit, got):
        torch.testing.assert_close(b, a, rtol=0, atol=0, equal_nan=True)

"""GPU parity of ms_fit_batched -- the whole method on many clouds at once
-- against the FP64 oracle's fit of each cloud alone (cloud c draws with the
SplitMix64 state rng_seed + c): the same mode count, the same modes in the
same order, the same labels except at near-ties."""
import sys

import numpy as np
import pytest

from parity import MARGIN_TOL, MODE_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _clouds(seed, sizes, d):
    rng = np.random.default_rng(seed)
    Xs = [workloads.cloud16(rng, n, d)[0] if n else np.zeros((0, d), np.float32) for n in sizes]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    return Xs, xo


def _compare(orc, Xs, xo, h, kernel, all_points, rng_seed, per, lab, k_off):
    lab = lab.cpu().numpy() if lab is not None else None
    for c, X in enumerate(Xs):
        if len(X) == 0:
            assert k_off[c + 1] == k_off[c]
            continue
        ref = orc.fit(X, h, kernel=kernel, all_points=all_points, rng_seed=rng_seed + c)
        g = per[c].cpu().numpy().astype(np.float64)
        assert len(g) == ref.k, (c, len(g), ref.k)
        err = np.abs(g - ref.modes[:ref.k]).max()
        assert err <= MODE_TOL * h, (c, err / h)
        if lab is not None:
            gl = lab[xo[c]:xo[c + 1]]
            diff = np.nonzero(gl != ref.labels)[0]
            assert (ref.margin[diff] < MARGIN_TOL * h).all(), (c, len(diff))


@pytest.mark.parametrize("d", [2, 16])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_fit_batched_pool_matches_oracle_per_cloud(orc, d, kernel):
    sizes = [300, 0, 2500, 1, 4100, 64, 1800]
    Xs, xo = _clouds(10 * d + (kernel == "flat"), sizes, d)
    say("fit_batched", d, kernel, sizes)
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0,
                                              kernel=kernel, rng_seed=7)
    torch.cuda.synchronize()
    say("K per cloud", np.diff(k_off).tolist(), "rounds", rounds)
    _compare(orc, Xs, xo, 1.0, kernel, False, 7, per, lab, k_off)


def test_fit_batched_all_points_matches_oracle(orc):
    sizes = [700, 5, 1500]
    Xs, xo = _clouds(3, sizes, 3)
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0,
                                              all_points=True)
    torch.cuda.synchronize()
    assert rounds == 1
    _compare(orc, Xs, xo, 1.0, "gaussian", True, 0, per, lab, k_off)


def test_fit_batched_capacity_reports_counts():
    Xs, xo = _clouds(4, [400, 900], 2)
    X = torch.from_numpy(np.concatenate(Xs)).to(DEV)
    _, _, k_off, _ = api.fit_batched(X, xo, 1.0)
    with pytest.raises(api.MeanShiftError) as e:
        api.fit_batched(X, xo, 1.0, max_modes=1)
    assert e.value.code == api.MS_E_CAPACITY and e.value.k == int(k_off[-1])


def test_fit_batched_wide_rows_match_oracle(orc):
    sizes = [900, 2200, 40]
    Xs, xo = _clouds(21, sizes, 32)
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0, rng_seed=3)
    torch.cuda.synchronize()
    _compare(orc, Xs, xo, 1.0, "gaussian", False, 3, per, lab, k_off)


def test_fit_batched_no_converged_seed_is_an_error():
    Xs, xo = _clouds(5, [500, 700], 2)
    with pytest.raises(api.MeanShiftError) as e:
        api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0, max_iter=1, tol=1e-9)
    assert e.value.code == api.MS_E_NO_MODES


def test_fit_batched_repeated_calls_are_reproducible():
    # a larger batch between two equal calls: the host staging grows, and the
    # second small call must give bitwise the first one's result
    small, xo_s = _clouds(6, [300, 800], 2)
    big, xo_b = _clouds(7, [5000, 3000, 4000], 2)
    Xs = torch.from_numpy(np.concatenate(small)).to(DEV)
    Xb = torch.from_numpy(np.concatenate(big)).to(DEV)
    first = api.fit_batched(Xs, xo_s, 1.0, rng_seed=5)
    mid = api.fit_batched(Xb, xo_b, 1.0, rng_seed=5)
    again = api.fit_batched(Xs, xo_s, 1.0, rng_seed=5)
    torch.cuda.synchronize()
    assert int(mid[2][-1]) > 0
    assert np.array_equal(first[2], again[2]) and first[3] == again[3]
    for a, b in zip(first[0], again[0]):
        assert torch.equal(a, b)
    assert torch.equal(first[1], again[1])


def test_fit_batched_many_clouds_host_threads_match_oracle(orc):
    # enough seeds in a round (>= 16,384) that the draws and merges run on
    # several host threads
    rng = np.random.default_rng(11)
    sizes = [int(v) for v in rng.integers(400, 900, 160)]
    Xs, xo = _clouds(12, sizes, 2)
    assert sum(min(n, 128) for n in sizes) >= 16384
    say("fit_batched threaded", len(sizes), int(xo[-1]))
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0,
                                              rng_seed=9)
    torch.cuda.synchronize()
    _compare(orc, Xs, xo, 1.0, "gaussian", False, 9, per, lab, k_off)


@pytest.mark.parametrize("all_points", [False, True])
def test_fit_batched_merge_chains(orc, all_points):
    """Isolated points on lines 5h apart with merge radius 6h: each seed stays
    on its point, and every merge decision waits on the previous link of its
    chain, so the device passes run as deep as the longest chain (each pass
    settles the first undecided seed of every cloud); the greedy result must
    be the sequential rule's, cloud by cloud."""
    rng = np.random.default_rng(5)
    Xs = []
    for n in (300, 7, 120, 1, 260):
        X = np.zeros((n, 2), np.float32)
        X[:, 0] = 5.0 * np.arange(n, dtype=np.float32)
        X[:, 1] = float(rng.integers(0, 100))
        Xs.append(X[rng.permutation(n)] if n > 1 else X)
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0,
                                              kernel="flat", merge_radius=6.0, all_points=all_points, rng_seed=3)
    torch.cuda.synchronize()
    say("chains: K per cloud", np.diff(k_off).tolist(), "rounds", rounds)
    lab = lab.cpu().numpy()
    for c, X in enumerate(Xs):
        ref = orc.fit(X, 1.0, kernel="flat", merge_radius=6.0, all_points=all_points, rng_seed=3 + c)
        g = per[c].cpu().numpy().astype(np.float64)
        assert len(g) == ref.k, (c, len(g), ref.k)
        assert np.abs(g - ref.modes[:ref.k]).max() <= MODE_TOL, c
        diff = np.nonzero(lab[xo[c]:xo[c + 1]] != ref.labels)[0]
        assert (ref.margin[diff] < MARGIN_TOL).all(), (c, len(diff))


@pytest.mark.parametrize("d", [5, 8, 16, 32])
def test_fit_batched_bf16_matches_oracle_per_cloud(orc, d):
    """The BF16 form of the batched step inside the whole method: each cloud's
    fit against the oracle's fit of that cloud alone (the modes within
    1e-4 h, the same K and order, labels except at near-ties)."""
    sizes = [300, 0, 2500, 1, 4100, 64, 1800, 257]
    Xs, xo = _clouds(40 + d, sizes, d)
    say("fit_batched bf16", d, sizes)
    per, lab, k_off, rounds = api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0,
                                              rng_seed=11, precision="bf16")
    torch.cuda.synchronize()
    say("K per cloud", np.diff(k_off).tolist(), "rounds", rounds)
    _compare(orc, Xs, xo, 1.0, "gaussian", False, 11, per, lab, k_off)


def test_fit_batched_bf16_all_points_and_repeat(orc):
    """Every point a seed (one round of the batched BF16 step over all of a
    cloud's points) against the oracle; a second call gives the same bits."""
    Xs, xo = _clouds(8, [700, 5, 1500, 300], 16)
    X = torch.from_numpy(np.concatenate(Xs)).to(DEV)
    first = api.fit_batched(X, xo, 1.0, all_points=True, precision="bf16")
    torch.cuda.synchronize()
    assert first[3] == 1
    _compare(orc, Xs, xo, 1.0, "gaussian", True, 0, first[0], first[1], first[2])
    again = api.fit_batched(X, xo, 1.0, all_points=True, precision="bf16")
    torch.cuda.synchronize()
    assert np.array_equal(first[2], again[2])
    for a, b in zip(first[0], again[0]):
        assert torch.equal(a, b)
    assert torch.equal(first[1], again[1])


def test_fit_batched_bf16_rejects_what_is_not_built():
    Xs, xo = _clouds(3, [300, 500], 3)
    with pytest.raises(api.MeanShiftError, match="Gaussian kernel at 5 <= d <= 32"):
        api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0, precision="bf16")
    Xs, xo = _clouds(3, [300, 500], 16)
    with pytest.raises(api.MeanShiftError, match="Gaussian kernel at 5 <= d <= 32"):
        api.fit_batched(torch.from_numpy(np.concatenate(Xs)).to(DEV), xo, 1.0, kernel="flat", precision="bf16")

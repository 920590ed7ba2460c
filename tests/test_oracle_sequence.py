"""Pins of the frame-sequence seed-count rule (Section II-D) and of the image
workload, on the CPU: the oracle's behaviour against what the paper states,
and the library's host-side rule against the oracle's."""
import numpy as np
import pytest

from paper_2112_13891_amd import workloads


def test_warm_start_runs_one_round_on_a_steady_scene(orc):
    """Frame 0 starts at N = 128 and doubles while N < L*M (three rounds for
    ~40 blobs); every later frame of the same scene starts at the count the
    previous one ended with, which already satisfies N >= L*M: one round."""
    frames = workloads.frames2d(seed=0, n=8000, n_frames=3, change_at=99)
    res, starts = orc.fit_sequence([f.X for f in frames], 5.0)
    assert list(res[0].round_N) == [128, 256, 512]
    assert starts == [128, 512, 512]
    for r in res[1:]:
        assert list(r.round_N) == [512]
        assert 8 * r.k <= 512 <= 32 * r.k


def test_quiet_scene_sheds_seeds_gradually(orc):
    """After the scene drops to 4 blobs, N = 512 exceeds H*M = 128, so each
    frame starts M = 4 seeds lower than the previous one; the frame itself
    still runs one round (N >= L*M)."""
    frames = workloads.frames2d(seed=0, n=8000, n_frames=6, change_at=2, k_after=4)
    res, starts = orc.fit_sequence([f.X for f in frames], 5.0)
    ks = [r.k for r in res]
    assert ks[2:] == [4, 4, 4, 4]
    assert starts[2] == 512
    assert starts[3:] == [508, 504, 500]
    assert all(len(r.round_N) == 1 for r in res[2:])


def test_seed_count_rule_edges(orc):
    # H*M exactly: not larger, no change; one below: shrinks by M
    assert orc.next_seed_count(512, 16, 32) == 512
    assert orc.next_seed_count(512, 15, 32) == 497
    # no modes: nothing to shed; the count never drops below one seed
    assert orc.next_seed_count(300, 0, 32) == 300
    assert orc.next_seed_count(2, 1, 1) == 1


def test_library_rule_matches_oracle(orc):
    from paper_2112_13891_amd import api
    for N in (1, 2, 31, 32, 33, 128, 500, 512, 4096, 2 ** 31 - 1):
        for M in (0, 1, 2, 15, 16, 17, 100, 4096):
            for H in (1, 8, 32):
                assert api.seed_count_next(N, M, H) == orc.next_seed_count(N, M, H), (N, M, H)
    for bad in ((0, 1, 32), (5, -1, 32), (5, 1, 0)):
        with pytest.raises(RuntimeError):
            api.seed_count_next(*bad)


def test_image_workload_shape():
    w = workloads.image_rgb(seed=0, side=64, regions=6)
    assert w.X.shape == (4096, 3) and w.X.dtype == np.float32
    assert w.X.min() >= 0.0 and w.X.max() <= 255.0
    # raster order: the region map is piecewise constant along rows
    lab = w.y.reshape(64, 64)
    assert (lab[:, 1:] == lab[:, :-1]).mean() > 0.9
    assert set(np.unique(w.y)) <= set(range(6))


def test_image_fit_recovers_regions(orc):
    """Region colours with per-channel noise 6 and h = 12: every mode lies
    near a region colour (clipping at 0 and 255 pulls a mode inward by a few
    units), and every large region whose colour is far from all others has a
    mode of its own."""
    w = workloads.image_rgb(seed=0, side=96, regions=10)
    r = orc.fit(w.X, w.h)
    present = np.unique(w.y)
    cols = w.extra["colours"][present]
    sizes = np.bincount(w.y)[present]
    d = np.linalg.norm(r.modes[:, None, :] - cols[None, :, :], axis=2)
    assert (d.min(axis=1) < w.h).all()
    sep = np.linalg.norm(cols[:, None] - cols[None], axis=2)
    np.fill_diagonal(sep, np.inf)
    for c in range(len(cols)):
        if sizes[c] >= 500 and sep[c].min() > 3 * w.h:
            assert d[:, c].min() < w.h, c

"""Full-size parity in the launch shapes the bench times.

* The whole method on the 262,144 x 32 embedding workload (Gaussian, h = 1.5,
  seed 0), FP32 and BF16, against the oracle's fit stored by
  tests/golden/make_embed32_fit.py (Algorithm 2 with Section II-C/D): the
  same drawn ids per round, the same K, every drawn seed's final position,
  the modes within 1e-4 h, the labels except at near-ties.
* The flat window on a 33,000-point slice of the same workload: every window
  holds one point, so K = n and the round of 16,384 seeds takes the tiled
  merge; against the oracle's fit.
* The largest step launch of that fit: 8,192 seeds over all 262,144 points
  (radix seed order, many seed tiles), a 256-seed sample against the
  oracle's trajectories.
* The whole method on the 512 uneven clouds in one ms_fit_batched call, FP32
  and BF16: the smallest, the largest and six random clouds against the
  oracle's fit of each cloud alone.
"""
import os
import sys

import numpy as np
import pytest

from parity import MARGIN_TOL, MODE_TOL, fit_parity, step_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "embed32_gauss_fit.npz")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def embed():
    return workloads.embed32(seed=0)


class StoredFit:
    """The oracle's fit as stored by tests/golden/make_embed32_fit.py, with
    the fields fit_parity reads.  Margins are stored for the points whose
    two-mode margin is below 1e-3 h; every other point's margin is larger."""

    def __init__(self, path, n):
        z = np.load(path, allow_pickle=False)
        self.k = int(z["k"])
        self.modes = z["modes"]
        self.labels = z["labels"].astype(np.int64)
        self.margin = np.full(n, np.inf)
        self.margin[z["near_idx"]] = z["near_margin"]
        self.round_N = z["round_N"]
        self.round_B = z["round_B"]
        self.drawn = z["drawn"]
        self.drawn_iters = z["drawn_iters"]
        self.drawn_status = z["drawn_status"]
        self.drawn_final = z["drawn_final"].astype(np.float64)
        self.pairs = int(z["pairs"])

    def rounds(self):
        out, o = [], 0
        for b in self.round_B:
            out.append(self.drawn[o:o + b])
            o += b
        return out


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fit_embed32_gaussian_vs_stored_oracle(orc, embed, precision):
    say("fit embed32 gaussian", precision)
    ref = StoredFit(GOLDEN, embed.n)
    g = api.fit(_gpu(embed.X), embed.h, precision=precision, trace=True)
    rep = fit_parity(g, ref, embed.X, embed.h, orc=orc)
    say("embed32", precision, rep, "K", g.k, "rounds", g.round_N.tolist(), "pairs", g.pairs,
        "exact pairs", g.refined_pairs, "ms", round(g.total_ms, 2))


@pytest.fixture(scope="module")
def flat_slice(orc, embed):
    X = embed.X[:33_000]
    say("oracle fit of the flat slice")
    return X, orc.fit(X, embed.h, kernel="flat")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fit_embed32_flat_slice_tiled_merge(orc, embed, flat_slice, precision):
    X, ref = flat_slice
    say("fit embed32 flat slice", precision)
    g = api.fit(_gpu(X), embed.h, kernel="flat", precision=precision, trace=True)
    assert g.round_B.max() >= 16_384   # the round that takes the tiled merge
    rep = fit_parity(g, ref, X, embed.h, orc=orc, kernel="flat")
    say("embed32 flat slice", precision, rep, "K", g.k, "rounds", g.round_B.tolist())
    assert g.k == len(X)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_step_embed32_8192_seeds(orc, embed, kernel, precision):
    rng = np.random.default_rng(8192)
    idx = rng.choice(embed.n, 8192, replace=False)
    S0 = embed.X[idx]
    say("step embed32 8192 seeds", kernel, precision)
    S, conv, it, sh = api.step(_gpu(embed.X), _gpu(S0), embed.h, kernel=kernel, precision=precision,
                               n_iter=100)
    torch.cuda.synchronize()
    S, conv, it = S.cpu().numpy(), conv.cpu().numpy(), it.cpu().numpy()
    sample = np.sort(rng.choice(8192, 256, replace=False))
    rep = step_parity(orc, embed.X, S0[sample], embed.h, kernel, 1e-3, S[sample], it[sample],
                      conv[sample])
    say(rep, "converged", int((conv == 1).sum()), "of 8192")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fit_batched_512_clouds_sampled(orc, precision):
    clouds = workloads.clouds16(seed=0)
    Xs = [c[0] for c in clouds]
    xo = np.concatenate([[0], np.cumsum([len(x) for x in Xs])]).astype(np.int64)
    say("fit_batched 512 clouds", int(xo[-1]), "points", precision)
    per, lab, k_off, rounds = api.fit_batched(_gpu(np.concatenate(Xs)), xo, 1.0, precision=precision)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    sizes = np.array([len(x) for x in Xs])
    rng = np.random.default_rng(512)
    pick = {int(sizes.argmin()), int(sizes.argmax())}
    while len(pick) < 8:
        pick.add(int(rng.integers(0, len(Xs))))
    for c in sorted(pick):
        ref = orc.fit(Xs[c], 1.0, rng_seed=c)
        g = per[c].cpu().numpy().astype(np.float64)
        assert len(g) == ref.k, (c, len(g), ref.k)
        err = np.abs(g - ref.modes[:ref.k]).max()
        assert err <= MODE_TOL, (c, err)
        gl = lab[xo[c]:xo[c + 1]]
        diff = np.nonzero(gl != ref.labels)[0]
        assert (ref.margin[diff] < MARGIN_TOL).all(), (c, len(diff))
        say("cloud", c, "n", len(Xs[c]), "K", ref.k, "max mode err/h", err, "label diffs", len(diff))

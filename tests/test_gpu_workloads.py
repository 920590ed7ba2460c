"""GPU parity on the image-shaped workload (RGB pixels, Section I, Fig. 1) and
on frame sequences with the seed-count adaptation of Section II-D."""
import sys

import numpy as np
import pytest

from parity import fit_parity, step_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_image_fit_128(orc, precision):
    w = workloads.image_rgb(seed=0, side=128)
    g = api.fit(_gpu(w.X), w.h, precision=precision, trace=True)
    ref = orc.fit(w.X, w.h)
    rep = fit_parity(g, ref, w.X, w.h, orc=orc)
    say("image 128^2", precision, rep, "K", g.k, "rounds", g.round_N.tolist())


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_image_step_512_sample(orc, precision):
    """512^2 pixels (262,144 points): 256 pixels as seeds, to convergence."""
    w = workloads.image_rgb(seed=1, side=512)
    rng = np.random.default_rng(2)
    S0 = w.X[rng.choice(w.n, 256, replace=False)]
    S, conv, it, sh = api.step(_gpu(w.X), _gpu(S0), w.h, precision=precision, tol=1e-3, n_iter=100)
    torch.cuda.synchronize()
    rep = step_parity(orc, w.X, S0, w.h, "gaussian", 1e-3, S.cpu().numpy(), it.cpu().numpy(),
                      conv.cpu().numpy())
    say("image 512^2 step", precision, rep)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_frame_sequence(orc, precision):
    """Six frames: drifting blobs, then a quieter scene.  The seed count each
    frame starts with, and every frame's clustering, match the oracle."""
    frames = workloads.frames2d(seed=0)
    gres, gstarts = api.fit_sequence([_gpu(f.X) for f in frames], 5.0, precision=precision, trace=True)
    ores, ostarts = orc.fit_sequence([f.X for f in frames], 5.0)
    say("frame starts", gstarts, ostarts)
    assert gstarts == ostarts
    for f, (g, o) in enumerate(zip(gres, ores)):
        rep = fit_parity(g, o, frames[f].X, 5.0, orc=orc)
        say("frame", f, "rounds", g.round_N.tolist(), "K", g.k, rep)
    # a warm-started frame of a steady scene runs one round
    assert all(len(g.round_N) == 1 for g in gres[1:])

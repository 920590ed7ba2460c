"""GPU parity of the merge for large batches (the tiled decision pass, taken
from 16,384 seeds up): every point is a seed (Algorithm 1) and the flat
window is narrow, so most seeds found their own mode while neighbours within
the merge radius join the first founder, in draw order -- the greedy rule
decides every mode and label.  Compared mode by mode with the FP64 oracle."""
import sys

import numpy as np
import pytest

from parity import MARGIN_TOL, MODE_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,d", [(20000, 2), (17000, 16)])
def test_large_batch_merge_matches_oracle(orc, n, d):
    rng = np.random.default_rng(n + d)
    if d == 2:
        # uniform points, h at 0.6 of the mean spacing: chains of neighbours
        X = np.ascontiguousarray(rng.uniform(0.0, 100.0, (n, d)), dtype=np.float32)
        h = float(0.6 * (100.0 ** d / n) ** 0.5)
    else:
        # groups of 1-3 points within 0.03 of far-apart centres: every group
        # converges to its mean and all but its first seed join it
        C = rng.uniform(0.0, 100.0, (n, d))
        y = np.sort(rng.integers(0, int(n * 0.55), n))
        X = np.ascontiguousarray(C[y] + 0.01 * rng.standard_normal((n, d)), dtype=np.float32)
        X = X[rng.permutation(n)]
        h = 0.1
    say("large merge", n, d, "h", h)
    g = api.fit(torch.from_numpy(X).to(DEV), h, kernel="flat", all_points=True)
    ref = orc.fit(X, h, kernel="flat", all_points=True)
    say("K gpu", g.k, "oracle", ref.k)
    assert g.k == ref.k
    assert g.k > n // 4   # many modes: the batch decides most of them itself
    gm = g.modes.detach().cpu().numpy().astype(np.float64)
    err = np.abs(gm - ref.modes[:g.k]).max()   # modes are created in draw order on both sides
    assert err <= MODE_TOL * h, err / h
    gl = g.labels.detach().cpu().numpy()
    diff = np.nonzero(gl != ref.labels)[0]
    assert (ref.margin[diff] < MARGIN_TOL * h).all(), (len(diff), ref.margin[diff][:5])

"""The block join that the fit uses once modes number in the thousands (the
merge against the old modes, the pool coverage, and the labels; spatially
ordered points and modes, only nearby blocks compared): its labels equal the
brute-force nearest-mode labelling of ms_assign on the same modes, element by
element, and a fit that goes through every join matches the FP64 oracle
(Algorithms 1-2: prune modes, cluster by distance to modes)."""
import os
import sys

import numpy as np
import pytest

from parity import fit_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api  # noqa: E402

DEV = "cuda:0"
JOIN_MIN = 4096   # modes (and seeds) from which the fit takes the join


@pytest.fixture(autouse=True)
def join_always():
    """These sizes are below the pair count from which the fit prefers the
    join for the merge and the coverage: the override makes it take the join
    wherever both sides have JOIN_MIN rows (the library reads it per call)."""
    old = os.environ.get("MS_JOIN_PAIRS")
    os.environ["MS_JOIN_PAIRS"] = "0"
    yield
    if old is None:
        del os.environ["MS_JOIN_PAIRS"]
    else:
        os.environ["MS_JOIN_PAIRS"] = old


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def sparse(seed, n, d, side):
    """Uniform points whose typical spacing is well above h: nearly every
    window holds one point, so nearly every seed founds a mode."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, side, (n, d)), dtype=np.float32)


@pytest.mark.parametrize("n,d,side,h,kernel", [(20011, 2, 100.0, 0.1, "flat"),
                                               (12000, 8, 10.0, 0.3, "gaussian"),
                                               (9000, 16, 10.0, 0.5, "flat"),
                                               (16500, 32, 10.0, 0.6, "gaussian")])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_join_labels_equal_bruteforce(n, d, side, h, kernel, precision):
    X = sparse(n + d, n, d, side)
    say("join labels", n, d, kernel, precision)
    g = api.fit(_gpu(X), h, kernel=kernel, precision=precision, trace=True)
    torch.cuda.synchronize()
    assert g.k >= JOIN_MIN, g.k
    ref = api.assign(_gpu(X), g.modes.contiguous())
    torch.cuda.synchronize()
    diff = int((g.labels != ref).sum())
    say("K", g.k, "rounds", g.round_B.tolist(), "labels differing", diff)
    assert diff == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_join_fit_matches_oracle(orc, precision):
    # rounds of 4,096 and 8,192 seeds after 8,064 modes: the match against
    # the old modes, the coverage and the labels all go through the join
    X = sparse(7, 20000, 8, 10.0)
    h = 0.3
    g = api.fit(_gpu(X), h, kernel="flat", precision=precision, trace=True)
    assert g.round_B.max() >= 8192 and g.k >= 8192, (g.round_B.tolist(), g.k)
    ref = orc.fit(X, h, kernel="flat")
    rep = fit_parity(g, ref, X, h, orc=orc, kernel="flat")
    say("join fit", precision, rep, "K", g.k, "rounds", g.round_B.tolist())

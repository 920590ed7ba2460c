"""GPU parity of the cosine-metric form (directions of the rows, unit-vector
seeds and modes, chord radii) against the FP64 oracle."""
import sys

import numpy as np
import pytest

from parity import fit_parity, ragged_check, step_parity

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


def _unit(a):
    a = np.asarray(a, np.float64)
    return a / np.linalg.norm(a, axis=1, keepdims=True)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_cosine_step_embed32_sample(orc, precision):
    w = workloads.embed_cos(seed=0)
    rng = np.random.default_rng(1)
    S0 = w.X[rng.choice(w.n, 256, replace=False)]
    S, conv, it, sh = api.step(_gpu(w.X), _gpu(S0), w.h, precision=precision, n_iter=100, metric="cosine")
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-5)
    rep = step_parity(orc, w.X, _unit(S0), w.h, "gaussian", 1e-3, S, it.cpu().numpy(), conv.cpu().numpy(),
                      metric="cosine")
    say("cosine step embed32", precision, rep)


@pytest.mark.parametrize("n,d", [(1, 2), (100, 3), (4099, 4), (20011, 3), (3000, 16), (1500, 32)])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_cosine_step_ragged(orc, n, d, kernel):
    rng = np.random.default_rng(n + d)
    X = (rng.standard_normal((n, d)) + 2.0 * (np.arange(d) == 0)).astype(np.float32)
    X *= rng.uniform(0.2, 5.0, (n, 1)).astype(np.float32)
    m = min(n, 200)
    S0 = X[rng.choice(n, m, replace=False)]
    h = 0.6
    for precision in (("fp32", "bf16") if d <= 32 else ("fp32",)):
        for n_iter in (1, 3):
            S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, precision=precision,
                                       n_iter=n_iter, metric="cosine")
            torch.cuda.synchronize()
            ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter,
                                          metric="cosine")
            # ragged_check works in the units of X: compare on the directions
            ties = ragged_check(orc, _unit(X).astype(np.float32), _unit(S0).astype(np.float32), h, kernel,
                                n_iter, S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy(), ref, oit,
                                ost, metric="cosine")
            if ties:
                say("flat boundary ties", ties)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_cosine_fit(orc, precision):
    w = workloads.embed_cos(seed=3, n=20000, k=12, d=16)
    g = api.fit(_gpu(w.X), w.h, precision=precision, metric="cosine", trace=True)
    ref = orc.fit(w.X, w.h, metric="cosine")
    U = _unit(w.X).astype(np.float32)
    rep = fit_parity(g, ref, U, w.h, orc=None)
    say("cosine fit", precision, rep, "K", g.k, "rounds", g.round_N.tolist())
    M = g.modes.cpu().numpy()
    assert np.allclose(np.linalg.norm(M, axis=1), 1.0, atol=1e-5)


def test_cosine_fit_rejects_zero_rows():
    X = np.ones((5000, 3), np.float32)
    X[17] = 0.0
    with pytest.raises(api.MeanShiftError):
        api.fit(_gpu(X), 0.5, metric="cosine")

"""ms_step_noalloc (workspace in the library's fixed device scratch) against
ms_step, through the C ABI: the same kernels on the same inputs give the same
bits.  Two calls in a row on each form, the second with a smaller input (the
scratch keeps the first call's contents), and a call too large for the
scratch is refused before anything runs."""
import sys

import numpy as np
import pytest

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


def _clustered(seed, n, d, k=8):
    rng = np.random.default_rng(seed)
    C = 4.0 * rng.standard_normal((k, d))
    y = rng.integers(0, k, n)
    return (C[y] + 0.5 * rng.standard_normal((n, d))).astype(np.float32)


def _same(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y)


CASES = [
    # (name, X builder, h, seeds, kernel, precision, iterations)
    ("aniso3d 100K fp32", lambda: workloads.aniso3d(seed=0).X[:100_000], 15.0, 512, "gaussian", "fp32", 100),
    ("aniso3d 20K fp32", lambda: workloads.aniso3d(seed=0).X[100_000:120_000], 15.0, 100, "gaussian", "fp32", 100),
    ("aniso3d 100K bf16", lambda: workloads.aniso3d(seed=0).X[:100_000], 15.0, 512, "gaussian", "bf16", 100),
    ("aniso3d 20K bf16", lambda: workloads.aniso3d(seed=0).X[100_000:120_000], 15.0, 100, "gaussian", "bf16", 100),
    ("16-D 30K fp32 flat", lambda: _clustered(3, 30_000, 16), 1.5, 300, "flat", "fp32", 5),
    ("16-D 5K fp32 flat", lambda: _clustered(4, 5_000, 16), 1.5, 77, "flat", "fp32", 5),
    ("16-D 30K bf16", lambda: _clustered(3, 30_000, 16), 1.5, 300, "gaussian", "bf16", 20),
    ("16-D 5K bf16", lambda: _clustered(4, 5_000, 16), 1.5, 77, "gaussian", "bf16", 20),
    ("5-D 3K plain", lambda: _clustered(5, 3_001, 5), 1.0, 65, "gaussian", "fp32", 10),
]


@pytest.mark.parametrize("first,second", [(0, 1), (2, 3), (4, 5), (6, 7), (8, 1)])
def test_noalloc_matches_step_twice(first, second):
    for idx in (first, second):
        name, mk, h, m, kernel, prec, n_iter = CASES[idx]
        say("noalloc vs step:", name)
        X = mk()
        rng = np.random.default_rng(idx)
        S0 = _gpu(X[rng.choice(len(X), m, replace=False)])
        Xg = _gpu(X)
        plain = name.endswith("plain")
        ref = api.step(Xg, S0, h, kernel=kernel, precision=prec, n_iter=n_iter, plain=plain)
        got = api.step(Xg, S0, h, kernel=kernel, precision=prec, n_iter=n_iter, plain=plain,
                       noalloc=True)
        torch.cuda.synchronize()
        _same(got, ref)
        assert int((got[2] > 0).sum()) == m


def test_noalloc_refuses_oversized_call():
    X = torch.zeros((262_144, 32), dtype=torch.float32, device=DEV)
    S0 = X[:64].clone()
    with pytest.raises(api.MeanShiftError) as e:
        api.step(X, S0, 1.5, n_iter=1, noalloc=True)
    assert e.value.code == api.MS_E_INVALID and "scratch" in str(e.value)
    # the library is still usable afterwards
    Y = _gpu(_clustered(9, 2_000, 3))
    a = api.step(Y, Y[:50].clone(), 1.0, n_iter=3, noalloc=True)
    b = api.step(Y, Y[:50].clone(), 1.0, n_iter=3)
    torch.cuda.synchronize()
    _same(a, b)

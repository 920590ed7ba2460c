"""GPU parity of the spatially ordered forms against the FP64 oracle: the FP32
step with block culling (d <= 32, n >= 16,384) and the BF16 form with its block
culling, on clustered layouts where most blocks are far from most seeds (so
whole blocks are skipped) and on ragged point counts (partial last block)."""
import sys

import numpy as np
import pytest

from parity import fit_parity, ragged_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def clustered(seed, n, d, k=30, box=200.0, sigma=1.0):
    """k blobs far apart relative to h = 1.5 (box 200 per axis), so that most
    blocks are far from most seeds."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, box, (k, d))
    y = rng.integers(0, k, n)
    X = C[y] + sigma * rng.standard_normal((n, d))
    return np.ascontiguousarray(X[rng.permutation(n)], dtype=np.float32)


@pytest.mark.parametrize("n", [16384, 16385, 20011, 65537])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 16, 29, 32])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_culled_step_ragged(orc, n, d, kernel, precision):
    say("culled step", precision, n, d, kernel)
    X = clustered(n * 10 + d, n, d)
    rng = np.random.default_rng(n + d)
    S0 = X[rng.choice(n, 300, replace=False)]
    h = 1.5
    for n_iter in (1, 3):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, precision=precision, n_iter=n_iter)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=n_iter)
        ties = ragged_check(orc, X, S0, h, kernel, n_iter, S.cpu().numpy(), it.cpu().numpy(),
                            conv.cpu().numpy(), ref, oit, ost)
        if ties:
            say("flat boundary ties", ties)


@pytest.mark.parametrize("m", [1, 63, 64, 65, 700, 4097])
def test_culled_step_seed_counts(orc, m):
    """Tile tails: seed counts around the 64-seed tile and above the one-
    workgroup seed sort."""
    n, d = 40000, 3
    X = clustered(5, n, d)
    rng = np.random.default_rng(m)
    S0 = X[rng.choice(n, m, replace=False)]
    for precision in ("fp32", "bf16"):
        S, conv, it, sh = api.step(_gpu(X), _gpu(S0), 1.5, precision=precision, n_iter=2)
        torch.cuda.synchronize()
        ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), 1.5, "gaussian", tol=1e-3, n_iter=2)
        ragged_check(orc, X, S0, 1.5, "gaussian", 2, S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy(),
                     ref, oit, ost)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_culled_fit(orc, kernel, precision):
    X = clustered(11, 30000, 2)
    g = api.fit(_gpu(X), 1.5, kernel=kernel, precision=precision, trace=True)
    ref = orc.fit(X, 1.5, kernel=kernel)
    rep = fit_parity(g, ref, X, 1.5, orc=orc, kernel=kernel)
    say("culled fit", kernel, precision, rep, "K", g.k, "rounds", g.round_N.tolist())


def test_culled_step_deterministic():
    X = _gpu(clustered(3, 50000, 3))
    S0 = X[:512].clone()
    for precision in ("fp32", "bf16"):
        a = api.step(X, S0, 1.5, precision=precision, n_iter=4)[0]
        b = api.step(X, S0, 1.5, precision=precision, n_iter=4)[0]
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("d", [3, 16])
@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_plain_fp32_form_matches_oracle_and_culled_form(orc, d, kernel):
    """plain=1 runs every pair in input order: oracle parity, and the culled
    form differs from it only by summation order (culled blocks add exact
    zeros)."""
    n = 20011
    say("plain form", d, kernel)
    X = clustered(700 + d, n, d)
    rng = np.random.default_rng(d)
    S0 = X[rng.choice(n, 300, replace=False)]
    h = 1.5
    Sp, cp, ip, _ = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, n_iter=3, plain=True)
    Sc, cc, ic, _ = api.step(_gpu(X), _gpu(S0), h, kernel=kernel, n_iter=3)
    torch.cuda.synchronize()
    ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, kernel, tol=1e-3, n_iter=3)
    ragged_check(orc, X, S0, h, kernel, 3, Sp.cpu().numpy(), ip.cpu().numpy(), cp.cpu().numpy(), ref, oit, ost)
    assert np.abs(Sp.cpu().numpy() - Sc.cpu().numpy()).max() <= 1e-4 * h
    rp = api.fit(_gpu(X), h, kernel=kernel, plain=True)
    rc = api.fit(_gpu(X), h, kernel=kernel)
    assert rp.k == rc.k


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("m", [64, 700])
def test_reduce_paths_at_many_chunks(orc, plain, m):
    """D = 3 at 300,007 points: up to 1,172 (plain, 256-point chunks) or 586
    (culled, 512-point chunks) chunk partials per seed, more than the
    one-launch reduce-and-finalize takes (2,048 floats per slot), so the
    spread reduction and the separate finalize run (every smaller case here
    takes the one-launch form).  Both match the oracle."""
    n, d, h = 300007, 3, 1.5
    say("reduce paths", "plain" if plain else "culled", m)
    X = clustered(4242, n, d, k=60, box=400.0)
    rng = np.random.default_rng(m)
    S0 = X[rng.choice(n, m, replace=False)]
    S, conv, it, sh = api.step(_gpu(X), _gpu(S0), h, n_iter=2, plain=plain)
    torch.cuda.synchronize()
    ref, ost, oit, osh = orc.step(X, S0.astype(np.float64), h, "gaussian", tol=1e-3, n_iter=2)
    ragged_check(orc, X, S0, h, "gaussian", 2, S.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy(),
                 ref, oit, ost)


def test_bf16_flat_step_repeatable():
    # a tile of the flat BF16 form is processed only for lanes holding a seed:
    # a lane past the active count once forced tiles whose points were not in
    # LDS, and a NaN left there by an earlier kernel spread into live seeds'
    # sums (even at weight 0), now and then
    n, d, h = 65537, 6, 1.5
    X = clustered(n * 10 + d, n, d)
    rng = np.random.default_rng(n + d)
    S0 = X[rng.choice(n, 300, replace=False)]
    Xg, Sg = _gpu(X), _gpu(S0)
    first = None
    for rep in range(16):
        S, conv, it, sh = api.step(Xg, Sg, h, kernel="flat", precision="bf16", n_iter=2)
        torch.cuda.synchronize()
        out = (S.cpu().numpy(), conv.cpu().numpy(), it.cpu().numpy())
        assert np.isfinite(out[0]).all() and (out[1] != 2).all(), rep
        if first is None:
            first = out
        else:
            assert all(np.array_equal(a, b) for a, b in zip(first, out)), rep


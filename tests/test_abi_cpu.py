"""CPU-only checks of the C ABI: the library loads, exports every entry point
the header declares, its ctypes layouts match the C header, argument
validation fails cleanly before any GPU work, and the host-side seed draw
equals the oracle's independently written draw."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fms.h")


@pytest.fixture(scope="module")
def api():
    from paper_2112_13891_amd import api as a
    if not os.path.exists(a.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    a.lib()
    return a


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*(ms_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported(api):
    names = _declared()
    assert {"ms_fit", "ms_step", "ms_assign", "ms_last_error"} <= set(names)
    L = ctypes.CDLL(api.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(api.EXPORTS) == set(names)


def test_struct_layout_matches_header(api, tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "fms.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ms_params), '
        'offsetof(ms_params, check_finite), sizeof(ms_diag), offsetof(ms_diag, pairs), '
        'offsetof(ms_diag, drawn), offsetof(ms_diag, counts)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(probe), "-o", str(exe)],
                   check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    P, D = api.Params, api.Diag
    want = [ctypes.sizeof(P), P.check_finite.offset, ctypes.sizeof(D), D.pairs.offset,
            D.drawn.offset, D.counts.offset]
    assert got == want


def test_default_params(api):
    p = api.Params()
    api.lib().ms_default_params(ctypes.byref(p))
    assert (p.h, p.kernel, p.precision, p.max_iter, p.n_initial, p.L) == (1.0, 1, 0, 100, 128, 8)
    assert abs(p.tol - 1e-3) < 1e-9 and p.gamma == 1.0 and p.merge_radius == 1.0


FAKE = ctypes.c_void_p(4096)   # never dereferenced: validation fails first


@pytest.mark.parametrize("field,value,msg", [
    ("h", 0.0, "h must"), ("h", float("nan"), "h must"), ("h", float("inf"), "h must"),
    ("tol", 0.0, "tol must"), ("max_iter", 0, "max_iter"), ("max_iter", 5000, "max_iter"),
    ("gamma", 0.0, "gamma"), ("gamma", 1.5, "gamma"), ("n_initial", 0, "n_initial"),
    ("L", 0, "L must"), ("kernel", 7, "kernel"), ("precision", 9, "precision"),
    ("merge_radius", -1.0, "merge_radius"), ("cover_radius", float("nan"), "cover_radius"),
])
def test_fit_rejects_bad_params(api, field, value, msg):
    p = api.make_params(1.0)
    setattr(p, field, value)
    k = ctypes.c_int32(0)
    rc = api.lib().ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None)
    assert rc == api.MS_E_INVALID and msg in api.last_error()


@pytest.mark.parametrize("n,d,msg", [(0, 2, "n must"), (10, 0, "d must"), (10, 257, "d must"),
                                     (2 ** 31, 2, "n must")])
def test_fit_rejects_bad_shapes(api, n, d, msg):
    p = api.make_params(1.0)
    k = ctypes.c_int32(0)
    rc = api.lib().ms_fit(ctypes.byref(p), FAKE, n, d, FAKE, 4, ctypes.byref(k), None, None, None)
    assert rc == api.MS_E_INVALID and msg in api.last_error()


def test_null_pointers_and_reserved(api):
    L = api.lib()
    p = api.make_params(1.0)
    k = ctypes.c_int32(0)
    assert L.ms_fit(ctypes.byref(p), None, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert L.ms_fit(None, FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert L.ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 0, ctypes.byref(k), None, None, None) == -1
    p.reserved[0] = 1
    assert L.ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert "reserved" in api.last_error()
    p = api.make_params(1.0)
    p.tile_R = 3
    assert L.ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert "tile_R" in api.last_error()
    p = api.make_params(1.0)
    p.plain = 2
    assert L.ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert "plain" in api.last_error()
    p = api.make_params(1.0)
    p.graph = 2
    assert L.ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None) == -1
    assert "graph" in api.last_error()
    p = api.make_params(1.0)
    assert L.ms_step(ctypes.byref(p), FAKE, 10, 2, FAKE, -1, 1, FAKE, FAKE, FAKE, None) == -1
    assert L.ms_step(ctypes.byref(p), FAKE, 10, 2, FAKE, 3, 5000, FAKE, FAKE, FAKE, None) == -1
    assert L.ms_step(ctypes.byref(p), FAKE, 10, 2, FAKE, 0, 1, FAKE, FAKE, FAKE, None) == 0
    assert L.ms_assign(FAKE, 10, 2, FAKE, 0, FAKE, None, None) == -1
    assert L.ms_assign(FAKE, 10, 2, FAKE, 3, None, None, None) == -1
    assert L.ms_forward_update(FAKE, 1, 10, FAKE, 10, 2, 1.0, FAKE, 2, None) == -1
    assert L.ms_step_adjoint(FAKE, 1, 10, FAKE, 10, 2, -1.0, FAKE, FAKE, FAKE, 4, None) == -1
    assert "h must" in api.last_error()
    xo = (ctypes.c_int64 * 3)(0, 5, 10)
    so = (ctypes.c_int64 * 3)(0, 0, 0)
    best = ctypes.c_int32(0)
    assert L.ms_tune_batched(ctypes.byref(p), FAKE, xo, FAKE, so, 2, 2, 4, ctypes.byref(best), None,
                             None, None, None) == -1
    assert "no cloud has seeds" in api.last_error()
    so = (ctypes.c_int64 * 3)(0, 2, 4)
    assert L.ms_tune_batched(ctypes.byref(p), FAKE, xo, FAKE, so, 2, 2, 0, ctypes.byref(best), None,
                             None, None, None) == -1
    assert "trials" in api.last_error()
    assert L.ms_tune_batched(ctypes.byref(p), FAKE, xo, None, so, 2, 2, 4, ctypes.byref(best), None,
                             None, None, None) == -1
    assert "seeds is NULL" in api.last_error()
    kf = (ctypes.c_int64 * 3)()
    pg = api.make_params(1.0, gamma=0.5)
    assert L.ms_fit_batched(ctypes.byref(pg), FAKE, xo, 2, 2, FAKE, 10, kf, None, None, None) == -1
    assert "gamma must be 1" in api.last_error()
    assert L.ms_fit_batched(ctypes.byref(p), FAKE, xo, 2, 2, FAKE, 10, None, None, None, None) == -1
    assert "k_off" in api.last_error()
    zo = (ctypes.c_int64 * 3)(0, 0, 0)
    assert L.ms_fit_batched(ctypes.byref(p), FAKE, zo, 2, 2, FAKE, 10, kf, None, None, None) == -1
    assert "no cloud has points" in api.last_error()
    p.precision = api.PRECISIONS["bf16"]
    assert L.ms_tune_batched(ctypes.byref(p), FAKE, xo, FAKE, so, 2, 2, 4, ctypes.byref(best), None,
                             None, None, None) == -1
    assert "Gaussian kernel at 5 <= d <= 32" in api.last_error()
    assert L.ms_fit_batched(ctypes.byref(p), FAKE, xo, 2, 4, FAKE, 10, kf, None, None, None) == -1
    assert "Gaussian kernel at 5 <= d <= 32" in api.last_error()
    pf = api.make_params(1.0, kernel="flat", precision="bf16")
    assert L.ms_fit_batched(ctypes.byref(pf), FAKE, xo, 2, 16, FAKE, 10, kf, None, None, None) == -1
    assert "Gaussian kernel at 5 <= d <= 32" in api.last_error()


def test_error_message_is_thread_local_and_cleared(api):
    p = api.make_params(-1.0)
    k = ctypes.c_int32(0)
    api.lib().ms_fit(ctypes.byref(p), FAKE, 10, 2, FAKE, 4, ctypes.byref(k), None, None, None)
    assert api.last_error()
    ids, _ = api.seed_draw(1, np.arange(10, dtype=np.int32), 3)
    assert api.last_error() == ""


def test_seed_draw_matches_oracle(api, orc):
    """Seed selection (Algorithm 2, Section II-D): the library's sparse
    Fisher-Yates and the oracle's in-place one give the same ids and state."""
    rng = np.random.default_rng(0)
    for trial in range(60):
        L = int(rng.integers(0, 3000))
        pool = np.sort(rng.choice(100_000, size=L, replace=False)).astype(np.int32)
        count = int(rng.integers(0, L + 1))
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        a, sa = api.seed_draw(seed, pool, count)
        b, sb = orc.draw(seed, pool, count)
        assert np.array_equal(a, b) and sa == sb
    with pytest.raises(api.MeanShiftError):
        api.seed_draw(0, np.arange(3, dtype=np.int32), 4)


def test_step_batched_rejects_bad_arguments(api):
    L = api.lib()
    I64 = ctypes.c_int64 * 4

    def call(xo, so, ncl=3, d=2, n_iter=1, prec="fp32", kernel="gaussian"):
        p = api.make_params(1.0, kernel=kernel, precision=prec)
        return L.ms_step_batched(ctypes.byref(p), FAKE, I64(*xo), FAKE, I64(*so), ncl, d, n_iter,
                                 FAKE, FAKE, FAKE, None)

    good_x, good_s = (0, 5, 9, 12), (0, 2, 2, 4)
    assert call((0, 5, 9, 12), (0, 0, 0, 0)) == 0     # no seeds: nothing to do
    cases = [
        (dict(xo=good_x, so=good_s, prec="bf16"), "Gaussian kernel at 5 <= d <= 32"),
        (dict(xo=good_x, so=good_s, prec="bf16", d=33), "Gaussian kernel at 5 <= d <= 32"),
        (dict(xo=good_x, so=good_s, prec="bf16", d=16, kernel="flat"), "Gaussian kernel at 5 <= d <= 32"),
        (dict(xo=good_x, so=good_s, ncl=0), "ncl must"),
        (dict(xo=good_x, so=good_s, ncl=9000), "ncl must"),
        (dict(xo=(1, 5, 9, 12), so=good_s), "start at 0"),
        (dict(xo=(0, 5, 4, 12), so=good_s), "nondecreasing"),
        (dict(xo=(0, 5, 5, 12), so=(0, 2, 3, 4)), "no points"),
        (dict(xo=good_x, so=good_s, d=65), "take d in [1, 64]"),
        (dict(xo=good_x, so=good_s, n_iter=5000), "n_iter"),
    ]
    for kw, msg in cases:
        assert call(**kw) == api.MS_E_INVALID, kw
        assert msg in api.last_error(), (kw, api.last_error())

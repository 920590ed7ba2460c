"""FP64 CPU oracle for GPU Faster Mean Shift (Euclidean), arXiv 2112.13891.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2112_13891_amd`` and never imports it.

The arithmetic lives in ``fms_oracle.c`` (plain C, FP64, index-order sums); this
module loads it with ctypes, marshals numpy arrays, and holds the host-side
seed-count rule for frame sequences (integer logic, Section II-D).  ``adjoint.py`` holds
the FP64 reference for the differentiated step, written with plain PyTorch CPU
ops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fms_oracle.c")
_LIB = os.path.join(_HERE, "libfms_oracle.so")

FLAT = 0
GAUSSIAN = 1
KERNELS = {"flat": FLAT, "gaussian": GAUSSIAN}
METRICS = {"euclidean": 0, "cosine": 1}

ACTIVE, CONVERGED, FAILED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        L.orc_weight.argtypes = [f64, f64, ctypes.c_int]
        L.orc_weight.restype = f64
        L.orc_mean.argtypes = [P, i64, ctypes.c_int, P, f64, ctypes.c_int, P]
        L.orc_mean.restype = f64
        L.orc_step.argtypes = [P, i64, ctypes.c_int, f64, ctypes.c_int, f64, P, i32, i32,
                               P, P, P, ctypes.c_int]
        L.orc_step.restype = ctypes.c_int
        L.orc_step_metric.argtypes = L.orc_step.argtypes + [ctypes.c_int]
        L.orc_step_metric.restype = ctypes.c_int
        L.orc_splitmix64.argtypes = [P]
        L.orc_splitmix64.restype = u64
        L.orc_draw.argtypes = [P, P, i32, i32]
        L.orc_draw.restype = None
        L.orc_assign.argtypes = [P, i64, ctypes.c_int, P, i32, P, P, ctypes.c_int]
        L.orc_assign.restype = ctypes.c_int
        L.orc_assign_metric.argtypes = L.orc_assign.argtypes + [ctypes.c_int]
        L.orc_assign_metric.restype = ctypes.c_int
        L.orc_fit.argtypes = ([P, i64, ctypes.c_int, f64, ctypes.c_int, f64, i32, f64, f64,
                               f64, i32, i32, i32, u64, ctypes.c_int, i32, P, P, P, P, P,
                               i32] + [P] * 10)
        L.orc_fit.restype = ctypes.c_int
        L.orc_fit_metric.argtypes = L.orc_fit.argtypes + [ctypes.c_int]
        L.orc_fit_metric.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f32(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be n x d")
    return X


def threads(nthreads=None) -> int:
    return int(nthreads) if nthreads else int(lib().orc_max_threads())


def weight(q, h, kernel="gaussian") -> float:
    return lib().orc_weight(float(q), float(h), KERNELS[kernel])


def mean(X, s, h, kernel="gaussian"):
    """One update m(s) over all points; returns (m, sum of weights)."""
    X = _f32(X)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = s.copy()
    w = lib().orc_mean(_ptr(X), X.shape[0], X.shape[1], _ptr(s), float(h),
                       KERNELS[kernel], _ptr(out))
    return out, w


def step(X, seeds, h, kernel="gaussian", tol=1e-3, n_iter=1, status=None,
         nthreads=None, metric="euclidean"):
    """Up to n_iter updates of the active seeds (status 0).  With
    ``metric="cosine"`` points and seeds are taken as their directions.

    Returns (seeds', status', iters, shift2)."""
    X = _f32(X)
    S = np.array(seeds, dtype=np.float64, copy=True, order="C").reshape(-1, X.shape[1])
    m = S.shape[0]
    st = np.zeros(m, np.uint8) if status is None else np.array(status, np.uint8, copy=True)
    iters = np.zeros(m, np.int32)
    sh = np.full(m, np.nan, np.float64)
    rc = lib().orc_step_metric(_ptr(X), X.shape[0], X.shape[1], float(h), KERNELS[kernel],
                               float(tol), _ptr(S), m, int(n_iter), _ptr(st), _ptr(iters),
                               _ptr(sh), threads(nthreads), METRICS[metric])
    if rc != 0:
        raise ValueError(f"orc_step failed: {rc}")
    return S, st, iters, sh


def splitmix64_stream(seed: int, count: int):
    state = np.array([seed], dtype=np.uint64)
    return [int(lib().orc_splitmix64(_ptr(state))) for _ in range(count)]


def draw(seed: int, pool, count: int):
    """Partial Fisher-Yates draw of ``count`` ids from ``pool`` (order kept)."""
    state = np.array([seed], dtype=np.uint64)
    a = np.array(pool, dtype=np.int32, copy=True)
    lib().orc_draw(_ptr(state), _ptr(a), a.shape[0], int(count))
    return a[:count].copy(), int(state[0])


def assign(X, modes, nthreads=None, metric="euclidean"):
    X = _f32(X)
    M = np.ascontiguousarray(modes, dtype=np.float64).reshape(-1, X.shape[1])
    labels = np.empty(X.shape[0], np.int32)
    margin = np.empty(X.shape[0], np.float64)
    rc = lib().orc_assign_metric(_ptr(X), X.shape[0], X.shape[1], _ptr(M), M.shape[0],
                                 _ptr(labels), _ptr(margin), threads(nthreads), METRICS[metric])
    if rc != 0:
        raise ValueError(f"orc_assign failed: {rc}")
    return labels, margin


@dataclass
class FitResult:
    status: int
    k: int
    modes: np.ndarray
    counts: np.ndarray
    labels: np.ndarray
    margin: np.ndarray
    round_N: np.ndarray
    round_B: np.ndarray
    round_M: np.ndarray
    round_T: np.ndarray
    drawn: np.ndarray
    drawn_iters: np.ndarray
    drawn_status: np.ndarray
    drawn_final: np.ndarray
    pairs: int

    def rounds(self):
        """Drawn ids split per round."""
        out, o = [], 0
        for b in self.round_B:
            out.append(self.drawn[o:o + b])
            o += b
        return out


def fit(X, h, kernel="gaussian", tol=1e-3, max_iter=100, merge_radius=1.0,
        cover_radius=1.0, gamma=1.0, n_initial=128, L=8, all_points=False,
        rng_seed=0, max_modes=None, nthreads=None, max_rounds=64,
        metric="euclidean") -> FitResult:
    """The whole method (Algorithm 2; Algorithm 1 with ``all_points``), on the
    points or, with ``metric="cosine"``, on their directions."""
    X = _f32(X)
    n, d = X.shape
    max_modes = int(max_modes or n)
    modes = np.zeros((max_modes, d), np.float64)
    counts = np.zeros(max_modes, np.int32)
    k = np.zeros(1, np.int32)
    labels = np.full(n, -1, np.int32)
    margin = np.full(n, np.nan, np.float64)
    nr = np.zeros(1, np.int32)
    rN, rB, rM, rT = (np.zeros(max_rounds, np.int32) for _ in range(4))
    drawn = np.full(n, -1, np.int32)
    diters = np.zeros(n, np.int32)
    dstat = np.zeros(n, np.int8)
    dfinal = np.zeros((n, d), np.float64)
    pairs = np.zeros(1, np.int64)
    # gamma, tol and radii are taken as the float32 values the library sees
    rc = lib().orc_fit_metric(_ptr(X), n, d, float(np.float32(h)), KERNELS[kernel],
                       float(np.float32(tol)), int(max_iter), float(np.float32(merge_radius)),
                       float(np.float32(cover_radius)), float(np.float32(gamma)),
                       int(n_initial), int(L), int(bool(all_points)), int(rng_seed) & (2**64 - 1),
                       threads(nthreads), max_modes, _ptr(modes), _ptr(counts), _ptr(k),
                       _ptr(labels), _ptr(margin), max_rounds, _ptr(nr), _ptr(rN), _ptr(rB),
                       _ptr(rM), _ptr(rT), _ptr(drawn), _ptr(diters), _ptr(dstat),
                       _ptr(dfinal), _ptr(pairs), METRICS[metric])
    K = int(k[0])
    R = int(nr[0])
    tot = int(rB[:R].sum())
    kk = min(K, max_modes)
    return FitResult(rc, K, modes[:kk].copy(), counts[:kk].copy(), labels, margin,
                     rN[:R].copy(), rB[:R].copy(), rM[:R].copy(), rT[:R].copy(),
                     drawn[:tot].copy(), diters[:tot].copy(), dstat[:tot].copy(),
                     dfinal[:tot].copy(), int(pairs[0]))


def next_seed_count(N: int, M: int, H: int = 32) -> int:
    """Section II-D (video / tracking): the seed count a frame starts with is
    the previous frame's final N, lowered by M (that frame's mode count)
    whenever it exceeds H * M, so that a count grown for a busy scene falls
    back gradually once the scene is quiet again; never below one seed."""
    if N > H * M:
        N = N - M
    return max(1, N)


def fit_sequence(frames, h, H: int = 32, n_initial: int = 128, **kw):
    """The method frame by frame, each fit warm-started with the seed count the
    previous one ended with (Section II-D).  Returns (results, start counts)."""
    results, starts = [], []
    N = int(n_initial)
    for X in frames:
        starts.append(N)
        r = fit(X, h, n_initial=N, **kw)
        results.append(r)
        N = next_seed_count(int(r.round_N[-1]), r.k, H)
    return results, starts

"""ctypes binding of libfms (see include/fms.h): argument marshalling only.

Every function here passes torch device pointers and the current HIP stream
to the C ABI; all of the method runs in the library's HIP kernels.  If the
library is missing, the import of this module's functions fails loudly:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfms.so")

MS_OK, MS_E_INVALID, MS_E_NONFINITE, MS_E_CAPACITY, MS_E_NO_MODES, MS_E_NOMEM, MS_E_HIP = (
    0, -1, -2, -3, -4, -5, -6)
KERNELS = {"flat": 0, "gaussian": 1}
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16_refine": 1}
METRICS = {"euclidean": 0, "cosine": 1}
DIAG_MAX_ROUNDS = 64


class MeanShiftError(RuntimeError):
    def __init__(self, code: int, message: str, k: int | None = None):
        super().__init__(f"libfms error {code}: {message}")
        self.code = code
        self.k = k


class Params(ctypes.Structure):
    _fields_ = [
        ("rng_seed", ctypes.c_uint64),
        ("h", ctypes.c_float),
        ("kernel", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("tol", ctypes.c_float),
        ("max_iter", ctypes.c_int32),
        ("merge_radius", ctypes.c_float),
        ("cover_radius", ctypes.c_float),
        ("gamma", ctypes.c_float),
        ("n_initial", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("refine_radius", ctypes.c_float),
        ("all_points_as_seeds", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("metric", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("tile_R", ctypes.c_int32),
        ("plain", ctypes.c_int32),
        ("tile_chunk", ctypes.c_int32),
        ("tile_grid", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("round_N", ctypes.c_int32 * DIAG_MAX_ROUNDS),
        ("round_B", ctypes.c_int32 * DIAG_MAX_ROUNDS),
        ("round_M", ctypes.c_int32 * DIAG_MAX_ROUNDS),
        ("round_T", ctypes.c_int32 * DIAG_MAX_ROUNDS),
        ("round_converged", ctypes.c_int32 * DIAG_MAX_ROUNDS),
        ("pairs", ctypes.c_int64),
        ("refined_pairs", ctypes.c_int64),
        ("iterate_ms", ctypes.c_double),
        ("merge_ms", ctypes.c_double),
        ("assign_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
        ("drawn", ctypes.c_void_p),
        ("drawn_iters", ctypes.c_void_p),
        ("drawn_status", ctypes.c_void_p),
        ("drawn_final", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
    ]


EXPORTS = ("ms_default_params", "ms_fit", "ms_step", "ms_step_noalloc", "ms_step_batched", "ms_tune_batched", "ms_fit_batched",
           "ms_assign",
           "ms_forward_update", "ms_step_adjoint", "ms_seed_draw", "ms_seed_count_next",
           "ms_release_workspace", "ms_graph_stats", "ms_last_error", "ms_version")

_lib = None


def lib():
    """Load libfms.so (built in-tree).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.ms_default_params.argtypes = [ctypes.POINTER(Params)]
    L.ms_default_params.restype = None
    L.ms_fit.argtypes = [ctypes.POINTER(Params), P, i64, i32, P, i32, P, P, P, P]
    L.ms_fit.restype = ctypes.c_int
    L.ms_step.argtypes = [ctypes.POINTER(Params), P, i64, i32, P, i32, i32, P, P, P, P]
    L.ms_step.restype = ctypes.c_int
    L.ms_step_noalloc.argtypes = L.ms_step.argtypes
    L.ms_step_noalloc.restype = ctypes.c_int
    L.ms_step_batched.argtypes = [ctypes.POINTER(Params), P, P, P, P, i32, i32, i32, P, P, P, P]
    L.ms_step_batched.restype = ctypes.c_int
    L.ms_tune_batched.argtypes = [ctypes.POINTER(Params), P, P, P, P, i32, i32, i32, P, P, P]
    L.ms_tune_batched.restype = ctypes.c_int
    L.ms_fit_batched.argtypes = [ctypes.POINTER(Params), P, P, i32, i32, P, i64, P, P, P, P]
    L.ms_fit_batched.restype = ctypes.c_int
    L.ms_assign.argtypes = [P, i64, i32, P, i32, P, P, P]
    L.ms_assign.restype = ctypes.c_int
    L.ms_forward_update.argtypes = [P, i32, i64, P, i64, i32, ctypes.c_double, P, i32, P]
    L.ms_forward_update.restype = ctypes.c_int
    L.ms_step_adjoint.argtypes = [P, i32, i64, P, i64, i32, ctypes.c_double, P, P, P, i32, P]
    L.ms_step_adjoint.restype = ctypes.c_int
    L.ms_seed_draw.argtypes = [P, P, i32, i32, P]
    L.ms_seed_draw.restype = ctypes.c_int
    L.ms_seed_count_next.argtypes = [i32, i32, i32, P]
    L.ms_seed_count_next.restype = ctypes.c_int
    L.ms_release_workspace.argtypes = []
    L.ms_release_workspace.restype = ctypes.c_int
    L.ms_last_error.argtypes = []
    L.ms_last_error.restype = ctypes.c_char_p
    L.ms_version.argtypes = []
    L.ms_version.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return lib().ms_last_error().decode()


def _check(rc: int, k: int | None = None):
    if rc != MS_OK:
        raise MeanShiftError(rc, last_error(), k)


def make_params(h, kernel="gaussian", precision="fp32", tol=1e-3, max_iter=100,
                merge_radius=1.0, cover_radius=1.0, gamma=1.0, n_initial=128, L=8,
                refine_radius=3.0, all_points=False, rng_seed=0, check_finite=False,
                metric="euclidean") -> Params:
    p = Params()
    lib().ms_default_params(ctypes.byref(p))
    p.h = float(h)
    p.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.tol = float(tol)
    p.max_iter = int(max_iter)
    p.merge_radius = float(merge_radius)
    p.cover_radius = float(cover_radius)
    p.gamma = float(gamma)
    p.n_initial = int(n_initial)
    p.L = int(L)
    p.refine_radius = float(refine_radius)
    p.all_points_as_seeds = int(bool(all_points))
    p.rng_seed = int(rng_seed) & (2 ** 64 - 1)
    p.check_finite = int(bool(check_finite))
    p.metric = METRICS[metric] if isinstance(metric, str) else int(metric)
    return p


def _torch():
    import torch
    return torch


def _stream_ptr(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t, dtype, ndim=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class FitResult:
    modes: "object"        # K x d float32 tensor (device)
    labels: "object"       # n int32 tensor (device) or None
    k: int
    rounds: int
    round_N: np.ndarray
    round_B: np.ndarray
    round_M: np.ndarray
    round_T: np.ndarray
    round_converged: np.ndarray
    pairs: int
    refined_pairs: int
    iterate_ms: float
    merge_ms: float
    assign_ms: float
    total_ms: float
    workspace_bytes: int
    counts: np.ndarray | None = None
    drawn: np.ndarray | None = None
    drawn_iters: np.ndarray | None = None
    drawn_status: np.ndarray | None = None
    drawn_final: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    def drawn_rounds(self):
        out, o = [], 0
        for b in self.round_B:
            out.append(self.drawn[o:o + b])
            o += b
        return out


def fit(X, h, kernel="gaussian", precision="fp32", tol=1e-3, max_iter=100, merge_radius=1.0,
        cover_radius=1.0, gamma=1.0, n_initial=128, L=8, refine_radius=3.0, all_points=False,
        rng_seed=0, check_finite=False, max_modes=None, labels=True, trace=False,
        metric="euclidean", plain=False) -> FitResult:
    """Whole method on device-resident X (n x d float32).  ``trace`` also returns
    the drawn ids, per-seed iterations, status and final positions.
    ``metric="cosine"`` clusters the directions of the rows (unit-vector modes).
    ``plain=True`` runs the FP32 step over every pair in input order (no
    spatial order or block culling), for comparison."""
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    n, d = X.shape
    max_modes = int(max_modes or n)
    p = make_params(h, kernel, precision, tol, max_iter, merge_radius, cover_radius, gamma,
                    n_initial, L, refine_radius, all_points, rng_seed, check_finite, metric)
    p.plain = int(bool(plain))
    modes = torch.empty((max_modes, d), dtype=torch.float32, device=X.device)
    lab = torch.empty((n,), dtype=torch.int32, device=X.device) if labels else None
    k = ctypes.c_int32(0)
    dg = Diag()
    host = {}
    if trace:
        host = dict(drawn=np.full(n, -1, np.int32), drawn_iters=np.zeros(n, np.int32),
                    drawn_status=np.zeros(n, np.int8), drawn_final=np.zeros((n, d), np.float32),
                    counts=np.zeros(max_modes, np.int32))
        for name, arr in host.items():
            setattr(dg, name, arr.ctypes.data_as(ctypes.c_void_p))
    rc = lib().ms_fit(ctypes.byref(p), Xp, n, d, ctypes.c_void_p(modes.data_ptr()), max_modes,
                      ctypes.byref(k), ctypes.c_void_p(lab.data_ptr()) if lab is not None else None,
                      ctypes.byref(dg), _stream_ptr(X))
    _check(rc, int(k.value))
    K = int(k.value)
    R = int(dg.rounds)
    res = FitResult(
        modes=modes[:K], labels=lab, k=K, rounds=R,
        round_N=np.array(dg.round_N[:R]), round_B=np.array(dg.round_B[:R]),
        round_M=np.array(dg.round_M[:R]), round_T=np.array(dg.round_T[:R]),
        round_converged=np.array(dg.round_converged[:R]), pairs=int(dg.pairs),
        refined_pairs=int(dg.refined_pairs), iterate_ms=dg.iterate_ms, merge_ms=dg.merge_ms,
        assign_ms=dg.assign_ms, total_ms=dg.total_ms, workspace_bytes=int(dg.workspace_bytes))
    if trace:
        tot = int(res.round_B.sum())
        res.drawn = host["drawn"][:tot]
        res.drawn_iters = host["drawn_iters"][:tot]
        res.drawn_status = host["drawn_status"][:tot]
        res.drawn_final = host["drawn_final"][:tot]
        res.counts = host["counts"][:K]
    return res


def step(X, seeds, h, kernel="gaussian", precision="fp32", tol=1e-3, n_iter=1, converged=None,
         refine_radius=3.0, metric="euclidean", plain=False, noalloc=False):
    """Up to n_iter updates of the active seeds.  Returns new tensors
    (seeds, converged uint8, iters int32, shift2 float32).  ``noalloc=True``
    calls ms_step_noalloc (workspace in the library's fixed device scratch)."""
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    n, d = X.shape
    S = seeds.detach().clone().contiguous()
    _dev(S, torch.float32, 2, "seeds")
    if S.shape[1] != d:
        raise ValueError("seeds must be m x d")
    m = S.shape[0]
    conv = (torch.zeros(m, dtype=torch.uint8, device=X.device) if converged is None
            else converged.detach().clone().to(torch.uint8).contiguous())
    iters = torch.zeros(m, dtype=torch.int32, device=X.device)
    sh = torch.full((m,), float("nan"), dtype=torch.float32, device=X.device)
    p = make_params(h, kernel, precision, tol, refine_radius=refine_radius, metric=metric)
    p.plain = int(bool(plain))
    fn = lib().ms_step_noalloc if noalloc else lib().ms_step
    rc = fn(ctypes.byref(p), Xp, n, d, ctypes.c_void_p(S.data_ptr()), m, int(n_iter),
                       ctypes.c_void_p(conv.data_ptr()), ctypes.c_void_p(iters.data_ptr()),
                       ctypes.c_void_p(sh.data_ptr()), _stream_ptr(X))
    _check(rc)
    return S, conv, iters, sh


def step_batched(X, x_off, seeds, s_off, h, kernel="gaussian", tol=1e-3, n_iter=1,
                 converged=None, graph=False, tile_R=0, tile_chunk=0, tile_grid=0, precision="fp32"):
    """ms_step over many clouds: cloud c owns X[x_off[c]:x_off[c+1]] and
    seeds[s_off[c]:s_off[c+1]].  Offsets are host sequences of ncl + 1 ints.
    graph=True runs the n_iter iterations as one captured HIP graph; tile_R,
    tile_chunk and tile_grid force the seeds per lane, points per chunk and
    step grid (0: tuned or default shape).  precision="bf16" takes the BF16
    form (Gaussian kernel, 5 <= d <= 32; tile_R does not apply).
    Returns new tensors (seeds, converged uint8, iters int32, shift2 float32)."""
    import numpy as np
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    d = X.shape[1]
    S = seeds.detach().clone().contiguous()
    _dev(S, torch.float32, 2, "seeds")
    if S.shape[1] != d:
        raise ValueError("seeds must be m x d")
    xo = np.ascontiguousarray(np.asarray(x_off, dtype=np.int64))
    so = np.ascontiguousarray(np.asarray(s_off, dtype=np.int64))
    if xo.shape != so.shape or xo.ndim != 1:
        raise ValueError("x_off and s_off must both have ncl + 1 entries")
    m = S.shape[0]
    conv = (torch.zeros(m, dtype=torch.uint8, device=X.device) if converged is None
            else converged.detach().clone().to(torch.uint8).contiguous())
    iters = torch.zeros(m, dtype=torch.int32, device=X.device)
    sh = torch.full((m,), float("nan"), dtype=torch.float32, device=X.device)
    p = make_params(h, kernel, precision, tol)
    p.graph = 1 if graph else 0
    p.tile_R = int(tile_R)
    p.tile_chunk = int(tile_chunk)
    p.tile_grid = int(tile_grid)
    rc = lib().ms_step_batched(ctypes.byref(p), Xp, xo.ctypes.data, ctypes.c_void_p(S.data_ptr()),
                               so.ctypes.data, int(len(xo) - 1), d, int(n_iter),
                               ctypes.c_void_p(conv.data_ptr()), ctypes.c_void_p(iters.data_ptr()),
                               ctypes.c_void_p(sh.data_ptr()), _stream_ptr(X))
    _check(rc)
    return S, conv, iters, sh


def fit_batched(X, x_off, h, kernel="gaussian", tol=1e-3, max_iter=100, merge_radius=1.0,
                cover_radius=1.0, n_initial=128, L=8, all_points=False, rng_seed=0, max_modes=None,
                labels=True, precision="fp32"):
    """ms_fit_batched: the whole method on every cloud of a CSR batch (cloud c
    owns X[x_off[c]:x_off[c+1]] and draws with SplitMix64 state rng_seed + c).
    precision "bf16" runs the iterations in the batched BF16 form (Gaussian,
    5 <= d <= 32).  Returns (modes list of per-cloud tensors, labels tensor
    or None, k_off numpy array, rounds)."""
    import numpy as np
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    n, d = X.shape
    xo = np.ascontiguousarray(np.asarray(x_off, dtype=np.int64))
    if xo.ndim != 1 or len(xo) < 2:
        raise ValueError("x_off must have ncl + 1 entries")
    ncl = len(xo) - 1
    max_modes = int(max_modes or n)
    p = make_params(h, kernel, precision, tol, max_iter, merge_radius, cover_radius, 1.0, n_initial, L,
                    all_points=all_points, rng_seed=rng_seed)
    modes = torch.empty((max_modes, d), dtype=torch.float32, device=X.device)
    lab = torch.empty((n,), dtype=torch.int32, device=X.device) if labels else None
    k_off = np.zeros(ncl + 1, np.int64)
    rounds = ctypes.c_int32(0)
    rc = lib().ms_fit_batched(ctypes.byref(p), Xp, xo.ctypes.data, ncl, d, ctypes.c_void_p(modes.data_ptr()),
                              max_modes, k_off.ctypes.data,
                              ctypes.c_void_p(lab.data_ptr()) if lab is not None else None,
                              ctypes.byref(rounds), _stream_ptr(X))
    _check(rc, int(k_off[-1]))
    # one split call makes every cloud's view (a slice per cloud in Python
    # costs microseconds each)
    per = list(torch.split(modes[:int(k_off[-1])], np.diff(k_off).tolist()))
    return per, lab, k_off, int(rounds.value)


def tune_batched(X, x_off, seeds, s_off, h, kernel="gaussian", tol=1e-3, trials=4, precision="fp32"):
    """ms_tune_batched: time each launch shape (seeds per lane, points per
    chunk, step grid) on this input and keep the fastest for later
    step_batched / fit_batched calls on inputs of the same kind and
    precision (the BF16 form: seed tiles of 128, R = 2, only).
    Returns (best R, {R: ms per iteration}, best chunk, best grid)."""
    import numpy as np
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    Sp = _dev(seeds, torch.float32, 2, "seeds")
    xo = np.ascontiguousarray(np.asarray(x_off, dtype=np.int64))
    so = np.ascontiguousarray(np.asarray(s_off, dtype=np.int64))
    if xo.shape != so.shape or xo.ndim != 1:
        raise ValueError("x_off and s_off must both have ncl + 1 entries")
    p = make_params(h, kernel, precision, tol)
    best = ctypes.c_int32(0)
    chunk = ctypes.c_int32(0)
    grid = ctypes.c_int32(0)
    ms = (ctypes.c_float * 3)()
    rc = lib().ms_tune_batched(ctypes.byref(p), Xp, xo.ctypes.data, Sp, so.ctypes.data,
                               int(len(xo) - 1), X.shape[1], int(trials), ctypes.byref(best), ms,
                               ctypes.byref(chunk), ctypes.byref(grid), _stream_ptr(X))
    _check(rc)
    return best.value, {r: ms[c] for c, r in enumerate((1, 2, 4)) if ms[c] >= 0}, chunk.value, grid.value


def assign(X, modes, margin=False):
    torch = _torch()
    Xp = _dev(X, torch.float32, 2, "X")
    M = _dev(modes, torch.float32, 2, "modes")
    n, d = X.shape
    if modes.shape[1] != d:
        raise ValueError("modes must be k x d")
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    mg = torch.empty(n, dtype=torch.float32, device=X.device) if margin else None
    rc = lib().ms_assign(Xp, n, d, M, modes.shape[0], ctypes.c_void_p(lab.data_ptr()),
                         ctypes.c_void_p(mg.data_ptr()) if mg is not None else None,
                         _stream_ptr(X))
    _check(rc)
    return (lab, mg) if margin else lab


def _batched(X, S):
    if X.dim() == 2:
        return X.unsqueeze(0), S.unsqueeze(0), True
    return X, S, False


def forward_update(X, S, h):
    """One Gaussian update of every seed, S' = m(S); X: [B,] n x d, S: [B,] m x d."""
    torch = _torch()
    Xb, Sb, squeeze = _batched(X, S)
    dt = X.dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError("float32 or float64 only")
    _dev(Xb.contiguous(), dt)
    Xb, Sb = Xb.contiguous(), Sb.contiguous()
    nb, n, d = Xb.shape
    m = Sb.shape[1]
    out = torch.empty_like(Sb)
    rc = lib().ms_forward_update(ctypes.c_void_p(Xb.data_ptr()), nb, n, ctypes.c_void_p(Sb.data_ptr()),
                                 m, d, float(h), ctypes.c_void_p(out.data_ptr()),
                                 Xb.element_size(), _stream_ptr(Xb))
    _check(rc)
    return out[0] if squeeze else out


def step_adjoint(X, S, h, G):
    """(dL/dS, dL/dX) of one Gaussian update for the upstream gradient G."""
    torch = _torch()
    Xb, Sb, squeeze = _batched(X, S)
    Gb = G.unsqueeze(0) if squeeze else G
    Xb, Sb, Gb = Xb.contiguous(), Sb.contiguous(), Gb.contiguous()
    _dev(Xb, X.dtype)
    nb, n, d = Xb.shape
    m = Sb.shape[1]
    dS = torch.zeros_like(Sb)
    dX = torch.zeros_like(Xb)
    rc = lib().ms_step_adjoint(ctypes.c_void_p(Xb.data_ptr()), nb, n, ctypes.c_void_p(Sb.data_ptr()),
                               m, d, float(h), ctypes.c_void_p(Gb.data_ptr()),
                               ctypes.c_void_p(dS.data_ptr()), ctypes.c_void_p(dX.data_ptr()),
                               Xb.element_size(), _stream_ptr(Xb))
    _check(rc)
    return (dS[0], dX[0]) if squeeze else (dS, dX)


def step_adjoint_accumulate(X, S, h, G, dS, dX):
    """ms_step_adjoint adding into caller arrays: dS += dL/dS and dX += dL/dX
    of one Gaussian update for the upstream gradient G.  dS may be dX itself
    when S is X (the first step of the unrolled form, S_0 = X)."""
    torch = _torch()
    squeeze = X.dim() == 2
    Xb = X.unsqueeze(0) if squeeze else X
    nb, n, d = Xb.shape
    m = S.shape[-2]
    for name, t, rows in (("S", S, m), ("G", G, m), ("dS", dS, m), ("dX", dX, n)):
        _dev(t, X.dtype, X.dim(), name)
        if t.shape[-2:] != (rows, d) or (not squeeze and t.shape[0] != nb):
            raise ValueError(f"{name} has shape {tuple(t.shape)}")
    _dev(X, X.dtype, None, "X")
    if G.data_ptr() in (dS.data_ptr(), dX.data_ptr()):
        raise ValueError("G must not share memory with dS or dX")
    if dS.data_ptr() == dX.data_ptr() and m != n:
        raise ValueError("dS may be dX only when S has as many rows as X")
    rc = lib().ms_step_adjoint(ctypes.c_void_p(X.data_ptr()), nb, n, ctypes.c_void_p(S.data_ptr()),
                               m, d, float(h), ctypes.c_void_p(G.data_ptr()),
                               ctypes.c_void_p(dS.data_ptr()), ctypes.c_void_p(dX.data_ptr()),
                               X.element_size(), _stream_ptr(X))
    _check(rc)


def seed_draw(rng_state: int, pool, count: int):
    """The library's seed draw on host memory.  Returns (ids, new_state)."""
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    out = np.empty(int(count), np.int32)
    st = ctypes.c_uint64(int(rng_state) & (2 ** 64 - 1))
    rc = lib().ms_seed_draw(ctypes.byref(st), pool.ctypes.data_as(ctypes.c_void_p), pool.shape[0],
                            int(count), out.ctypes.data_as(ctypes.c_void_p))
    _check(rc)
    return out, int(st.value)


def graph_stats():
    """(instantiations, in-place updates) of ms_step_batched's graph launches
    on the calling thread."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().ms_graph_stats(ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def release_workspace():
    """Free the device workspace and pinned staging the library keeps for
    the calling thread between ms_fit / ms_fit_batched calls."""
    _check(lib().ms_release_workspace())


def seed_count_next(n_last: int, modes: int, H: int = 32) -> int:
    """Seed count the next frame of a sequence starts with (Section II-D):
    n_last - modes when n_last > H * modes, else n_last."""
    out = ctypes.c_int32(0)
    _check(lib().ms_seed_count_next(int(n_last), int(modes), int(H), ctypes.byref(out)))
    return int(out.value)


def fit_sequence(frames, h, H: int = 32, n_initial: int = 128, **kw):
    """The method over a sequence of point sets (frames of a video or a
    tracking run): each frame is one ms_fit that starts from the seed count
    the previous frame ended with, adapted by seed_count_next.  Returns the
    per-frame FitResults and the seed count each frame started with."""
    results, starts = [], []
    N = int(n_initial)
    for X in frames:
        starts.append(N)
        r = fit(X, h, n_initial=N, **kw)
        results.append(r)
        N = seed_count_next(int(r.round_N[-1]), r.k, H)
    return results, starts

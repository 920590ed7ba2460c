"""Differentiable unrolled mean shift on the library's hand-written adjoint.

MeanShiftT.apply(X, h, T) returns S_T, where S_0 = X and S_{t+1} = m(S_t) is
the Gaussian batched update of every point over all points (Section II-B).
Forward: T launches of ms_forward_update.  Backward: for t = T-1 .. 0 one
ms_step_adjoint launch recomputes the weights of step t from the stored S_t
(no n x n matrix is stored), adds dL/dS_t into a fresh array and the point
term of step t into dX; for t = 0, where S_0 = X, the library adds dL/dS_0
into dX as well, so this module does no arithmetic of its own.

Checkpointing: with ``every = k`` only S_0, S_k, S_2k, ... are stored and the
states in between are recomputed by forward launches during backward.

X may be n x d or B x n x d (B independent clouds in one launch), float32 or
float64, on the GPU.  All arithmetic runs in libfms.
"""
from __future__ import annotations

import torch

from . import api


class MeanShiftT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, h, T, every=1):
        h = float(h)
        T = int(T)
        every = max(1, int(every))
        Xc = X.detach().contiguous()
        S = Xc
        saved = {0: S}
        for t in range(T):
            S = api.forward_update(Xc, S, h)
            if (t + 1) % every == 0 and t + 1 < T:
                saved[t + 1] = S
        ctx.h, ctx.T, ctx.every = h, T, every
        ctx.saved_states = saved
        ctx.save_for_backward(Xc)
        return S

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        h, T, every = ctx.h, ctx.T, ctx.every
        saved = ctx.saved_states
        G = G.contiguous().to(X.dtype)
        if T == 0:   # S_T = S_0 = X
            return G, None, None, None
        # ms_step_adjoint adds dL/dS_t into a fresh array and the point term of
        # step t into dX; at t = 0, where S_0 = X, dL/dS_0 is added into dX too
        dX = torch.zeros_like(X)
        cache = {}
        for t in range(T - 1, -1, -1):
            if t in saved:
                S_t = saved[t]
            elif t in cache:
                S_t = cache.pop(t)
            else:
                # replay forward from the nearest stored state below t
                base = max(k for k in saved if k <= t)
                S = saved[base]
                for u in range(base, t):
                    S = api.forward_update(X, S, h)
                    if u + 1 < t:
                        cache[u + 1] = S
                S_t = S
            dS = dX if t == 0 else torch.zeros_like(S_t)
            api.step_adjoint_accumulate(X, S_t, h, G, dS, dX)
            G = dS
        return dX, None, None, None


def mean_shift_unrolled(X, h, T, every=1):
    return MeanShiftT.apply(X, h, T, every)

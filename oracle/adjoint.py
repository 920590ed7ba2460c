"""FP64 reference for the differentiable (unrolled) mean-shift step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain PyTorch CPU ops in
float64, autograd for the derivative; nothing here is shared with the HIP
library.

One Gaussian update of every seed over all points (Section II-B, the batched
update; Gaussian profile exp(-q / (2 h^2)), the reading of the kernel used throughout):
    m(s_j) = sum_i w_ij x_i / sum_i w_ij,   w_ij = exp(-|s_j - x_i|^2 / (2 h^2)).
The unrolled form starts from S_0 = X and applies T updates; the loss of the
differentiable benchmark is sum_p |S_T[p] - c_{y_p}|^2 (each shifted point
against its generating cluster's centre).
"""
from __future__ import annotations

import torch


def update(X: torch.Tensor, S: torch.Tensor, h: float) -> torch.Tensor:
    """m(S): X (n x d) points, S (m x d) seeds, all float64."""
    diff = S[:, None, :] - X[None, :, :]          # m x n x d
    q = (diff * diff).sum(-1)                      # m x n
    w = torch.exp(-q / (2.0 * h * h))
    return (w @ X) / w.sum(1, keepdim=True)


def unrolled(X: torch.Tensor, h: float, T: int) -> torch.Tensor:
    S = X
    for _ in range(T):
        S = update(X, S, h)
    return S


def loss(X: torch.Tensor, h: float, T: int, centres: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    S = unrolled(X, h, T)
    return ((S - centres[y]) ** 2).sum()


def grad_step(X, S, h, G):
    """(dL/dS, dL/dX) of one update for upstream gradient G, via autograd."""
    X = X.detach().clone().double().requires_grad_(True)
    S = S.detach().clone().double().requires_grad_(True)
    out = update(X, S, h)
    out.backward(G.double())
    return S.grad, X.grad


def grad_unrolled(X, h, T, centres, y):
    X = X.detach().clone().double().requires_grad_(True)
    L = loss(X, h, T, centres.double(), y)
    L.backward()
    return L.detach(), X.grad

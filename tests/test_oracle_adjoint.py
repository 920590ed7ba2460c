"""Pins of the FP64 reference for the differentiable step (oracle/adjoint.py):
the update equals the pinned C oracle's mean, the gradient equals central
finite differences, and closed forms hold."""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj


def test_update_matches_c_oracle(orc):
    rng = np.random.default_rng(0)
    X = (rng.standard_normal((300, 5)) * 2).astype(np.float32)
    S = rng.standard_normal((17, 5)) * 2
    h = 1.3
    got = adj.update(torch.from_numpy(X).double(), torch.from_numpy(S), h).numpy()
    for j in range(S.shape[0]):
        m, _ = orc.mean(X, S[j], h, "gaussian")
        assert np.abs(got[j] - m).max() < 1e-12


def test_single_point_gradient_closed_form():
    # one point: every update returns the point itself, so S_T = X and the
    # loss |x - c|^2 has gradient 2 (x - c)
    X = torch.tensor([[0.3, -1.2, 2.0]], dtype=torch.float64)
    c = torch.tensor([[1.0, 1.0, 1.0]], dtype=torch.float64)
    L, g = adj.grad_unrolled(X, 0.7, 5, c, torch.tensor([0]))
    assert torch.allclose(g, 2 * (X - c), atol=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    X = torch.from_numpy(rng.standard_normal((20, 3)) * 1.5)
    C = torch.from_numpy(rng.standard_normal((3, 3)))
    y = torch.from_numpy(rng.integers(0, 3, 20))
    h, T = 1.1, 3
    _, g = adj.grad_unrolled(X, h, T, C, y)
    eps = 1e-6
    num = torch.zeros_like(X)
    for i in range(X.shape[0]):
        for k in range(X.shape[1]):
            Xp = X.clone(); Xp[i, k] += eps
            Xm = X.clone(); Xm[i, k] -= eps
            num[i, k] = (adj.loss(Xp, h, T, C, y) - adj.loss(Xm, h, T, C, y)) / (2 * eps)
    rel = (num - g).abs().max() / g.abs().max()
    assert rel < 1e-6, float(rel)


def test_step_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    X = torch.from_numpy(rng.standard_normal((15, 2)))
    S = torch.from_numpy(rng.standard_normal((6, 2)))
    G = torch.from_numpy(rng.standard_normal((6, 2)))
    h = 0.9
    dS, dX = adj.grad_step(X, S, h, G)
    f = lambda X_, S_: float((adj.update(X_, S_, h) * G).sum())
    eps = 1e-6
    for i in range(S.shape[0]):
        for k in range(2):
            Sp = S.clone(); Sp[i, k] += eps
            Sm = S.clone(); Sm[i, k] -= eps
            assert abs((f(X, Sp) - f(X, Sm)) / (2 * eps) - float(dS[i, k])) < 1e-7
    for i in range(X.shape[0]):
        for k in range(2):
            Xp = X.clone(); Xp[i, k] += eps
            Xm = X.clone(); Xm[i, k] -= eps
            assert abs((f(Xp, S) - f(Xm, S)) / (2 * eps) - float(dX[i, k])) < 1e-7

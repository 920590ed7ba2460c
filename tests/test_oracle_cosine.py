"""Pins of the oracle's cosine-metric form against closed forms and brute
force written with angles (not with the oracle's dot products)."""
import math

import numpy as np
import pytest

from paper_2112_13891_amd import workloads


def _circle(phi, r):
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1).astype(np.float32)


@pytest.mark.parametrize("kernel", ["gaussian", "flat"])
def test_one_update_in_angles(orc, kernel):
    """2-D: with angles, the chord between directions phi and psi is
    2 sin(|phi - psi| / 2); the update is the weighted mean direction."""
    rng = np.random.default_rng(3)
    phi = rng.uniform(-1.0, 1.0, 40)
    r = rng.uniform(0.3, 3.0, 40)
    X = _circle(phi, r)
    phi = np.arctan2(X[:, 1].astype(np.float64), X[:, 0].astype(np.float64))
    h = 0.5
    psi = 0.1
    chord = 2.0 * np.abs(np.sin((phi - psi) / 2.0))
    w = np.exp(-chord ** 2 / (2 * h * h)) if kernel == "gaussian" else (chord <= h).astype(float)
    v = np.array([np.sum(w * np.cos(phi)), np.sum(w * np.sin(phi))])
    want = v / np.linalg.norm(v)
    S, st, it, sh = orc.step(X, [[math.cos(psi) * 7.0, math.sin(psi) * 7.0]], h, kernel, n_iter=1,
                             metric="cosine")
    assert np.allclose(S[0], want, atol=1e-13)
    assert abs(sh[0] - np.sum((want - [math.cos(psi), math.sin(psi)]) ** 2)) < 1e-13


def test_symmetric_cone_converges_to_axis(orc):
    """Points at equal angles around an axis (rotations by 120 degrees): by
    symmetry the only fixed point near the axis is the axis itself."""
    a = np.array([1.0, 2.0, 2.0]) / 3.0
    b = np.cross(a, [1.0, 0.0, 0.0]); b /= np.linalg.norm(b)
    c = np.cross(a, b)
    pts = []
    for t in (0.2, 0.35):
        for k in range(3):
            ang = 2 * math.pi * k / 3 + t
            for lenf in (0.5, 3.0):
                pts.append(lenf * (math.cos(0.3) * a + math.sin(0.3) * (math.cos(ang) * b + math.sin(ang) * c)))
    X = np.array(pts, np.float32)
    s0 = a + 0.05 * b
    S, st, it, sh = orc.step(X, [s0], 0.4, "gaussian", tol=1e-9, n_iter=500, metric="cosine")
    assert st[0] == 1
    assert np.linalg.norm(S[0] - a) < 1e-6


def test_unit_inputs_match_normalized_euclidean_update(orc):
    """On unit vectors the chord is the Euclidean distance, so one cosine
    update is the Euclidean update, normalized."""
    rng = np.random.default_rng(5)
    U = rng.standard_normal((300, 5))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    U = U.astype(np.float32)
    s = U[7].astype(np.float64)
    s = s / np.linalg.norm(s)
    e, _, _, _ = orc.step(U, [s], 0.8, "gaussian", n_iter=1)
    c, _, _, _ = orc.step(U, [s], 0.8, "gaussian", n_iter=1, metric="cosine")
    assert np.allclose(c[0], e[0] / np.linalg.norm(e[0]), atol=1e-7)


def test_flat_window_boundary_by_angle(orc):
    """Flat window: a direction is inside iff its chord is <= h, i.e. its
    angle to the seed is <= 2 asin(h / 2)."""
    h = 0.6
    lim = 2 * math.asin(h / 2)
    phi = np.array([lim - 1e-3, -(lim - 2e-3), lim + 1e-3, 0.0, -(lim + 5e-3)])
    X = _circle(phi, np.ones(5))
    phi = np.arctan2(X[:, 1].astype(np.float64), X[:, 0].astype(np.float64))
    inside = np.abs(phi) <= lim
    v = np.array([np.cos(phi[inside]).sum(), np.sin(phi[inside]).sum()])
    S, _, _, _ = orc.step(X, [[1.0, 0.0]], h, "flat", n_iter=1, metric="cosine")
    assert np.allclose(S[0], v / np.linalg.norm(v), atol=1e-12)


def test_row_lengths_do_not_matter(orc):
    w = workloads.embed_cos(seed=1, n=4000, k=6, d=8)
    a = orc.fit(w.X, w.h, metric="cosine")
    rng = np.random.default_rng(0)
    X2 = (w.X * rng.uniform(0.1, 10.0, (w.n, 1))).astype(np.float32)
    b = orc.fit(X2, w.h, metric="cosine")
    assert a.k == b.k
    assert np.allclose(a.modes, b.modes, atol=1e-6)
    assert (a.labels == b.labels).mean() > 0.999
    assert np.allclose(np.linalg.norm(a.modes, axis=1), 1.0, atol=1e-12)


def test_labels_are_largest_cosine(orc):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((500, 4)).astype(np.float32)
    M = rng.standard_normal((7, 4))
    M /= np.linalg.norm(M, axis=1, keepdims=True)
    lab, _ = orc.assign(X, M, metric="cosine")
    U = X.astype(np.float64) / np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True)
    ang = np.arccos(np.clip(U @ M.T, -1, 1))
    assert np.array_equal(lab, ang.argmin(axis=1))


def test_cosine_fit_finds_the_directions(orc):
    w = workloads.embed_cos(seed=2, n=6000, k=8, d=16, outlier_frac=0.0)
    r = orc.fit(w.X, w.h, metric="cosine")
    assert r.k == 8
    cos = r.modes @ w.extra["centres"].T
    assert (cos.max(axis=1) > 0.99).all()


def test_zero_row_is_rejected(orc):
    X = np.ones((10, 3), np.float32)
    X[4] = 0.0
    with pytest.raises(ValueError):
        orc.step(X, [[1.0, 0.0, 0.0]], 0.5, n_iter=1, metric="cosine")

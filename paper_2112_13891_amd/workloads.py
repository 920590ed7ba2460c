"""Seeded synthetic inputs for the mean-shift hot path.

This module only draws numbers.  It holds none of the method's arithmetic, so
both the FP64 oracle (under ``oracle/``) and the HIP library may take their
inputs from it without sharing any part of the computation.

Every set is a Gaussian mixture shaped like the paper's simulation workload
(2-D sklearn-style blobs at up to 200K points, Section III, Table 1) or like the
larger embedding/batched/differentiable cases built on top of it.  All draws use
``numpy.random.default_rng(seed)`` (PCG64) in the fixed order written in each
function, the rows are shuffled last with ``rng.permutation(n)`` and stored as
float32 (row-major, contiguous).

Workloads
---------
``blobs2d``    2,000 points, D=2, 5 equal isotropic blobs (sigma 2) with centres
               uniform in [0,100]^2; Gaussian kernel, h=5.
``aniso3d``    200,000 points, D=3, 50 axis-aligned anisotropic blobs (per-axis
               sigma uniform in [3,8]) with Dirichlet(2) mixture weights and
               centres uniform in [0,1000]^3; Gaussian kernel, h=15.
``embed32``    262,144 points, D=32: 100 clusters (centres N(0,16 I), sigma 0.5)
               plus 5 % uniform outliers in [-12,12]^32; flat or Gaussian, h=1.5.
``clouds16``   many independent D=16 clouds with log-uniform sizes, 2..40
               clusters each (centres N(0,9 I), sigma 0.4); Gaussian, h=1.
``image_rgb``  an RGB image as side^2 colour 3-vectors in [0,255]: a Voronoi
               partition into coloured regions plus per-channel noise, pixels
               in raster order (the segmentation shape of Section I, Fig. 1);
               Gaussian, h=12.
``embed_cos``  cosine-metric embeddings, D=32: 100 random unit directions,
               points at angular spread ~0.2 rad around them plus 5 % uniform
               directions, every row scaled by a length in [0.5, 2] (only the
               direction counts); chord bandwidth h=0.3.
``frames2d``   a sequence of 2-D frames (video / tracking, Section II-D):
               drifting blobs, and from one frame on a quieter scene with
               fewer blobs; Gaussian, h=5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """A point set plus the method parameters it is clustered with."""
    name: str
    X: np.ndarray                 # float32, n x d, row-major
    y: np.ndarray                 # int32 generating component, -1 = outlier
    h: float
    kernel: str                   # "gaussian" or "flat"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def _finish(rng, X, y):
    perm = rng.permutation(X.shape[0])
    X = np.ascontiguousarray(X[perm], dtype=np.float32)
    y = np.ascontiguousarray(y[perm], dtype=np.int32)
    return X, y


def blobs2d(seed: int = 0, n: int = 2000, k: int = 5, sigma: float = 2.0,
            box: float = 100.0) -> Workload:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, box, (k, 2))
    y = np.repeat(np.arange(k), n // k)
    X = centres[y] + sigma * rng.standard_normal((y.shape[0], 2))
    X, y = _finish(rng, X, y)
    return Workload("blobs2d", X, y, h=5.0, kernel="gaussian",
                    extra={"centres": centres, "sigma": sigma})


def aniso3d(seed: int = 0, n: int = 200_000, k: int = 50) -> Workload:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1000.0, (k, 3))
    sig = rng.uniform(3.0, 8.0, (k, 3))
    wts = rng.dirichlet(2.0 * np.ones(k))
    cnt = rng.multinomial(n, wts)
    y = np.repeat(np.arange(k), cnt)
    X = centres[y] + sig[y] * rng.standard_normal((n, 3))
    X, y = _finish(rng, X, y)
    return Workload("aniso3d", X, y, h=15.0, kernel="gaussian",
                    extra={"centres": centres, "sigma": sig})


def embed32(seed: int = 0, n: int = 262_144, k: int = 100, d: int = 32,
            outlier_frac: float = 0.05, kernel: str = "gaussian") -> Workload:
    rng = np.random.default_rng(seed)
    centres = 4.0 * rng.standard_normal((k, d))
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    y_in = rng.integers(0, k, n_in)
    X_in = centres[y_in] + 0.5 * rng.standard_normal((n_in, d))
    X_out = rng.uniform(-12.0, 12.0, (n_out, d))
    X = np.concatenate([X_in, X_out], axis=0)
    y = np.concatenate([y_in, -np.ones(n_out, dtype=np.int64)])
    X, y = _finish(rng, X, y)
    return Workload("embed32", X, y, h=1.5, kernel=kernel,
                    extra={"centres": centres, "sigma": 0.5})


def cloud16(rng, n: int, d: int = 16):
    """One cloud of the batched / differentiable recipe (draws from ``rng``)."""
    k = int(rng.integers(2, 41))
    centres = 3.0 * rng.standard_normal((k, d))
    y = rng.integers(0, k, n)
    X = centres[y] + 0.4 * rng.standard_normal((n, d))
    perm = rng.permutation(n)
    return (np.ascontiguousarray(X[perm], dtype=np.float32),
            np.ascontiguousarray(y[perm], dtype=np.int32), centres)


def clouds16(seed: int = 0, n_clouds: int = 512, lo: int = 1000, hi: int = 65536,
             d: int = 16):
    """Uneven clouds: sizes log-uniform in [lo, hi]. Returns a list of (X, y, centres)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_clouds):
        n_c = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(cloud16(rng, n_c, d))
    return out


def diffclouds(seed: int = 0, n_clouds: int = 64, n: int = 16384, d: int = 16):
    """Equal-size clouds for the differentiable form. Returns a list of (X, y, centres)."""
    rng = np.random.default_rng(seed)
    return [cloud16(rng, n, d) for _ in range(n_clouds)]


def image_rgb(seed: int = 0, side: int = 512, regions: int = 24, noise: float = 6.0) -> Workload:
    """side x side pixels: region sites uniform in the image, each pixel takes
    the colour (uniform in [0,255]^3) of its nearest site, plus N(0, noise^2)
    per channel, clipped to [0,255].  Raster order, not shuffled: an image is
    stored that way."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, float(side), (regions, 2))
    colours = rng.uniform(0.0, 255.0, (regions, 3))
    yy, xx = np.meshgrid(np.arange(side, dtype=np.float64) + 0.5, np.arange(side, dtype=np.float64) + 0.5,
                         indexing="ij")
    pix = np.stack([yy.ravel(), xx.ravel()], axis=1)
    y = np.empty(pix.shape[0], np.int64)
    for a in range(0, pix.shape[0], 1 << 16):   # nearest site, in slices
        d2 = ((pix[a:a + (1 << 16), None, :] - sites[None, :, :]) ** 2).sum(axis=2)
        y[a:a + (1 << 16)] = d2.argmin(axis=1)
    X = colours[y] + noise * rng.standard_normal((pix.shape[0], 3))
    X = np.clip(X, 0.0, 255.0)
    return Workload(f"image_rgb{side}", np.ascontiguousarray(X, dtype=np.float32),
                    np.ascontiguousarray(y, dtype=np.int32), h=12.0, kernel="gaussian",
                    extra={"sites": sites, "colours": colours, "side": side})


def embed_cos(seed: int = 0, n: int = 262_144, k: int = 100, d: int = 32, spread: float = 0.2,
              outlier_frac: float = 0.05) -> Workload:
    """Directions u = (c + sigma g) / |c + sigma g| around unit centres c, with
    sigma = spread / sqrt(d - 1) (angular spread ~ spread), outliers uniform on
    the sphere; each row is then multiplied by a length uniform in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((k, d))
    centres /= np.linalg.norm(centres, axis=1, keepdims=True)
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    y_in = rng.integers(0, k, n_in)
    U = centres[y_in] + (spread / math.sqrt(d - 1)) * rng.standard_normal((n_in, d))
    U_out = rng.standard_normal((n_out, d))
    U = np.concatenate([U, U_out], axis=0)
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    X = U * rng.uniform(0.5, 2.0, (n, 1))
    y = np.concatenate([y_in, -np.ones(n_out, dtype=np.int64)])
    X, y = _finish(rng, X, y)
    return Workload("embed_cos", X, y, h=0.3, kernel="gaussian", extra={"centres": centres, "metric": "cosine"})


def frames2d(seed: int = 0, n: int = 20_000, k: int = 40, n_frames: int = 6, change_at: int = 3,
             k_after: int = 4, drift: float = 0.5, sigma: float = 2.0, box: float = 400.0):
    """A frame sequence: k blobs (sigma 2, centres uniform in [0, box]^2) whose
    centres move by N(0, drift^2 I) from frame to frame; from frame change_at on
    only the first k_after blobs hold points.  n points per frame, each frame
    drawn and shuffled in turn.  Returns a list of Workloads."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, box, (k, 2))
    out = []
    for f in range(n_frames):
        if f > 0:
            centres = centres + drift * rng.standard_normal((k, 2))
        kk = k if f < change_at else k_after
        y = rng.integers(0, kk, n)
        X = centres[y] + sigma * rng.standard_normal((n, 2))
        X, y = _finish(rng, X, y)
        out.append(Workload(f"frames2d[{f}]", X, y, h=5.0, kernel="gaussian",
                            extra={"centres": centres[:kk].copy()}))
    return out


WORKLOADS = {
    "blobs2d": blobs2d,
    "aniso3d": aniso3d,
    "embed32": embed32,
}

"""Scattered measurement sites for the spline reconstruction of Sec. 6.

The paper's application reconstructs a 4-D spline field (128x128x128x16
coefficients) from about nine million measurements at scattered points.  That
data set is not available.  The stand-in draws the sites uniformly in the unit
hypercube, optionally mixed with Gaussian clusters for an uneven density.  The
coordinates are float32 numbers, which are exact in float64 as well, so both
sides start from the same points.

This module holds no solver arithmetic: the basis values at the sites, the
forward model and its adjoint are formed by each side with its own code.
Random draws: ``numpy.random.default_rng(seed)``; sites first (mode-major,
shape (order, count)), then X_true, then the noise.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .bspline import second_difference

# The paper's application size: 33,554,432 coefficients, ~9M measurements.
SCATTERED = dict(name="scattered_4d_128x128x128x16_9M", n=(128, 128, 128, 16),
                 count=9_000_000, lam=1e-3, sigma=0.01, seed=5000, rtol=1e-6)


@dataclass
class ScatteredProblem:
    n: tuple
    coords: np.ndarray          # (order, count) float32 in [0, 1]
    D: List[np.ndarray]
    lam: float
    X_true: Optional[np.ndarray]
    noise: Optional[np.ndarray]  # (count,)
    rtol: float
    seed: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def order(self):
        return len(self.n)

    @property
    def count(self):
        return int(self.coords.shape[1])


def scattered_sites(order, count, seed, clustered=0.0, rng=None):
    """(order, count) float32 sites in [0, 1].

    A fraction ``clustered`` of the sites is drawn from 1..6 Gaussian clusters
    (centre U[0.1, 0.9], width U[0.02, 0.1] per mode, clipped to [0, 1]); the
    rest is uniform on [0, 1).
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    u = rng.random((order, count), dtype=np.float32)
    nc = int(round(clustered * count))
    if nc > 0:
        K = int(rng.integers(1, 7))
        which = rng.integers(0, K, nc)
        centre = rng.uniform(0.1, 0.9, (order, K))
        width = rng.uniform(0.02, 0.1, (order, K))
        pts = centre[:, which] + width[:, which] * rng.standard_normal((order, nc))
        u[:, :nc] = np.clip(pts, 0.0, 1.0).astype(np.float32)
    return u


def with_endpoints(coords):
    """Copy of ``coords`` whose first samples sit on the ends of every mode
    (t = 0 and t = 1 exactly), the degenerate sites of the clamped basis."""
    c = coords.copy()
    N, S = c.shape
    for s in range(min(S, 2 ** N)):
        for k in range(N):
            c[k, s] = 1.0 if (s >> k) & 1 else 0.0
    return c


def scattered_problem(n, count, lam, sigma, seed, rtol, clustered=0.0, with_data=True, name=""):
    """Sites, second-difference factors, X_true ~ N(0, 1) and noise ~ sigma*N(0, 1)."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    coords = scattered_sites(len(n), count, seed, clustered, rng=rng)
    D = [second_difference(k) for k in n]
    X_true = noise = None
    if with_data:
        X_true = rng.standard_normal(n)
        noise = sigma * rng.standard_normal(count)
    return ScatteredProblem(n=n, coords=coords, D=D, lam=lam, X_true=X_true, noise=noise,
                            rtol=rtol, seed=seed, name=name)


def scattered_config(scale=None, count=None, with_data=True):
    """The application-size instance; ``scale`` shrinks every mode (keeping
    at least 4 coefficients) and the site count by the same volume factor."""
    cfg = SCATTERED
    n, S = cfg["n"], cfg["count"]
    if scale:
        n = tuple(max(4, v // scale) for v in n)
        S = max(1, int(S * np.prod(n) / np.prod(cfg["n"])))
    if count is not None:
        S = int(count)
    return scattered_problem(n, S, cfg["lam"], cfg["sigma"], cfg["seed"], cfg["rtol"],
                             with_data=with_data, name=cfg["name"])

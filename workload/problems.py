"""Seeded problem instances for the regularised tensor equation.

A problem is the tuple (n, m, A_k, D_k, lambda, X_true, noise): unknown tensor
shape n, sample-grid shape m, per-mode collocation A_k (m_k x n_k), per-mode
second difference D_k ((n_k-2) x n_k), regularisation weight lambda, the
ground-truth field X_true and the additive measurement noise (shape m).  The
observation Y = X_true x_1 A_1 ... x_N A_N + noise is *not* formed here: that
product is solver arithmetic and each side (oracle or GPU path) forms it with
its own code.

Random draws: ``numpy.random.default_rng(seed)``; within one problem X_true is
drawn first and the noise second, both in C order, both in float64.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from .bspline import collocation_matrix, second_difference

BATCH_SIZES = (24, 32, 48, 64, 96)


@dataclass
class Problem:
    n: tuple
    m: tuple
    A: List[np.ndarray]
    D: List[np.ndarray]
    lam: float
    X_true: Optional[np.ndarray]
    noise: Optional[np.ndarray]
    rtol: float
    seed: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def order(self):
        return len(self.n)

    @property
    def unknowns(self):
        return int(np.prod(self.n))


# The five workloads: shapes, lambda, noise level, seed and tolerance.
CONFIGS = {
    0: dict(name="3d_32cubed_f64", n=(32, 32, 32), m=(48, 48, 48), lam=1e-3,
            sigma=0.01, seed=0, rtol=1e-10),
    1: dict(name="4d_64x64x64x32_f32", n=(64, 64, 64, 32), m=(96, 96, 96, 48),
            lam=1e-3, sigma=0.01, seed=1000, rtol=1e-6),
    2: dict(name="4d_128x128x96x24_bf16_refine", n=(128, 128, 96, 24),
            m=(192, 192, 144, 36), lam=1e-4, sigma=0.01, seed=2000, rtol=1e-8),
    3: dict(name="batched_256x3d", lam=1e-3, sigma=0.01, seed=3000, rtol=1e-6,
            count=256),
    4: dict(name="warmstart_64x64x64x16", n=(64, 64, 64, 16), m=(96, 96, 96, 24),
            lam=1e-3, sigma=0.01, rtol=1e-8, blob_noise=0.1),
}


def factors(n: Sequence[int], m: Sequence[int]):
    """Per-mode collocation and second-difference matrices (float64)."""
    A = [collocation_matrix(mk, nk) for mk, nk in zip(m, n)]
    D = [second_difference(nk) for nk in n]
    return A, D


def make_problem(n, m, lam, sigma, seed, rtol, name="", with_data=True):
    """Problem with X_true ~ N(0,1) (shape n) and noise ~ sigma*N(0,1) (shape m)."""
    n = tuple(int(v) for v in n)
    m = tuple(int(v) for v in m)
    A, D = factors(n, m)
    X_true = noise = None
    if with_data:
        rng = np.random.default_rng(seed)
        X_true = rng.standard_normal(n)
        noise = sigma * rng.standard_normal(m)
    return Problem(n=n, m=m, A=A, D=D, lam=lam, X_true=X_true, noise=noise,
                   rtol=rtol, seed=seed, name=name)


def config_problem(c, with_data=True, scale=None):
    """Problem for workload ``c`` in (0, 1, 2).

    ``scale`` (optional) shrinks every mode by an integer factor, keeping the
    1.5x sample ratio; it gives small instances with the same structure.
    """
    cfg = CONFIGS[c]
    n, m = cfg["n"], cfg["m"]
    if scale:
        n = tuple(max(4, v // scale) for v in n)
        m = tuple(max(6, (3 * v) // 2) for v in n)
    return make_problem(n, m, cfg["lam"], cfg["sigma"], cfg["seed"], cfg["rtol"],
                        name=cfg["name"], with_data=with_data)


def batched_sizes(count=256, seed=3000):
    """(count, 3) array of per-mode sizes drawn uniformly from BATCH_SIZES."""
    idx = np.random.default_rng(seed).integers(0, len(BATCH_SIZES), (count, 3))
    return np.asarray(BATCH_SIZES)[idx]


def batched_problem(p, sizes=None, with_data=True):
    """Problem ``p`` of the batched workload: m_k = 1.5 n_k, seed 3001 + p."""
    cfg = CONFIGS[3]
    if sizes is None:
        sizes = batched_sizes(cfg["count"], cfg["seed"])
    n = tuple(int(v) for v in sizes[p])
    m = tuple((3 * v) // 2 for v in n)
    return make_problem(n, m, cfg["lam"], cfg["sigma"], cfg["seed"] + 1 + p,
                        cfg["rtol"], name=f"batched_{p}", with_data=with_data)


def blob_field(n, rng, noise_sigma=0.1):
    """Sum of 1..8 axis-aligned anisotropic Gaussian blobs plus white noise.

    Each blob has amplitude U[0.5, 2] with a random sign, centre U[0, n_k-1]
    and width U[1.5, n_k/4] per mode; the field is the sum of separable
    Gaussians plus ``noise_sigma`` * N(0, 1).
    """
    n = tuple(int(v) for v in n)
    K = int(rng.integers(1, 9))
    X = np.zeros(n)
    for _ in range(K):
        amp = rng.uniform(0.5, 2.0) * (1.0 if rng.integers(0, 2) else -1.0)
        profs = []
        for nk in n:
            c = rng.uniform(0.0, nk - 1.0)
            w = rng.uniform(1.5, nk / 4.0)
            i = np.arange(nk, dtype=np.float64)
            profs.append(np.exp(-0.5 * ((i - c) / w) ** 2))
        blob = profs[0]
        for p in profs[1:]:
            blob = np.multiply.outer(blob, p)
        X += amp * blob
    X += noise_sigma * rng.standard_normal(n)
    return X


def blob_field_torch(n, seed, noise_sigma=0.1, device="cuda"):
    """The recipe of blob_field, drawn with torch so that thousands of fields
    can be made on the device (training data of the warm start).

    The small draws (blob count, amplitudes, signs, centres, widths) come from
    a CPU torch generator seeded with ``seed``; the white noise from a device
    generator seeded with ``seed`` (returned, so that further draws for the
    same sample continue its stream).  Float32.
    """
    import torch

    n = tuple(int(v) for v in n)
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    K = int(torch.randint(1, 9, (1,), generator=g))
    X = torch.zeros(n, dtype=torch.float32, device=device)
    for _ in range(K):
        u = torch.rand(2, generator=g, dtype=torch.float64)
        amp = (0.5 + 1.5 * float(u[0])) * (1.0 if float(u[1]) < 0.5 else -1.0)
        blob = None
        for k, nk in enumerate(n):
            cw = torch.rand(2, generator=g, dtype=torch.float64)
            c = float(cw[0]) * (nk - 1.0)
            w = 1.5 + float(cw[1]) * (nk / 4.0 - 1.5)
            i = torch.arange(nk, dtype=torch.float32, device=device)
            prof = torch.exp(-0.5 * ((i - c) / w) ** 2)
            shape = [1] * len(n)
            shape[k] = nk
            prof = prof.reshape(shape)
            blob = prof if blob is None else blob * prof
        X += amp * blob
    gd = torch.Generator(device=device).manual_seed(int(seed))
    X += noise_sigma * torch.randn(n, generator=gd, device=device, dtype=torch.float32)
    return X, gd


def warmstart_problem(seed, n=None, m=None, with_data=True):
    """Warm-start workload instance: blob X_true, noise sigma=0.01 on Y."""
    cfg = CONFIGS[4]
    n = tuple(n or cfg["n"])
    m = tuple(m or cfg["m"])
    A, D = factors(n, m)
    X_true = noise = None
    if with_data:
        rng = np.random.default_rng(seed)
        X_true = blob_field(n, rng, cfg["blob_noise"])
        noise = cfg["sigma"] * rng.standard_normal(m)
    return Problem(n=n, m=m, A=A, D=D, lam=cfg["lam"], X_true=X_true, noise=noise,
                   rtol=cfg["rtol"], seed=seed, name=f"warmstart_{seed}")


def integer_tensor(shape, lo, hi, seed):
    """Integer-valued float64 tensor with entries in [lo, hi] (exact in bf16)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=tuple(shape)).astype(np.float64)

"""Seeded permeability fields and workload recipes.

All arrays are C-ordered with shape (nx, ny, nz), so the flat index of cell
(i, j, k) is (i*ny + j)*nz + k: z is the fastest index, x the slowest.
Permeabilities are in FP64. Random numbers come from NumPy's PCG64
(``numpy.random.default_rng``); a seed fully determines every field.

The paper runs one unspecified geomodel (injector to producer, Sec. V-B); the
workloads below are synthetic stand-ins with the statistics stated in each
recipe: independent log-normal cells, Gaussian-filtered (correlated)
log-normal fields, and a two-facies channelised field.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage


def lognormal_iid(shape, sigma: float, seed: int) -> np.ndarray:
    """k = exp(sigma * g), g ~ N(0, 1) independently per cell (mean of ln k = 0)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(tuple(shape)))


def lognormal_correlated(shape, sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """Correlated log-normal field.

    White noise is smoothed by a periodic Gaussian filter of standard deviation
    ``corr_len`` cells, re-standardised to zero mean and unit variance, scaled
    by ``sigma`` and exponentiated.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(tuple(shape))
    f = ndimage.gaussian_filter(g, sigma=corr_len, mode="wrap")
    del g
    f -= f.mean()
    f /= f.std()
    f *= sigma
    return np.exp(f, out=f)


def channelised(shape, seed: int, n_channels: int = 8, width: int = 6,
                amplitude: float = 12.0, wavelength: float = 64.0,
                k_channel: float = 1000.0, k_background: float = 1.0) -> np.ndarray:
    """Two-facies field: sinusoidal high-permeability channels in a background.

    Each channel runs along x. Its centreline in y is
    ``y0 + amplitude*sin(2*pi*x/wavelength + phase)``; a cell belongs to it when
    its y lies strictly within ``width/2`` of the centreline and its z lies in
    the band ``[z0, z0 + width)``. ``y0``, ``z0`` and the phase are drawn per
    channel from the seed.
    """
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    y0 = rng.uniform(0, ny, n_channels)
    z0 = rng.integers(0, max(1, nz - width + 1), n_channels)
    phase = rng.uniform(0, 2 * np.pi, n_channels)
    k = np.full((nx, ny, nz), k_background, dtype=np.float64)
    xs = np.arange(nx)[:, None]
    ys = np.arange(ny)[None, :]
    for c in range(n_channels):
        yc = y0[c] + amplitude * np.sin(2 * np.pi * xs / wavelength + phase[c])
        inside = np.abs(ys - yc) < width / 2.0            # (nx, ny)
        zlo, zhi = int(z0[c]), int(min(nz, z0[c] + width))
        k[:, :, zlo:zhi][inside] = k_channel
    return k


@dataclass
class BatchSystem:
    shape: tuple
    k: np.ndarray
    c: float


def batch_systems(n_systems: int = 64, lo: int = 32, hi: int = 128,
                  sigma: float = 1.5, dims_seed: int = 2, seed0: int = 2000,
                  with_fields: bool = True) -> list:
    """Independent systems of uneven sizes.

    Each dimension is an integer drawn uniformly from [lo, hi] (inclusive) by
    ``default_rng(dims_seed)``. System s draws, from ``default_rng(seed0 + s)``,
    first its accumulation ``c = 10**U(-4, -2)`` and then an independent
    log-normal field with the given sigma.
    """
    dims = np.random.default_rng(dims_seed).integers(lo, hi + 1, (n_systems, 3))
    out = []
    for s in range(n_systems):
        shape = tuple(int(v) for v in dims[s])
        rng = np.random.default_rng(seed0 + s)
        c = float(10.0 ** rng.uniform(-4.0, -2.0))
        k = np.exp(sigma * rng.standard_normal(shape)) if with_fields else None
        out.append(BatchSystem(shape=shape, k=k, c=c))
    return out


@dataclass
class Workload:
    """A single-system recipe: grid, permeability statistics, accumulation, tolerances."""
    name: str
    shape: tuple
    kind: str                      # "iid" | "correlated" | "channelised"
    sigma: float = 1.0
    corr_len: float = 0.0
    kz_ratio: float = 1.0          # k_z / k_x
    c: float = 1e-3                # accumulation per cell
    seed: int = 0
    tol: float = 1e-6              # relative residual target
    tol_refined: float = 1e-6      # target of FP64 iterative refinement
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))


WORKLOADS = {
    "lognormal_iid_32cube": Workload(
        "lognormal_iid_32cube", (32, 32, 32), "iid", sigma=1.0, c=1e-3, seed=0,
        notes="32^3 unit cells, ln k ~ N(0,1) iid, c=1e-3, x-plane Dirichlet 1/0"),
    "lognormal_corr8_256cube": Workload(
        "lognormal_corr8_256cube", (256, 256, 256), "correlated", sigma=2.0,
        corr_len=8.0, c=1e-3, seed=1, tol_refined=1e-8,
        notes="256^3, ln k Gaussian-filtered (8 cells), sigma=2, c=1e-3"),
    "channelised_128cube": Workload(
        "channelised_128cube", (128, 128, 128), "channelised", c=1e-3, seed=3500,
        notes="128^3 two-facies channels 1000/1 mD, c=1e-3"),
    "anisotropic_512x512x1024": Workload(
        "anisotropic_512x512x1024", (512, 512, 1024), "correlated", sigma=2.0,
        corr_len=8.0, kz_ratio=0.1, c=1e-4, seed=4, tol_refined=1e-8,
        notes="268M cells, ln k Gaussian-filtered (8 cells), sigma=2, kz/kx=0.1, c=1e-4"),
}


def workload_field(w: Workload, seed: int | None = None, shape=None) -> np.ndarray:
    """Permeability of a workload (optionally with another seed or shape)."""
    seed = w.seed if seed is None else seed
    shape = w.shape if shape is None else tuple(shape)
    if w.kind == "iid":
        return lognormal_iid(shape, w.sigma, seed)
    if w.kind == "correlated":
        return lognormal_correlated(shape, w.sigma, w.corr_len, seed)
    if w.kind == "channelised":
        return channelised(shape, seed)
    raise ValueError(f"unknown field kind {w.kind!r}")


def white_residuals(shape, count: int, seed: int) -> np.ndarray:
    """``count`` independent standard-normal fields of the grid's shape (FP32),
    each rescaled to unit RMS: random residuals for training the learned
    preconditioner."""
    rng = np.random.default_rng(seed)
    out = rng.standard_normal((count,) + tuple(shape)).astype(np.float32)
    out /= np.sqrt(np.mean(out.reshape(count, -1) ** 2, axis=1)).reshape((count,) + (1,) * len(shape))
    return out

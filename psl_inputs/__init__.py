"""Seeded synthetic workloads for the subdomain-levelset deflated PCG solve.

This module produces problem *inputs* only: a permeability field K, a source
vector q (wells), and the descriptors a caller hands to the solver (grid,
subdomain counts, levelset thresholds, Dirichlet face mask). It holds none of
the method's arithmetic (no transmissibilities, no labels, no coarse matrix,
no iteration), so both the CPU oracle and the GPU path can consume the same
inputs without sharing any computation.

Cell ordering everywhere: c = ix + nx*(iy + ny*iz); arrays are returned flat
(float64, C order over (nz, ny, nx)).

Workloads (the paper's datasets are not available; these stand in for them):
  * ``layered2d``   -- 2D sandwich of alternating high/low permeability rows,
                       the modified-SPE5 "sandwich" pattern of Section 2
                       repeated into a layered medium.
  * ``layered3d``   -- 3D horizontal layers, log-normal K per cell around
                       layer means that jump by a fixed contrast.
  * ``channelized`` -- thresholded Gaussian random field (channels vs
                       background), log-normal inside each facies; a synthetic
                       stand-in for the heterogeneity of SPE10 (Section 4,
                       Model D).
  * ``batch``       -- many independent layered systems of uneven size with
                       vertical well columns.
  * ``learned_x0_instance`` -- one random layered-or-channelized instance.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem",
    "rng",
    "layered2d",
    "layered3d",
    "channelized",
    "grf",
    "well_columns",
    "batch",
    "learned_x0_instance",
    "config",
    "CONFIG_NAMES",
]

# Dirichlet face mask bits (p = 0 on the masked outer faces, Neumann elsewhere)
X_LO, X_HI, Y_LO, Y_HI, Z_LO, Z_HI = 1, 2, 4, 8, 16, 32


@dataclasses.dataclass
class Problem:
    """One pressure-equation instance: -div(K grad p) = q on a unit-spacing grid."""

    grid: Tuple[int, int, int]          # (nx, ny, nz); nz == 1 -> 2D
    K: np.ndarray                       # float64 [n], isotropic permeability
    q: np.ndarray                       # float64 [n], sources (+) / sinks (-)
    nsub: Tuple[int, int, int]          # subdomains per axis (floor partition)
    thr: np.ndarray                     # float64 ascending levelset thresholds on K
    dirichlet_mask: int = X_LO          # which outer faces carry p = 0
    tol: float = 1e-8                   # relative residual target ||b-Ax||/||b||
    name: str = ""
    seed: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        nx, ny, nz = self.grid
        return nx * ny * nz


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _corner_source_sink(grid) -> np.ndarray:
    """Unit source in the first cell, unit sink in the last (opposite corners)."""
    nx, ny, nz = grid
    q = np.zeros(nx * ny * nz)
    q[0] = 1.0
    q[-1] = -1.0
    return q


def layered2d(nx: int = 64, ny: int = 64, rows_per_layer: int = 8, k_low: float = 1e-4,
              nsub=(4, 4), thr: float = 1e-2, seed: int = 0) -> Problem:
    """2D alternating layers: rows ``iy // rows_per_layer`` even -> K=1, odd -> k_low."""
    iy = np.arange(ny)
    layer = iy // rows_per_layer
    krow = np.where(layer % 2 == 0, 1.0, k_low)
    K = np.repeat(krow, nx).astype(np.float64)
    return Problem(grid=(nx, ny, 1), K=K, q=_corner_source_sink((nx, ny, 1)),
                   nsub=(nsub[0], nsub[1], 1), thr=np.array([thr]), name="layered2d",
                   seed=seed, meta={"k_low": k_low, "rows_per_layer": rows_per_layer})


def layered3d(nx: int = 128, ny: int = 128, nz: int = 64, nlayers: int = 8,
              contrast: float = 1e6, sigma_ln: float = 1.0, nsub=(8, 8, 4),
              thr: Optional[float] = None, seed: int = 0, wells: str = "corners") -> Problem:
    """3D horizontal layers L = (nlayers*iz)//nz; ln K ~ N(ln mu_L, sigma_ln^2) per cell,
    mu_L = 1 for even L and 1/contrast for odd L. Threshold defaults to the
    geometric mean of the two layer means."""
    g = rng(seed)
    iz = np.arange(nz)
    layer = (nlayers * iz) // nz
    ln_mu = np.where(layer % 2 == 0, 0.0, -math.log(contrast))
    lnK = ln_mu[:, None, None] + sigma_ln * g.standard_normal((nz, ny, nx))
    K = np.exp(lnK).reshape(-1)
    if thr is None:
        thr = 1.0 / math.sqrt(contrast)
    if wells == "corners":
        q = _corner_source_sink((nx, ny, nz))
    else:
        q = well_columns((nx, ny, nz), g)
    return Problem(grid=(nx, ny, nz), K=K, q=q, nsub=tuple(nsub), thr=np.array([thr]),
                   name="layered3d", seed=seed,
                   meta={"contrast": contrast, "sigma_ln": sigma_ln, "nlayers": nlayers})


def grf(shape: Sequence[int], corr_len: float, g: np.random.Generator) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field with covariance close to
    exp(-(r/corr_len)^2): white noise smoothed by a Gaussian kernel of standard
    deviation corr_len/2 per axis (the square-root kernel of that covariance),
    reflecting boundaries, then standardised. ``shape`` is (nz, ny, nx)."""
    from scipy.ndimage import gaussian_filter

    w = g.standard_normal(tuple(shape)).astype(np.float32)
    f = gaussian_filter(w, sigma=corr_len / 2.0, mode="reflect", truncate=3.0)
    f = f.astype(np.float64)
    f -= f.mean()
    f /= f.std()
    return f


def channelized(nx: int = 256, ny: int = 256, nz: int = 128, contrast: float = 1e6,
                corr_len: float = 16.0, channel_frac: float = 0.30, sigma_ln: float = 0.5,
                nsub=(16, 16, 8), seed: int = 0, wells: str = "corners") -> Problem:
    """Channel facies = GRF above its (1 - channel_frac) quantile; ln K ~ N(0, sigma_ln^2)
    in channels and N(-ln contrast, sigma_ln^2) in the background."""
    g = rng(seed)
    f = grf((nz, ny, nx), corr_len, g)
    cut = np.quantile(f, 1.0 - channel_frac)
    chan = f > cut
    lnK = np.where(chan, 0.0, -math.log(contrast)) + sigma_ln * g.standard_normal(f.shape)
    K = np.exp(lnK).reshape(-1)
    thr = 1.0 / math.sqrt(contrast)
    if wells == "corners":
        q = _corner_source_sink((nx, ny, nz))
    else:
        q = well_columns((nx, ny, nz), g)
    return Problem(grid=(nx, ny, nz), K=K, q=q, nsub=tuple(nsub), thr=np.array([thr]),
                   name="channelized", seed=seed,
                   meta={"contrast": contrast, "corr_len": corr_len,
                         "channel_frac": float(chan.mean())})


def well_columns(grid, g: np.random.Generator, n_inj: int = 2, n_prod: int = 2) -> np.ndarray:
    """Vertical well columns at random (ix, iy): injectors share +1 in total, producers
    -1 in total, each well's rate split evenly over its nz cells."""
    nx, ny, nz = grid
    q = np.zeros((nz, ny, nx))
    picks = g.choice(nx * ny, size=n_inj + n_prod, replace=False)
    for k, c in enumerate(picks):
        ix, iy = int(c % nx), int(c // nx)
        rate = (1.0 / n_inj) if k < n_inj else (-1.0 / n_prod)
        q[:, iy, ix] += rate / nz
    return q.reshape(-1)


def batch(nsys: int = 64, side_lo: int = 32, side_hi: int = 96, c_lo: float = 1e4,
          c_hi: float = 1e6, seed: int = 0) -> List[Problem]:
    """Independent cubic layered systems of seed-drawn side n_s ~ U{side_lo..side_hi},
    contrast log-uniform in [c_lo, c_hi], 4x4x4 subdomains x 2 levelsets, wells."""
    g = rng(seed)
    sides = g.integers(side_lo, side_hi + 1, size=nsys)
    cs = np.exp(g.uniform(math.log(c_lo), math.log(c_hi), size=nsys))
    out = []
    for i in range(nsys):
        s = int(sides[i])
        p = layered3d(s, s, s, nlayers=8, contrast=float(cs[i]), sigma_ln=1.0,
                      nsub=(4, 4, 4), seed=seed * 100003 + 17 + i, wells="columns")
        p.name = "batch"
        p.meta["index"] = i
        out.append(p)
    return out


def learned_x0_instance(seed: int, shape=(128, 128, 64), c_lo: float = 1e4,
                        c_hi: float = 1e6, nsub=(8, 8, 4)) -> Problem:
    """Random layered (even draw) or channelized (odd draw) instance with well columns."""
    g = rng(seed)
    kind = int(g.integers(0, 2))
    c = float(math.exp(g.uniform(math.log(c_lo), math.log(c_hi))))
    nx, ny, nz = shape
    sub_seed = int(g.integers(0, 2**31 - 1))
    if kind == 0:
        p = layered3d(nx, ny, nz, nlayers=8, contrast=c, sigma_ln=1.0, nsub=nsub,
                      seed=sub_seed, wells="columns")
    else:
        p = channelized(nx, ny, nz, contrast=c, corr_len=16.0, nsub=nsub, seed=sub_seed,
                        wells="columns")
    p.name = "learned_x0_" + ("layered" if kind == 0 else "channelized")
    p.seed = seed
    return p


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def config(name: str, seed: int = 0, scale: int = 1, **kw):
    """The five named workloads at full size (scale=1) or shrunk by ``scale`` per axis
    (small parity cases keep the same structure). ``c4`` returns a list."""
    if name == "c1":
        return layered2d(64 // scale if scale > 1 else 64, 64 // scale if scale > 1 else 64,
                         rows_per_layer=max(1, 8 // scale), seed=seed, **kw)
    if name == "c2":
        return layered3d(128 // scale, 128 // scale, 64 // scale, nlayers=8, contrast=1e6,
                         sigma_ln=1.0, nsub=(8, 8, 4), thr=1e-3, seed=seed, **kw)
    if name == "c3":
        contrast = kw.pop("contrast", (1e4, 1e5, 1e6, 1e7)[seed % 4])
        return channelized(256 // scale, 256 // scale, 128 // scale, contrast=contrast,
                           corr_len=16.0 / scale, nsub=(16, 16, 8), seed=seed, **kw)
    if name == "c4":
        if scale > 1:
            return batch(kw.pop("nsys", 8), max(8, 32 // scale), max(8, 96 // scale), seed=seed)
        return batch(seed=seed, **kw)
    if name == "c5":
        shape = (128 // scale, 128 // scale, 64 // scale)
        return learned_x0_instance(seed, shape=shape, **kw)
    raise KeyError(name)

"""Seeded synthetic workloads: configuration presets and coefficient generators.

This module holds sizes and seeded random media only; it contains none of the
homogenization arithmetic, so both the HIP path and the CPU oracle may import it.

Media follow the form used in the paper's numerical section (Sec. 4): a
piecewise-constant high-contrast field k(x) times a slowly varying modulation.
The paper's own k fields exist only as figures, so seeded channel / inclusion
media of the same character stand in for them:

* channels: horizontal (2D) or x1-aligned (3D) stripes two fine elements wide,
  one per period of 8 elements, each shifted by a seeded integer jitter in
  [-2, 2] (2D: one draw per channel; 3D: two draws per channel, x2 then x3, in
  row-major (a, b) order);
* inclusions (N = 3 preset): discs of radius 3h, uniformly placed, membership by
  element centroid with periodic wrap, overriding channels;
* modulation m(x) = 1 + 0.5 * prod_k sin(2 pi x_k) at element centroids;
* kappa = value(label) * m(x) with matrix 1, channel 1e4, inclusion 1e-4.

Array layout: element e = i1 + n1*(i2 + n2*i3); numpy arrays are C-ordered
with shape (n3, n2, n1) / (n2, n1), x1 fastest. Labels are uint8: 0 matrix,
1 channel, 2 inclusion.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MATRIX, CHANNEL, INCLUSION = 0, 1, 2
VALUES = {MATRIX: 1.0, CHANNEL: 1.0e4, INCLUSION: 1.0e-4}


@dataclasses.dataclass(frozen=True)
class Config:
    """Mirror of the C struct ``mch_config`` (include/mch.h)."""

    dim: int
    n_fine: int          # fine elements per axis of the unit square / cube
    n_macro: int         # macropoints per axis
    n_cell: int          # oversampled cell width in fine elements
    n_sub: int           # constraint sub-blocks per axis
    n_cont: int          # number of continua N
    levels: int = 1      # L
    eta: int = 2         # coarsening factor
    interp: int = 0      # 0: inherit the level-1 solution of the group (paper's experiments)
    bc: int = 0          # 0: homogeneous Dirichlet on the cell boundary
    rtol: float = 1e-13  # Krylov tolerance on the preconditioned residual (relative)
    max_iter: int = 4000

    @property
    def h(self) -> float:
        return 1.0 / self.n_fine

    @property
    def H_el(self) -> int:
        return self.n_fine // self.n_macro

    @property
    def n_rhs(self) -> int:
        return self.n_cont * (1 + self.dim)

    @property
    def n_points(self) -> int:
        return self.n_macro ** self.dim

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


PRESETS = {
    # flat L=1, 2D, 128^2 fine grid, 8x8 macropoints, 32^2 cells
    "c1": Config(dim=2, n_fine=128, n_macro=8, n_cell=32, n_sub=2, n_cont=2, levels=1),
    # hierarchical L=3, eta=2, 512^2 fine grid, 32x32 macropoints, 64^2 cells
    "c2": Config(dim=2, n_fine=512, n_macro=32, n_cell=64, n_sub=4, n_cont=2, levels=3),
    "c2flat": Config(dim=2, n_fine=512, n_macro=32, n_cell=64, n_sub=4, n_cont=2, levels=1),
    # the same with multilinear inheritance from T_(n-1)
    "c2ml": Config(dim=2, n_fine=512, n_macro=32, n_cell=64, n_sub=4, n_cont=2, levels=3, interp=1),
    # 3D hierarchical L=2, 128^3, 8^3 macropoints, 32^3 cells
    "c3": Config(dim=3, n_fine=128, n_macro=8, n_cell=32, n_sub=2, n_cont=2, levels=2),
    "c3flat": Config(dim=3, n_fine=128, n_macro=8, n_cell=32, n_sub=2, n_cont=2, levels=1),
    # large uneven batch: 2048^2, 256^2 macropoints, N=3, L=4
    "c5": Config(dim=2, n_fine=2048, n_macro=256, n_cell=64, n_sub=2, n_cont=3, levels=4),
    "c5ml": Config(dim=2, n_fine=2048, n_macro=256, n_cell=64, n_sub=2, n_cont=3, levels=4, interp=1),
    # small cases for unit tests (several tiles, fast on the CPU)
    # larger oversampled cells: 128^2 fine elements (4H, H = 32; level widths
    # 128, 64, 32), and a block-aligned cell of 3 x 3 coarse blocks centred on
    # K_p with the constraint regions the blocks themselves (one coarse layer
    # of oversampling; level widths 96, 48, 24)
    "c6": Config(dim=2, n_fine=512, n_macro=16, n_cell=128, n_sub=4, n_cont=2, levels=3),
    "c7": Config(dim=2, n_fine=512, n_macro=16, n_cell=96, n_sub=3, n_cont=2, levels=3),
    "t2": Config(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=2),
    "t3": Config(dim=2, n_fine=128, n_macro=16, n_cell=32, n_sub=2, n_cont=2, levels=3),
    "t3d": Config(dim=3, n_fine=32, n_macro=4, n_cell=16, n_sub=2, n_cont=2, levels=2),
}
PRESET_SEEDS = {"c1": 1, "c2": 2, "c2flat": 2, "c2ml": 2, "c3": 3, "c3flat": 3, "c5": 5, "c5ml": 5, "c6": 6, "c7": 10,
                "t2": 7, "t3": 8, "t3d": 9}


def _modulation(n: int, dim: int) -> np.ndarray:
    x = (np.arange(n) + 0.5) / n
    s = np.sin(2.0 * np.pi * x)
    if dim == 2:
        return 1.0 + 0.5 * s[:, None] * s[None, :]
    return 1.0 + 0.5 * s[:, None, None] * s[None, :, None] * s[None, None, :]


def channel_labels(n: int, dim: int, seed: int, period: int = 8) -> np.ndarray:
    """Channel labels; one jitter draw per channel (2D) or two (3D)."""
    rng = np.random.default_rng(seed)
    nch = n // period
    shape = (n,) * dim
    lab = np.zeros(shape, np.uint8)
    if dim == 2:
        jit = rng.integers(-2, 3, size=nch)
        for c in range(nch):
            rows = (period * c + 3 + jit[c] + np.arange(2)) % n
            lab[rows, :] = CHANNEL
    else:
        jit = rng.integers(-2, 3, size=(nch, nch, 2))  # (a, b) row-major, x2 then x3
        for a in range(nch):
            for b in range(nch):
                r2 = (period * a + 3 + jit[a, b, 0] + np.arange(2)) % n
                r3 = (period * b + 3 + jit[a, b, 1] + np.arange(2)) % n
                lab[np.ix_(r3, r2, np.arange(n))] = CHANNEL
    return lab


def add_inclusions(lab: np.ndarray, seed: int, radius_el: float = 3.0, fraction: float = 0.10) -> np.ndarray:
    """Overlay discs of radius ``radius_el`` fine elements (2D only)."""
    n = lab.shape[0]
    count = int(round(fraction * n * n / (9.0 * math.pi)))
    rng = np.random.default_rng(seed)
    centres = rng.random((count, 2)) * n  # (x1, x2) in element units
    out = lab.copy()
    r = int(math.ceil(radius_el)) + 1
    off = np.arange(-r, r + 1)
    for c1, c2 in centres:
        i1 = np.floor(c1).astype(int) + off
        i2 = np.floor(c2).astype(int) + off
        d1 = (i1 + 0.5) - c1
        d2 = (i2 + 0.5) - c2
        inside = d2[:, None] ** 2 + d1[None, :] ** 2 <= radius_el ** 2
        ii2, ii1 = np.nonzero(inside)
        out[i2[ii2] % n, i1[ii1] % n] = INCLUSION
    return out


def kappa_from_labels(lab: np.ndarray, channel_factor: float = 1.0) -> np.ndarray:
    n = lab.shape[0]
    vals = np.array([VALUES[MATRIX], VALUES[CHANNEL] * channel_factor, VALUES[INCLUSION]])
    return vals[lab] * _modulation(n, lab.ndim)


def source_from_labels(lab: np.ndarray) -> np.ndarray:
    """Source term per fine element, of the form used in the paper's examples
    (Sec. 4): exp(-40 |x - 1/2|^2) at the element centroid, times 1e-4 outside
    the high-conductivity channels (the contrast of the low-conductivity
    continuum)."""
    n = lab.shape[0]
    x = (np.arange(n) + 0.5) / n
    r2 = (x - 0.5) ** 2
    if lab.ndim == 2:
        g = np.exp(-40.0 * (r2[:, None] + r2[None, :]))
    else:
        g = np.exp(-40.0 * (r2[:, None, None] + r2[None, :, None] + r2[None, None, :]))
    return np.where(lab == CHANNEL, 1.0, 1.0e-4) * g


def medium(name: str, seed: int | None = None, channel_factor: float = 1.0):
    """Return (kappa float64, label uint8) on the preset's global fine grid."""
    cfg = PRESETS[name]
    if seed is None:
        seed = PRESET_SEEDS[name]
    lab = channel_labels(cfg.n_fine, cfg.dim, seed)
    if cfg.n_cont == 3:
        lab = add_inclusions(lab, seed * 11)
    return kappa_from_labels(lab, channel_factor), lab


def medium_for(cfg: Config, seed: int, channel_factor: float = 1.0, inclusions: bool | None = None):
    """Channel medium (plus inclusions when N = 3) for an arbitrary config."""
    lab = channel_labels(cfg.n_fine, cfg.dim, seed)
    if inclusions or (inclusions is None and cfg.n_cont == 3):
        lab = add_inclusions(lab, seed * 11)
    return kappa_from_labels(lab, channel_factor), lab


def target_factor(seed: int = 4) -> float:
    """Lognormal(0, 0.3) factor on the channel value for the adjoint target."""
    z = np.random.default_rng(seed).standard_normal()
    return float(np.exp(0.3 * z))


def fd_elements(lab: np.ndarray, seed: int = 44, n_each: int = 10) -> np.ndarray:
    """Flat indices of n_each channel and n_each matrix elements, without replacement."""
    rng = np.random.default_rng(seed)
    flat = lab.reshape(-1)
    ch = np.flatnonzero(flat == CHANNEL)
    mx = np.flatnonzero(flat == MATRIX)
    return np.concatenate([rng.choice(ch, n_each, replace=False), rng.choice(mx, n_each, replace=False)])

"""Oracle, part 6: the global fine-grid problem, the reference of the paper's Type 1 and Type 2 errors.

TEST INFRASTRUCTURE ONLY.

Sec. 4 compares the multiscale solutions with the fine-grid solution u
through its continuum averages per coarse block (Eq. U_h_defi):
U_h^(i)(p) = int_{K_p cap Omega_i} u / |K_p cap Omega_i|. Type 1 is e_2
between U_h and the flat (MH) block averages, Type 2 between U_h and the
hierarchical (HMH) ones. Readings, as for the macroscopic system: the fine
problem is -div(kappa grad u) = f on the unit square / cube with u = 0 on its
boundary, discretised by Q1 on the fine elements (the elements of the cells),
with f piecewise constant per element; Omega_i is the union of the elements
labelled i, and the integrals of the Q1 function u over an element are |e|
times the mean of its corner values.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def fine_solution(kappa: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Nodal u [(n+1)^d] of the global fine problem (zero on the boundary)."""
    dim, n = kappa.ndim, kappa.shape[0]
    h = 1.0 / n
    K = fem.assemble_stiffness(kappa, h)
    nodes = fem.element_nodes(n, dim)
    F = np.zeros((n + 1) ** dim)
    np.add.at(F, nodes.reshape(-1), np.repeat(f.reshape(-1) * h ** dim / 2 ** dim, 2 ** dim))
    free = fem.free_nodes(n, dim)
    u = np.zeros((n + 1) ** dim)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), F[free])
    return u


def continuum_block_averages(u: np.ndarray, label: np.ndarray, n_macro: int, n_cont: int) -> np.ndarray:
    """U_h[p, i]: the average of u over K_p cap Omega_i (NaN where the block has no element of i)."""
    dim, n = label.ndim, label.shape[0]
    H = n // n_macro
    nodes = fem.element_nodes(n, dim)
    ue = u[nodes].mean(axis=1)  # element means, x1 fastest
    ac = fem.element_coords(n, dim)
    blk = np.zeros(len(ac), np.int64)
    stride = 1
    for k in range(dim):
        blk += (ac[:, k] // H) * stride
        stride *= n_macro
    lab = label.reshape(-1)
    out = np.full((n_macro ** dim, n_cont), np.nan)
    for i in range(n_cont):
        m = lab == i
        s = np.bincount(blk[m], weights=ue[m], minlength=n_macro ** dim)
        c = np.bincount(blk[m], minlength=n_macro ** dim)
        ok = c > 0
        out[ok, i] = s[ok] / c[ok]
    return out


def e2(Uref: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Per continuum sqrt(sum |Uref - U|^2 / sum |Uref|^2) over the blocks where Uref is defined."""
    ok = np.isfinite(Uref)
    d = np.where(ok, Uref - U, 0.0)
    r = np.where(ok, Uref, 0.0)
    return np.sqrt((d ** 2).sum(axis=0) / (r ** 2).sum(axis=0))

"""Oracle, part 2: the hierarchy of macrogrids (paper Sec. 3.1, Eq. defi_Sn; Figs. 2-3).

TEST INFRASTRUCTURE ONLY.

Nested macrogrids T_1 subset ... subset T_L = T, where T_n keeps, per axis, the
macropoint indices congruent to o modulo eta^(L-n), with o = floor(eta^(L-1)/2)
(this phase reproduces the 8x8, L=3, eta=2 example of Figs. 2-3).
S_1 = T_1 and S_n = T_n minus the union of earlier S_k.

Interpolation (paper's experiments, Sec. 3.3): a macropoint of level n >= 2
inherits the local solutions of the level-1 macropoint of its aligned
eta^(L-1)-per-axis block of macropoints, with weight c_t = 1.
"""
from __future__ import annotations

import numpy as np


def macro_coords(n_macro: int, dim: int) -> np.ndarray:
    """[P, dim] macro index per axis (j1 fastest), p = j1 + nm*(j2 + nm*j3)."""
    p = np.arange(n_macro ** dim)
    return np.stack([(p // n_macro ** k) % n_macro for k in range(dim)], axis=1)


def in_T(j: np.ndarray, n: int, L: int, eta: int) -> np.ndarray:
    o = (eta ** (L - 1)) // 2
    step = eta ** (L - n)
    return np.all((j - o) % step == 0, axis=1)


def levels(n_macro: int, dim: int, L: int, eta: int) -> np.ndarray:
    """Level (1..L) of every macropoint."""
    j = macro_coords(n_macro, dim)
    lev = np.zeros(len(j), np.int64)
    for n in range(L, 0, -1):
        lev[in_T(j, n, L, eta)] = n
    return lev


def parents(n_macro: int, dim: int, L: int, eta: int) -> np.ndarray:
    """Index of the inherited level-1 macropoint (-1 for level-1 points)."""
    j = macro_coords(n_macro, dim)
    lev = levels(n_macro, dim, L, eta)
    g = eta ** (L - 1)
    o = g // 2
    pj = (j // g) * g + o
    par = np.zeros(len(j), np.int64)
    stride = 1
    for k in range(dim):
        par += pj[:, k] * stride
        stride *= n_macro
    par[lev == 1] = -1
    return par

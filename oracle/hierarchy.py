"""Oracle, part 2: the hierarchy of macrogrids (paper Sec. 3.1, Eq. defi_Sn; Figs. 2-3).

TEST INFRASTRUCTURE ONLY.

Nested macrogrids T_1 subset ... subset T_L = T, where T_n keeps, per axis, the
macropoint indices congruent to o modulo eta^(L-n), with o = floor(eta^(L-1)/2)
(this phase reproduces the 8x8, L=3, eta=2 example of Figs. 2-3).
S_1 = T_1 and S_n = T_n minus the union of earlier S_k.

Interpolation (Sec. 3.3, Eq. phiXiI_all): a macropoint of level n >= 2 takes
I = sum_t c_t Phi_t over neighbours t in the union of S_k, k < n (= T_(n-1)),
with sum_t c_t = 1.
* interp = 0 (the paper's experiments): the single neighbour is the level-1
  macropoint of the aligned eta^(L-1)-per-axis block, c_t = 1.
* interp = 1 (multilinear): per axis, the two T_(n-1) lattice indices that
  bracket the point's index (lattice step eta^(L-n+1), periodic in the
  macropoint index), with the 1D linear-interpolation weights; the neighbours
  are their tensor products with weight the product of the 1D weights (axis 1
  fastest), zero weights left out. Every neighbour lies within one lattice
  step per axis, i.e. within O(eta^(L-n) H).
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


def _axis_bracket(i: int, step: int, o: int, n_macro: int):
    """1D neighbours of index i on the lattice {o + k*step}, periodic in n_macro."""
    lo = o + ((i - o) // step) * step
    frac = (i - lo) / step
    if frac == 0.0:
        return [(lo % n_macro, 1.0)]
    return [(lo % n_macro, 1.0 - frac), ((lo + step) % n_macro, frac)]


def interp_weights(n_macro: int, dim: int, L: int, eta: int, interp: int):
    """Per macropoint, the list [(t, c_t), ...] of Eq. phiXiI_all ([] on level 1)."""
    lev = levels(n_macro, dim, L, eta)
    j = macro_coords(n_macro, dim)
    if interp == 0:
        par = parents(n_macro, dim, L, eta)
        return [[] if lev[p] == 1 else [(int(par[p]), 1.0)] for p in range(len(j))]
    o = (eta ** (L - 1)) // 2
    out = []
    for p in range(len(j)):
        n = int(lev[p])
        if n == 1:
            out.append([])
            continue
        step = eta ** (L - n + 1)
        axes = [_axis_bracket(int(j[p, k]), step, o, n_macro) for k in range(dim)]
        combos = [(0, 1.0)]
        stride = 1
        for k in range(dim):
            # the new axis is the outer loop, so axis 1 varies fastest
            combos = [(t + i * stride, c * w) for (i, w) in axes[k] for (t, c) in combos]
            stride *= n_macro
        out.append(combos)
    return out

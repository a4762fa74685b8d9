"""Oracle, part 4: Algorithm 1 steps 1-4 over all macropoints, and the adjoint gradient.

TEST INFRASTRUCTURE ONLY.

Forward (paper Algorithm 1): build S_1..S_L, then for n = 1..L solve every
cell of S_n (level-1 cells from scratch, later levels as inherited solution
plus correction in V_n), then form the effective tensors (Eq. Bs_defi).

Backward (not in the paper; derived from the same equations): for a loss with
G_p = dLoss/dA_eff(p), per cell

    Phibar_a = sum_b (G_ab + G_ba) K^{K_p} Phi_b   (+ seeds from inheriting cells)
    [K_n B_n^T; B_n 0][w_a; mu_a] = [P_n^T Phibar_a; 0]
    dLoss/dkappa_e += -(P_n w_a)|_e^T K_ref Phi_a|_e              (every e in the cell)
                      + sum_ab G_ab Phi_a|_e^T K_ref Phi_b|_e   (e in K_p)
    Ibar_a = Phibar_a - K_h P_n w_a - B_h^T mu_a   -> c_t Ibar_a added to the seed of
                                                    every point t the cell inherits from,

processed from level L down to level 1, and finally dLoss/dlog kappa = kappa * dLoss/dkappa.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import cells, fem, hierarchy

_G = {}


def _init(cfg, kappa, label):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    _G["cfg"], _G["kappa"], _G["label"] = cfg, kappa, label


def _fwd_one(args):
    p, level, I_full = args
    cfg = _G["cfg"]
    cs = cells.assemble_cell(cfg, _G["kappa"], _G["label"], p, level)
    Phi, xi, beta = cells.solve_cell(cs, I_full, cfg.n_rhs)
    A = cells.effective_tensor(cs, Phi)
    return p, Phi, A, beta


def _pool_map(fn, items, workers):
    if workers <= 1 or len(items) < 2:
        return [fn(it) for it in items]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init, initargs=(_G["cfg"], _G["kappa"], _G["label"])) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (4 * workers)))


class Forward:
    def __init__(self, cfg, lev, par, inherit, A, Phi, beta):
        self.cfg, self.level, self.parent, self.inherit = cfg, lev, par, inherit
        self.A, self.Phi, self.beta = A, Phi, beta


def _inherited(inherit_p, Phi):
    """I = sum_t c_t Phi_t (Eq. phiXiI_all), None for a level-1 point."""
    if not inherit_p:
        return None
    I = None
    for t, c in inherit_p:
        I = c * Phi[t] if I is None else I + c * Phi[t]
    return I


def forward(cfg, kappa, label, points=None, workers: int | None = None) -> Forward:
    """Solve the cells of ``points`` (default: all) plus every point they inherit from.

    Returns per-point local solutions Phi [n_nodes, M] (all cell nodes), multipliers,
    and effective tensors A_eff [M, M] (dicts keyed by macropoint index).
    """
    workers = workers if workers is not None else (os.cpu_count() or 1)
    lev = hierarchy.levels(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
    par = hierarchy.parents(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
    inherit = hierarchy.interp_weights(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta, cfg.interp)
    if points is None:
        points = np.arange(cfg.n_points)
    need = set(int(p) for p in np.asarray(points))
    todo = list(need)
    while todo:  # close the set under "inherits from"
        q = todo.pop()
        for t, _ in inherit[q]:
            if t not in need:
                need.add(t)
                todo.append(t)
    _init(cfg, kappa, label)
    Phi, A, beta = {}, {}, {}
    for n in range(1, cfg.levels + 1):
        todo = [p for p in sorted(need) if lev[p] == n]
        items = [(p, n, _inherited(inherit[p], Phi)) for p in todo]
        for p, ph, a, b in _pool_map(_fwd_one, items, workers):
            Phi[p], A[p], beta[p] = ph, a, b
    return Forward(cfg, lev, par, inherit, A, Phi, beta)


def _bwd_one(args):
    p, level, I_full, Phi, G, seed = args
    cfg = _G["cfg"]
    cs = cells.assemble_cell(cfg, _G["kappa"], _G["label"], p, level)
    dim, h = cfg.dim, cfg.h
    Phibar = cs.Kkp @ (Phi @ (G + G.T))  # [n_nodes, M]
    Phibar_f = Phibar[cs.free]
    if seed is not None:
        Phibar_f = Phibar_f + seed
    m = cs.Bn.shape[0]
    w, mu = cells.kkt_solve(cs, cs.P.T @ Phibar_f, np.zeros((m, cfg.n_rhs)))
    Pw = np.zeros((cs.n_nodes, cfg.n_rhs))
    Pw[cs.free] = cs.P @ w
    nodes = fem.element_nodes(cfg.n_cell, dim)
    kr = fem.kref(dim, h)
    Phe = Phi[nodes]   # [n_elem, 2^d, M]
    Pwe = Pw[nodes]
    KPhe = np.einsum("cd,edm->ecm", kr, Phe)
    gk = -np.einsum("ecm,ecm->e", Pwe, KPhe)
    kpm = fem.kp_element_mask(cfg.n_cell, cfg.H_el, dim)
    gk[kpm] += np.einsum("ecm,mn,ecn->e", Phe[kpm], G, KPhe[kpm])
    Ibar = None
    if I_full is not None:
        Ibar = Phibar_f - cs.Kf @ (cs.P @ w) - cs.Bf.T @ mu
    return p, gk, Ibar


def backward(cfg, kappa, label, fwd: Forward, gA: dict, workers: int | None = None) -> np.ndarray:
    """Gradient of the loss w.r.t. log kappa per global fine element, given gA[p] = dLoss/dA_eff(p).

    Requires a forward over all macropoints.
    """
    workers = workers if workers is not None else (os.cpu_count() or 1)
    _init(cfg, kappa, label)
    n = cfg.n_fine
    gk = np.zeros(n ** cfg.dim)
    seeds = {}
    for lvl in range(cfg.levels, 0, -1):
        todo = [p for p in range(cfg.n_points) if fwd.level[p] == lvl]
        items = []
        for p in todo:
            I_full = _inherited(fwd.inherit[p], fwd.Phi)
            items.append((p, lvl, I_full, fwd.Phi[p], np.asarray(gA[p]), seeds.get(p)))
        for p, gke, Ibar in _pool_map(_bwd_one, items, workers):
            idx = fem.window_flat_indices(n, cells.cell_origin(cfg, p), cfg.n_cell, cfg.dim)
            np.add.at(gk, idx, gke)
            if Ibar is not None:
                for t, c in fwd.inherit[p]:
                    seeds[t] = seeds.get(t, 0.0) + c * Ibar
    return (kappa.reshape(-1) * gk).reshape(kappa.shape)


def stack_A(fwd: Forward, cfg) -> np.ndarray:
    return np.stack([fwd.A[p] for p in range(cfg.n_points)])

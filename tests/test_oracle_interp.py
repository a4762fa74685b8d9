"""Pins for the oracle's multilinear interpolation mode (interp = 1; no GPU).

Sec. 3.3, Eq. phiXiI_all: a level-n macropoint takes I = sum_t c_t Phi_t over
neighbours t in T_(n-1) with sum_t c_t = 1 and distance O(eta^(L-n) H). The
multilinear reading takes, per axis, the two T_(n-1) lattice indices that
bracket the point with 1D linear weights, and their tensor products.
"""
import numpy as np
import pytest

import oracle
from oracle import cells, fem, hierarchy
from paper_2503_01276_amd import workloads as W

from test_oracle_solve import _dense_hier_solution


def _unwrap(d, n):
    """Periodic difference mapped into (-n/2, n/2]."""
    d = (d + n // 2) % n - n // 2
    return np.where(d == -(n // 2), n // 2, d) if n % 2 == 0 else d


def test_hand_example_8x8_L3():
    # 8x8 macropoints, L = 3, eta = 2 (the grid of Figs. 2-3): T_1 = {2, 6}^2,
    # T_2 = even indices. Weights derived by hand from the bracketing rule.
    w = hierarchy.interp_weights(8, 2, 3, 2, 1)
    lev = hierarchy.levels(8, 2, 3, 2)

    def P(i, j):
        return i + 8 * j

    # level 2 at (0, 0): per axis T_1 neighbours 6 (index -2 wrapped) and 2, weight 1/2 each
    assert lev[P(0, 0)] == 2
    assert w[P(0, 0)] == [(P(6, 6), 0.25), (P(2, 6), 0.25), (P(6, 2), 0.25), (P(2, 2), 0.25)]
    # level 2 at (4, 2): on the T_1 lattice in x2, halfway between 2 and 6 in x1
    assert lev[P(4, 2)] == 2
    assert w[P(4, 2)] == [(P(2, 2), 0.5), (P(6, 2), 0.5)]
    # level 3 at (1, 1): T_2 neighbours 0 and 2 per axis
    assert lev[P(1, 1)] == 3
    assert w[P(1, 1)] == [(P(0, 0), 0.25), (P(2, 0), 0.25), (P(0, 2), 0.25), (P(2, 2), 0.25)]
    # level 3 at (7, 4): x1 between 6 and 8 = 0 (wrapped), on the lattice in x2
    assert lev[P(7, 4)] == 3
    assert w[P(7, 4)] == [(P(6, 4), 0.5), (P(0, 4), 0.5)]
    # level-1 points inherit nothing
    assert w[P(2, 2)] == [] and w[P(6, 2)] == []


@pytest.mark.parametrize("nm,dim,L,eta", [(32, 2, 3, 2), (256, 2, 4, 2), (16, 2, 3, 2), (8, 3, 2, 2),
                                          (27, 2, 3, 3), (8, 3, 3, 2)])
def test_weights_partition_of_unity_and_linear_reproduction(nm, dim, L, eta):
    w = hierarchy.interp_weights(nm, dim, L, eta, 1)
    lev = hierarchy.levels(nm, dim, L, eta)
    j = hierarchy.macro_coords(nm, dim)
    for p in range(nm ** dim):
        n = lev[p]
        if n == 1:
            assert w[p] == []
            continue
        ts = np.array([t for t, _ in w[p]])
        cs = np.array([c for _, c in w[p]])
        assert abs(cs.sum() - 1.0) < 1e-15 and np.all(cs > 0)
        assert np.all(lev[ts] < n)  # neighbours in T_(n-1)
        step = eta ** (L - n + 1)
        d = _unwrap(j[ts] - j[p], nm)  # [k, dim]
        assert np.all(np.abs(d) < step)  # within one T_(n-1) lattice step per axis
        # linear functions of the (unwrapped) macro position are reproduced exactly
        assert np.all(np.abs(cs @ d) < 1e-12)
        # one neighbour per lattice-aligned axis, two per other axis
        off = int(np.sum((j[p] - (eta ** (L - 1)) // 2) % step != 0))
        assert len(ts) == 2 ** off and off >= 1


def _cfg_t3(**kw):
    base = dict(dim=2, n_fine=128, n_macro=16, n_cell=32, n_sub=2, n_cont=2, levels=3, interp=1)
    base.update(kw)
    return W.Config(**base)


def test_interp0_lists_match_group_parents():
    cfg = _cfg_t3(interp=0)
    w = hierarchy.interp_weights(cfg.n_macro, 2, cfg.levels, cfg.eta, 0)
    par = hierarchy.parents(cfg.n_macro, 2, cfg.levels, cfg.eta)
    for p in range(cfg.n_points):
        assert w[p] == ([] if par[p] < 0 else [(int(par[p]), 1.0)])


def test_fine_constraints_and_bruteforce_with_weighted_I():
    # P3 and P4 in interp = 1: each hierarchical cell meets the fine
    # constraints and equals a dense null-space minimisation over
    # I + V_n with I = sum_t c_t Phi_t formed here from the weights.
    cfg = _cfg_t3()
    k, l = W.medium_for(cfg, 3)
    pts = [p for p in range(0, cfg.n_points, 11)]
    fwd = oracle.forward(cfg, k, l, points=pts, workers=1)
    assert set(pts) <= set(fwd.Phi)
    checked = 0
    for p in pts:
        n = int(fwd.level[p])
        cs = cells.assemble_cell(cfg, k, l, p, n)
        assert np.abs(cs.Bf @ fwd.Phi[p][cs.free] - cs.g).max() < 1e-12
        if n == 1:
            continue
        I_full = sum(c * fwd.Phi[t] for t, c in fwd.inherit[p])
        dense = _dense_hier_solution(cs, I_full, cfg.n_rhs)
        got = fwd.Phi[p][cs.free]
        assert np.abs(got - dense).max() < 1e-10 * np.abs(dense).max()
        checked += 1
    assert checked >= 10


def test_exact_rescaling_gives_zero_correction_multilinear():
    # P10 in interp = 1: kappa of every cell is a multiple of every other's
    # with identical labels, so sum_t c_t = 1 gives g' = 0 and f in the range
    # of B_n^T: Xi_p = 0, Phi_p = Phi_t and A(p) = c A(t) for each neighbour.
    cfg = _cfg_t3()
    n = cfg.n_fine
    l = np.zeros((n, n), np.uint8)
    for c in range(n // 8):
        l[(8 * c + 3 + np.arange(2)) % n, :] = 1
    x = (np.arange(n) + 0.5) / n
    g = np.exp((x[None, :] + x[:, None]) / 2)
    k = np.where(l == 1, 1e4, 1.0) * g
    lev = hierarchy.levels(cfg.n_macro, 2, cfg.levels, cfg.eta)
    w = hierarchy.interp_weights(cfg.n_macro, 2, cfg.levels, cfg.eta, 1)

    def no_wrap(q):
        org = cells.cell_origin(cfg, q)
        return all(0 <= o and o + cfg.n_cell <= n for o in org)

    def closed(q):
        return no_wrap(q) and all(closed(t) for t, _ in w[q])

    pts = [p for p in range(cfg.n_points) if lev[p] >= 2 and closed(p)][::3]
    assert len(pts) >= 5
    f = oracle.forward(cfg, k, l, points=pts, workers=1)
    for p in pts:
        for t, _ in f.inherit[p]:
            jp = np.array([p % 16, p // 16])
            jt = np.array([t % 16, t // 16])
            c = np.exp(((jp - jt) * cfg.H_el * cfg.h).sum() / 2)
            assert np.linalg.norm(f.A[p] - c * f.A[t]) < 1e-11 * np.linalg.norm(f.A[p])
            assert np.abs(f.Phi[p] - f.Phi[t]).max() < 1e-11


def test_energy_above_flat_multilinear():
    # P12: I + V_n is a subset of V_h for any inherited I.
    cfg = _cfg_t3()
    k, l = W.medium_for(cfg, 5)
    pts = list(range(0, cfg.n_points, 13))
    fh = oracle.forward(cfg, k, l, points=pts, workers=1)
    ff = oracle.forward(cfg.replace(levels=1), k, l, points=pts, workers=1)
    for p in pts:
        cs = cells.assemble_cell(cfg, k, l, p, 1)
        K = fem.assemble_stiffness(cs.kc, cfg.h)
        Jh = np.einsum("na,na->a", fh.Phi[p], K @ fh.Phi[p])
        Jf = np.einsum("na,na->a", ff.Phi[p], K @ ff.Phi[p])
        assert np.all(Jh >= Jf * (1 - 1e-12))


def test_adjoint_vs_complex_step_multilinear_L3():
    # P13 through the multilinear chain: level-2 points are both inheritors
    # (of level 1) and neighbours (of level 3), so their adjoint carries seeds
    # from level 3 and passes c_t Ibar on to level 1.
    cfg = _cfg_t3(n_fine=64, n_macro=8, n_cell=32)
    k, l = W.medium_for(cfg, 9)
    kt, _ = W.medium_for(cfg, 9, channel_factor=W.target_factor(4))
    T = oracle.stack_A(oracle.forward(cfg, kt, l, workers=4), cfg)
    fwd = oracle.forward(cfg, k, l, workers=4)
    A = oracle.stack_A(fwd, cfg)
    gA = {p: 2 * (A[p] - T[p]) for p in range(cfg.n_points)}
    g = oracle.backward(cfg, k, l, fwd, gA, workers=4).reshape(-1)
    delta = 1e-30
    for e in W.fd_elements(l, seed=44, n_each=2):
        kc = k.astype(complex).reshape(-1)
        kc[e] *= 1 + 1j * delta
        Ac = oracle.stack_A(oracle.forward(cfg, kc.reshape(k.shape), l, workers=4), cfg)
        dL = np.imag(np.sum((Ac - T) ** 2)) / delta
        assert abs(dL - g[e]) <= 1e-9 * max(abs(dL), 1e-12 * np.abs(g).max()), (e, dL, g[e])

"""Pins for the oracle's cell solves, hierarchy and effective tensors (no GPU)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import cells, fem, hierarchy
from paper_2503_01276_amd import workloads as W

HERE = os.path.dirname(__file__)


def _load_golden():
    sets = {}
    with open(os.path.join(HERE, "golden", "hierarchy_fig2_fig3.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, *vals = line.split()
            sets[name] = vals
    return sets


def test_hierarchy_matches_paper_figures():
    # Paper Sec. 3.1, Figs. 2-3: 8x8 macropoints, L = 3, eta = 2.
    g = _load_golden()
    lev = hierarchy.levels(8, 2, 3, 2)
    j = hierarchy.macro_coords(8, 2)

    def pts(vals):
        v = list(map(int, vals))
        return {(v[k], v[k + 1]) for k in range(0, len(v), 2)}

    S = {n: {tuple(j[p]) for p in range(64) if lev[p] == n} for n in (1, 2, 3)}
    assert S[1] == pts(g["S1"])
    assert S[2] == pts(g["S2"])
    assert len(S[3]) == int(g["S3_count"][0])
    assert all(i % 2 == 1 or jj % 2 == 1 for i, jj in S[3])
    T1 = {tuple(j[p]) for p in range(64) if hierarchy.in_T(j[p:p + 1], 1, 3, 2)[0]}
    T2 = {tuple(j[p]) for p in range(64) if hierarchy.in_T(j[p:p + 1], 2, 3, 2)[0]}
    assert T1 == pts(g["T1"]) and T2 == pts(g["T2"])


@pytest.mark.parametrize("dim,L,counts", [(2, 3, (1, 3, 12)), (2, 2, (1, 3)), (3, 2, (1, 7))])
def test_group_counts(dim, L, counts):
    # One level-1 macropoint and its inheritors: 1/3/12 (Sec. 3.3 and Table
    # tab:cpu2dL3), 1/3 (Table tab:cpu2dL2), 1/7 (Table tab:cpu3dL2).
    nm = 2 ** (L - 1) * 2
    lev = hierarchy.levels(nm, dim, L, 2)
    par = hierarchy.parents(nm, dim, L, 2)
    t = int(np.flatnonzero(lev == 1)[0])
    group = [p for p in range(nm ** dim) if p == t or par[p] == t]
    got = tuple(sum(1 for p in group if lev[p] == n) for n in range(1, L + 1))
    assert got == counts


def test_parents_are_level1_in_same_block():
    lev = hierarchy.levels(32, 2, 3, 2)
    par = hierarchy.parents(32, 2, 3, 2)
    j = hierarchy.macro_coords(32, 2)
    for p in range(32 * 32):
        if lev[p] == 1:
            assert par[p] == -1
        else:
            assert lev[par[p]] == 1
            assert np.all(j[p] // 4 == j[par[p]] // 4)
    assert np.bincount(lev)[1:].tolist() == [64, 192, 768]


def _cfg_small(**kw):
    base = dict(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=2, eta=2)
    base.update(kw)
    return W.Config(**base)


def _medium(cfg, seed=3):
    return W.medium_for(cfg, seed)


def test_kkt_residual_and_fine_constraints():
    # P3: every solve satisfies the KKT system and the *fine* constraints
    # B_h Phi = g, including hierarchical cells (B_h Phi = B_h I + B_n xi = g).
    cfg = _cfg_small(levels=3, n_fine=128, n_macro=16, n_cell=32)
    k, l = _medium(cfg)
    fwd = oracle.forward(cfg, k, l, points=range(0, cfg.n_points, 7), workers=1)
    for p, Phi in fwd.Phi.items():
        cs = cells.assemble_cell(cfg, k, l, p, int(fwd.level[p]))
        assert np.abs(cs.Bf @ Phi[cs.free] - cs.g).max() < 1e-12
        # stationarity: P^T K_h Phi + B_n^T beta = 0
        res = cs.P.T @ (cs.Kf @ Phi[cs.free]) + cs.Bn.T @ fwd.beta[p]
        scale = np.abs(cs.Kf @ Phi[cs.free]).max()
        assert np.abs(res).max() < 1e-10 * scale


def _dense_hier_solution(cs, I_full, M):
    """Brute force: minimise J over {I + P xi} subject to B_h Phi = g via a dense null-space basis."""
    K = cs.Kf.toarray()
    P = cs.P.toarray()
    Bn = cs.Bf @ P
    nf = len(cs.free)
    If = np.zeros((nf, M)) if I_full is None else I_full[cs.free]
    out = []
    Z = sla.null_space(Bn)
    for a in range(M):
        # particular solution of Bn xi = g - B I (least norm), then minimise over null space
        rhs = cs.g[:, a] - cs.Bf @ If[:, a]
        xi0 = np.linalg.lstsq(Bn, rhs, rcond=None)[0]
        Kn = P.T @ K @ P
        grad0 = P.T @ (K @ (If[:, a] + P @ xi0))
        y = np.linalg.solve(Z.T @ Kn @ Z, -Z.T @ grad0)
        out.append(If[:, a] + P @ (xi0 + Z @ y))
    return np.stack(out, axis=1)


def test_sparse_equals_dense_bruteforce():
    # P4: sparse SuperLU KKT path equals a dense null-space minimisation.
    cfg = _cfg_small(n_fine=32, n_macro=4, n_cell=8, levels=2)
    k, l = _medium(cfg, seed=11)
    fwd = oracle.forward(cfg, k, l, workers=1)
    for p in range(cfg.n_points):
        cs = cells.assemble_cell(cfg, k, l, p, int(fwd.level[p]))
        I_full = fwd.Phi[fwd.parent[p]] if fwd.level[p] > 1 else None
        dense = _dense_hier_solution(cs, I_full, cfg.n_rhs)
        got = fwd.Phi[p][cs.free]
        assert np.abs(got - dense).max() < 1e-11 * np.abs(dense).max()


def test_scaling_invariance():
    # P5: Phi(c kappa) = Phi(kappa), A(c kappa) = c A(kappa).
    cfg = _cfg_small()
    k, l = _medium(cfg)
    f1 = oracle.forward(cfg, k, l, workers=1)
    f2 = oracle.forward(cfg, 3.7 * k, l, workers=1)
    for p in range(cfg.n_points):
        assert np.allclose(f2.Phi[p], f1.Phi[p], atol=1e-11 * np.abs(f1.Phi[p]).max())
        assert np.allclose(f2.A[p], 3.7 * f1.A[p], rtol=0, atol=1e-10 * np.abs(f2.A[p]).max())


def test_symmetric_psd_and_isotropy():
    # P6: A_eff symmetric PSD; N = 1 with constant kappa gives an isotropic
    # B^{mn} block with zero off-diagonal and zero mixed B^m block.
    cfg = _cfg_small(n_cont=1, levels=1)
    k = np.full((cfg.n_fine,) * 2, 2.0)
    l = np.zeros_like(k, dtype=np.uint8)
    f = oracle.forward(cfg, k, l, points=[9], workers=1)
    A = f.A[9]
    assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > -1e-12 * np.abs(A).max()
    s = np.abs(A).max()
    assert abs(A[1, 1] - A[2, 2]) < 1e-12 * s
    assert abs(A[1, 2]) < 1e-12 * s and abs(A[0, 1]) < 1e-12 * s and abs(A[0, 2]) < 1e-12 * s


def test_mirror_symmetry():
    # P6: kappa, labels invariant under x1 -> -x1 about the cell centre
    # (unjittered horizontal channels, no modulation): type-2 solutions along
    # x1 decouple from the others, so A[j, N + i*d + 0] = 0 and the (x1, x2)
    # entries of B^{mn} vanish.
    cfg = _cfg_small(levels=1)
    n = cfg.n_fine
    l = np.zeros((n, n), np.uint8)
    for c in range(n // 8):
        l[(8 * c + 3 + np.arange(2)) % n, :] = 1
    k = np.where(l == 1, 1e4, 1.0)
    f = oracle.forward(cfg, k, l, points=[18], workers=1)
    A = f.A[18]
    N, d = 2, 2
    s = np.abs(A).max()
    for j in range(N):
        for i in range(N):
            assert abs(A[j, N + i * d + 0]) < 1e-10 * s
            assert abs(A[N + j * d + 0, N + i * d + 1]) < 1e-10 * s


def test_single_region_gives_zero_type2():
    # P7: s = 1, N = 1, cell centred on K_p: the type-2 right-hand side is
    # x-bar - c = 0 for symmetric placement only if the centroids coincide;
    # with constant labels they do, so phi^m == 0.
    cfg = _cfg_small(n_cont=1, n_sub=1, levels=1)
    rng = np.random.default_rng(2)
    k = np.exp(rng.standard_normal((cfg.n_fine,) * 2))
    l = np.zeros_like(k, dtype=np.uint8)
    f = oracle.forward(cfg, k, l, points=[10], workers=1)
    Phi = f.Phi[10]
    assert np.abs(Phi[:, 1:]).max() == 0.0 or np.abs(Phi[:, 1:]).max() < 1e-14
    assert np.abs(Phi[:, 0]).max() > 0.5


def test_L1_equals_flat_and_eta1():
    # P9: L = 1 is the flat method; eta = 1 puts every macropoint on level 1.
    cfg = _cfg_small(levels=1)
    k, l = _medium(cfg)
    f1 = oracle.forward(cfg, k, l, workers=1)
    f2 = oracle.forward(cfg.replace(levels=3, eta=1), k, l, workers=1)
    assert np.all(f2.level == 1)
    for p in range(cfg.n_points):
        assert np.array_equal(f1.A[p], f2.A[p])


def test_exact_rescaling_gives_zero_correction():
    # P10: kappa_p = c * kappa_t with identical labels (period-H medium times a
    # multiplicative modulation, cells without wrap) => Xi_p = 0 and
    # A(p) = c A(t): the mechanism of the paper's machine-precision Type-3
    # error in Example 5 (Table tab:Herror5).
    cfg = W.Config(dim=2, n_fine=128, n_macro=16, n_cell=32, n_sub=2, n_cont=2, levels=3)
    n = cfg.n_fine
    l = np.zeros((n, n), np.uint8)
    for c in range(n // 8):
        l[(8 * c + 3 + np.arange(2)) % n, :] = 1
    x = (np.arange(n) + 0.5) / n
    g = np.exp((x[None, :] + x[:, None]) / 2)
    k = np.where(l == 1, 1e4, 1.0) * g
    par = hierarchy.parents(cfg.n_macro, 2, cfg.levels, cfg.eta)

    def no_wrap(q):
        org = cells.cell_origin(cfg, q)
        return all(0 <= o and o + cfg.n_cell <= n for o in org)

    pts = [p for p in range(cfg.n_points) if no_wrap(p) and (par[p] < 0 or no_wrap(par[p]))]
    f = oracle.forward(cfg, k, l, points=pts[::5], workers=1)
    checked = 0
    for p in pts[::5]:
        if f.level[p] == 1:
            continue
        t = int(f.parent[p])
        jp = np.array([p % 16, p // 16])
        jt = np.array([t % 16, t // 16])
        c = np.exp(((jp - jt) * cfg.H_el * cfg.h).sum() / 2)
        assert np.linalg.norm(f.A[p] - c * f.A[t]) < 1e-11 * np.linalg.norm(f.A[p])
        assert np.abs(f.Phi[p] - f.Phi[t]).max() < 1e-11
        checked += 1
    assert checked >= 5


def test_hierarchical_energy_above_flat():
    # P12: V_n subset V_h, so the hierarchical minimiser has energy over the
    # oversampled cell at least that of the flat one, per (p, alpha).
    cfg = _cfg_small(levels=2)
    k, l = _medium(cfg)
    fh = oracle.forward(cfg, k, l, workers=1)
    ff = oracle.forward(cfg.replace(levels=1), k, l, workers=1)
    for p in range(cfg.n_points):
        cs = cells.assemble_cell(cfg, k, l, p, 1)
        K = fem.assemble_stiffness(cs.kc, cfg.h)
        Jh = np.einsum("na,na->a", fh.Phi[p], K @ fh.Phi[p])
        Jf = np.einsum("na,na->a", ff.Phi[p], K @ ff.Phi[p])
        assert np.all(Jh >= Jf * (1 - 1e-12))

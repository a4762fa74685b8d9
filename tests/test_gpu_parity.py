"""Parity of the HIP path with the oracle, through the C ABI (needs an MI355X).

Bars: local solutions 1e-8 relative (2-norm per cell and right-hand side),
effective tensors 1e-9 relative (Frobenius per macropoint), constraints
B_h Phi = g to 1e-12, integer hierarchy bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import check_forward, gpu_forward

pytestmark = pytest.mark.gpu

_check = check_forward


def test_hierarchy_matches_oracle():
    from paper_2503_01276_amd import mch
    for name in ("c1", "c2", "t2", "t3", "c5"):
        cfg = W.PRESETS[name]
        plan = mch.Plan(cfg) if name != "c5" else None
        lev, par = (plan.hierarchy() if plan else mch.build_hierarchy(cfg))
        olev = oracle.hierarchy.levels(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
        opar = oracle.hierarchy.parents(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
        assert np.array_equal(lev, olev) and np.array_equal(par, opar), name


def test_small_hierarchical_L2_full():
    cfg = W.PRESETS["t2"]
    k, l = W.medium("t2")
    _check("t2", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=1)


def test_flat_c1_full():
    cfg = W.PRESETS["c1"]
    k, l = W.medium("c1")
    _check("c1", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=1)


def test_hierarchical_L3_small_full():
    cfg = W.PRESETS["t3"]
    k, l = W.medium("t3")
    _check("t3", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=1)


def test_hierarchical_c2_all_tensors_sampled_phi():
    cfg = W.PRESETS["c2"]
    k, l = W.medium("c2")
    lev = oracle.hierarchy.levels(cfg.n_macro, 2, cfg.levels, cfg.eta)
    par = oracle.hierarchy.parents(cfg.n_macro, 2, cfg.levels, cfg.eta)
    t = int(np.flatnonzero(lev == 1)[5])
    group = [t] + [int(p) for p in np.flatnonzero(par == t)]
    sample = sorted(set(group) | set(range(0, cfg.n_points, 97)))
    _check("c2", cfg, k, l, phi_cells=sample, workers=1)


def test_determinism_bitwise():
    cfg = W.PRESETS["t3"]
    k, l = W.medium("t3")
    _, A1, _, _, _, _ = gpu_forward(cfg, k, l)
    _, A2, _, _, _, _ = gpu_forward(cfg, k, l)
    assert np.array_equal(A1, A2)


def test_workgroup_numbering_is_bitwise_neutral(monkeypatch):
    # the 2D solve's XCD-grouped workgroup order (default) and plain order
    # (MCH_XCD=0) solve the same (cell, rhs) pairs with the same arithmetic;
    # 49 level-1 cells (six whole groups of 8 and a tail of 1) and 147
    # level-2 cells (18 groups and a tail of 3)
    cfg = W.Config(dim=2, n_fine=168, n_macro=14, n_cell=32, n_sub=2, n_cont=2, levels=2)
    k, l = W.medium_for(cfg, 41)
    _, A1, _, _, _, _ = gpu_forward(cfg, k, l)
    monkeypatch.setenv("MCH_XCD", "0")
    _, A2, _, _, _, _ = gpu_forward(cfg, k, l)
    assert np.array_equal(A1, A2)


def test_L1_plan_equals_flat_bitwise():
    # a hierarchical configuration with L = 1 runs the flat path exactly
    cfg = W.PRESETS["t2"].replace(levels=1)
    k, l = W.medium("t2")
    _, A1, _, _, _, _ = gpu_forward(cfg, k, l)
    _, A2, _, _, _, _ = gpu_forward(cfg.replace(eta=3), k, l)
    assert np.array_equal(A1, A2)


def test_band_correction_two_sub_bands(monkeypatch):
    # 64^2 fine cells over 8 x 8 coarse blocks of 8 elements (the shape of the
    # 2048^2 batch, where the two sub-bands pay off), three continua with
    # inclusions, the band correction on two sub-bands of 4 node rows per
    # thread (MCH_PREC_64=2): forward on every cell and the adjoint gradient
    # against the oracle
    from gpu_util import grad_case

    monkeypatch.setenv("MCH_PREC_64", "2")
    cfg = W.Config(dim=2, n_fine=128, n_macro=16, n_cell=64, n_sub=2, n_cont=3, levels=2)
    k, l = W.medium_for(cfg, 51)
    plan, _ = _check("two sub-bands", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=8)
    info = (plan.band_subbands[0], plan.rows_per_thread[0])
    plan.close()
    assert info == (2, 8), info
    grad_case("two sub-bands", cfg, 52, workers=8)

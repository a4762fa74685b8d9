"""Adjoint gradient of the HIP path versus the oracle's (needs an MI355X).

Loss: sum_p ||A_eff(p) - A_target(p)||_F^2 with the target computed by the
oracle from a medium whose channel value carries a seeded lognormal factor.
Both sides receive the same dLoss/dA_eff, so the comparison isolates the
backward pass. Bar: relative 2-norm over the field <= 1e-8.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-8


def _grad_case(name, cfg, seed):
    import torch

    from paper_2503_01276_amd import mch

    k, l = W.medium_for(cfg, seed)
    kt, _ = W.medium_for(cfg, seed, channel_factor=W.target_factor(4))
    say(f"[gpu] {name}: oracle forward (target and medium)")
    T = oracle.stack_A(oracle.forward(cfg, kt, l, workers=1), cfg)
    fwd = oracle.forward(cfg, k, l, workers=1)
    A = oracle.stack_A(fwd, cfg)
    gA = 2.0 * (A - T)
    say(f"[gpu] {name}: oracle backward")
    gref = oracle.backward(cfg, k, l, fwd, {p: gA[p] for p in range(cfg.n_points)}, workers=1).reshape(-1)
    say(f"[gpu] {name}: GPU forward + backward")
    plan = mch.Plan(cfg)
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    plan.solve_cells(kd, ld)
    Ad = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    plan.effective_coeffs(kd, Ad)
    gAd = torch.from_numpy(gA.reshape(-1).copy()).to(dev)
    gd = torch.empty_like(kd)
    plan.effective_coeffs_backward(kd, gAd, gd)
    torch.cuda.synchronize()
    g = gd.cpu().numpy()
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"[gpu] {name}: grad rel err {err:.3e} (|g| = {np.linalg.norm(gref):.3e})")
    assert err <= GRAD_TOL, err
    return g, gref


def test_adjoint_flat_small():
    cfg = W.Config(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=1)
    _grad_case("adj-flat", cfg, 9)


def test_adjoint_hierarchical_L2_small():
    cfg = W.PRESETS["t2"]
    _grad_case("adj-t2", cfg, 9)


def test_adjoint_hierarchical_L3():
    cfg = W.PRESETS["t3"]
    _grad_case("adj-t3", cfg, 8)

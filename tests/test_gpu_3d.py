"""3D cells through the C ABI (needs an MI355X): local solutions, effective
tensors and the adjoint gradient of the HIP path against the oracle.

Bars as in 2D: Phi 1e-8, A_eff 1e-9, fine constraints 1e-12, gradient 1e-8,
finite differences 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import check_forward, gpu_forward, grad_case, say

pytestmark = pytest.mark.gpu


def test_3d_small_L2_full():
    # 32^3 grid, 4^3 macropoints, 16^3 cells (level 2 on 8^3 at 2h): every cell
    cfg = W.PRESETS["t3d"]
    k, l = W.medium("t3d")
    check_forward("t3d", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=4)


def test_3d_c3_sampled():
    # 128^3 grid, 8^3 macropoints, 32^3 cells, levels 32^3 / 16^3: all tensors of
    # one level-1 group and two more points, Phi of the group's first four cells
    cfg = W.PRESETS["c3"]
    k, l = W.medium("c3")
    lev = oracle.hierarchy.levels(cfg.n_macro, 3, cfg.levels, cfg.eta)
    par = oracle.hierarchy.parents(cfg.n_macro, 3, cfg.levels, cfg.eta)
    t = int(np.flatnonzero(lev == 1)[9])
    group = [t] + [int(p) for p in np.flatnonzero(par == t)]
    pts = sorted(set(group) | {0, cfg.n_points - 1})
    check_forward("c3", cfg, k, l, phi_cells=group[:4], a_points=pts, workers=8)


def test_3d_determinism_bitwise():
    cfg = W.PRESETS["t3d"]
    k, l = W.medium("t3d")
    _, A1, _, _, _, _ = gpu_forward(cfg, k, l)
    _, A2, _, _, _, _ = gpu_forward(cfg, k, l)
    assert np.array_equal(A1, A2)


def test_3d_adjoint_small():
    grad_case("adj-t3d", W.PRESETS["t3d"], 9, workers=4)


def test_3d_c3_finite_differences():
    # adjoint of the full 3D configuration against central differences of the
    # GPU forward (delta = 1e-3 in log kappa) on 6 channel and 6 matrix elements
    import torch

    from paper_2503_01276_amd import autograd, mch

    cfg = W.PRESETS["c3"]
    k, l = W.medium("c3")
    kt, _ = W.medium("c3", channel_factor=W.target_factor(4))
    dev = torch.device("cuda:0")
    plan = mch.Plan(cfg)
    lab = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    with torch.no_grad():
        T = autograd.effective_tensors(torch.from_numpy(np.log(kt).reshape(-1)).to(dev), lab, plan).clone()
    logk = torch.from_numpy(np.log(k).reshape(-1)).to(dev).requires_grad_(True)
    A = autograd.effective_tensors(logk, lab, plan)
    ((A - T) ** 2).sum().backward()
    torch.cuda.synchronize()
    it, _ = plan.diagnostics(adjoint=True)
    say(f"[gpu] c3: adjoint iterations min/median/max {it.min()}/{int(np.median(it))}/{it.max()}")
    g = logk.grad.detach().cpu().numpy()
    base = logk.detach().clone()
    d = 1e-3
    worst = 0.0
    for e in W.fd_elements(l, seed=44, n_each=6):
        vals = []
        for sgn in (1.0, -1.0):
            lk = base.clone()
            lk[int(e)] += sgn * d
            with torch.no_grad():
                Ae = autograd.effective_tensors(lk, lab, plan)
                vals.append(float(((Ae - T) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * d)
        tol = 1e-4 * abs(fd) + 1e-8 * np.abs(g).max()
        worst = max(worst, abs(fd - g[e]) / max(abs(fd), 1e-300))
        assert abs(fd - g[e]) <= tol, (int(e), fd, g[e])
    say(f"[gpu] c3: worst FD relative difference {worst:.2e}")

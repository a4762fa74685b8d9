"""Multilinear interpolation (interp = 1) on the HIP path, through the C ABI (needs an MI355X).

A level-n point inherits I = sum_t c_t Phi_t over the points of T_(n-1) that
bracket it (Sec. 3.3, Eq. phiXiI_all), so the levels form a chain: level n
reads the fine solutions of every level below it, and the adjoint passes
c_t Ibar back down. Same bars as the paper-mode parity tests: Phi 1e-8,
A_eff 1e-9, gradient 1e-8 relative; finite differences 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import check_forward, gpu_forward, grad_case, say

pytestmark = pytest.mark.gpu


def test_t3_multilinear_full():
    cfg = W.PRESETS["t3"].replace(interp=1)
    k, l = W.medium("t3")
    check_forward("t3 ml", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=8)


def test_t2_multilinear_full():
    # L = 2: every neighbour is a level-1 point, 2 or 4 of them per point
    cfg = W.PRESETS["t2"].replace(interp=1)
    k, l = W.medium("t2")
    check_forward("t2 ml", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=8)


def test_t3_multilinear_adjoint():
    grad_case("adj-t3 ml", W.PRESETS["t3"].replace(interp=1), 8, workers=8)


def _t4_three_continua():
    # L = 4 with three continua (contrast 1e8): levels 2 and 3 both receive
    # seeds from above and pass them down; the kernel shapes of the 2048^2
    # workload (64^2 cells, s = 2, N = 3)
    return W.Config(dim=2, n_fine=256, n_macro=16, n_cell=64, n_sub=2, n_cont=3, levels=4, interp=1)


def test_L4_three_continua_multilinear_full():
    cfg = _t4_three_continua()
    k, l = W.medium_for(cfg, 12)
    check_forward("t4 ml N=3", cfg, k, l, phi_cells=list(range(0, cfg.n_points, 5)), workers=8)


def test_L4_three_continua_multilinear_adjoint():
    # Contrast 1e8: at the default tolerance 1e-12 the gradient meets the
    # relative 2-norm bar (3.6e-10) but its largest element errors are
    # 2e-10 of the field's maximum, above the element-wise bar; they come
    # from the Krylov tolerance (1.3e-11 at 1e-13, 7.7e-13 at 1e-14), so the
    # element-wise check runs at rtol = 1e-14.
    grad_case("adj-t4 ml N=3", _t4_three_continua().replace(rtol=1e-14), 12, workers=8)


def test_c2_multilinear_all_tensors_sampled_phi():
    cfg = W.PRESETS["c2"].replace(interp=1)
    k, l = W.medium("c2")
    lev = oracle.hierarchy.levels(cfg.n_macro, 2, cfg.levels, cfg.eta)
    sample = sorted(set(int(p) for p in np.flatnonzero(lev == 3)[:6]) | set(range(0, cfg.n_points, 97)))
    check_forward("c2 ml", cfg, k, l, phi_cells=sample, workers=8)


def test_c2_multilinear_gradient_full_field():
    # the whole gradient field at full size against the oracle's backward
    grad_case("adj-c2 ml", W.PRESETS["c2ml"], W.PRESET_SEEDS["c2ml"], workers=16)


def _loss_and_grad(plan, kd, ld, T, want_grad):
    import torch

    A = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=kd.device)
    plan.solve_cells(kd, ld)
    plan.effective_coeffs(kd, A)
    loss = float(((A - T) ** 2).sum())
    g = None
    if want_grad:
        g = torch.empty_like(kd)
        plan.effective_coeffs_backward(kd, 2.0 * (A - T), g)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
    return loss, g


def test_c2_multilinear_finite_differences():
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["c2"].replace(interp=1)
    k, l = W.medium("c2")
    kt, _ = W.medium("c2", channel_factor=W.target_factor(4))
    dev = torch.device("cuda:0")
    plan = mch.Plan(cfg)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    T = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    ktd = torch.from_numpy(kt.reshape(-1).copy()).to(dev)
    plan.solve_cells(ktd, ld)
    plan.effective_coeffs(ktd, T)
    base = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    _, g = _loss_and_grad(plan, base, ld, T, True)
    d = 1e-3
    worst = 0.0
    for e in W.fd_elements(l, seed=44, n_each=3):
        vals = []
        for sgn in (1.0, -1.0):
            kd = base.clone()
            kd[int(e)] *= np.exp(sgn * d)
            vals.append(_loss_and_grad(plan, kd, ld, T, False)[0])
        fd = (vals[0] - vals[1]) / (2 * d)
        worst = max(worst, abs(fd - g[e]) / max(abs(fd), 1e-300))
        assert abs(fd - g[e]) <= 1e-4 * abs(fd) + 1e-8 * np.abs(g).max(), (int(e), fd, g[e])
    say(f"[gpu] c2 ml: worst FD relative difference {worst:.2e}")


@pytest.mark.parametrize("preset", ["t3", "t3d"])
def test_multilinear_eager_equals_graph_replays(preset):
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS[preset].replace(interp=1)
    k, l = W.medium(preset)
    dev = torch.device("cuda:0")
    plan = mch.Plan(cfg)
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    n = plan.P * plan.M * plan.M
    A0 = torch.empty(n, dtype=torch.float64, device=dev)
    g0 = torch.empty_like(kd)
    plan.solve_cells(kd, ld)
    plan.effective_coeffs(kd, A0)
    gA = (A0 * 1e-3).contiguous()
    plan.effective_coeffs_backward(kd, gA, g0)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    A = torch.empty_like(A0)
    g = torch.empty_like(g0)
    with torch.cuda.stream(st):
        for rep in range(3):
            plan.solve_cells(kd, ld)
            plan.effective_coeffs(kd, A)
            plan.effective_coeffs_backward(kd, gA, g)
            st.synchronize()
            assert torch.equal(A, A0), rep
            assert torch.equal(g, g0), rep
            A.zero_()
            g.zero_()
            _ = (kd * 2.0).sum().item()
    _, A2, _, _, _, _ = gpu_forward(cfg, k, l)
    assert np.array_equal(A2, A0.cpu().numpy().reshape(A2.shape))
    say(f"[gpu] {preset} ml: eager, 3 graph replays and a fresh plan agree bitwise")


def test_t3d_multilinear_full():
    # 3D, L = 2: every level-2 point interpolates from up to 8 level-1 points
    cfg = W.PRESETS["t3d"].replace(interp=1)
    k, l = W.medium("t3d")
    check_forward("t3d ml", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=8)


def test_t3d_multilinear_adjoint():
    grad_case("adj-t3d ml", W.PRESETS["t3d"].replace(interp=1), 9, workers=8)


def test_3d_L3_multilinear_sampled_and_finite_differences():
    # 3D, L = 3 (32^3 / 16^3 / 8^3 cells): level-2 points both inherit and are
    # inherited from, so their adjoint takes the level-3 seeds through P^T at
    # r = 2. Oracle parity on sampled cells, finite differences of the GPU path.
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.Config(dim=3, n_fine=64, n_macro=8, n_cell=32, n_sub=2, n_cont=2, levels=3, interp=1)
    k, l = W.medium_for(cfg, 13)
    lev = oracle.hierarchy.levels(cfg.n_macro, 3, cfg.levels, cfg.eta)
    pts = [int(np.flatnonzero(lev == 3)[0]), int(np.flatnonzero(lev == 3)[200]), int(np.flatnonzero(lev == 2)[10])]
    check_forward("3d L3 ml", cfg, k, l, phi_cells=pts, a_points=pts, workers=8)
    kt, _ = W.medium_for(cfg, 13, channel_factor=W.target_factor(4))
    dev = torch.device("cuda:0")
    plan = mch.Plan(cfg)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    ktd = torch.from_numpy(kt.reshape(-1).copy()).to(dev)
    T = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    plan.solve_cells(ktd, ld)
    plan.effective_coeffs(ktd, T)
    base = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    _, g = _loss_and_grad(plan, base, ld, T, True)
    d = 1e-3
    worst = 0.0
    for e in W.fd_elements(l, seed=44, n_each=2):
        vals = []
        for sgn in (1.0, -1.0):
            kd = base.clone()
            kd[int(e)] *= np.exp(sgn * d)
            vals.append(_loss_and_grad(plan, kd, ld, T, False)[0])
        fd = (vals[0] - vals[1]) / (2 * d)
        worst = max(worst, abs(fd - g[e]) / max(abs(fd), 1e-300))
        assert abs(fd - g[e]) <= 1e-4 * abs(fd) + 1e-8 * np.abs(g).max(), (int(e), fd, g[e])
    say(f"[gpu] 3d L3 ml: worst FD relative difference {worst:.2e}")

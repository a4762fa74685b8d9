"""Edge cases of the HIP path (needs an MI355X): one and three continua in 2D
and 3D, non-convergence reporting, unsupported shapes, call-order errors and
degenerate argument lists, all through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import check_forward, grad_case, say

pytestmark = pytest.mark.gpu


def _inclusion_blocks_3d(lab: np.ndarray, seed: int, count: int) -> np.ndarray:
    """Mark `count` seeded 2x2x2 element blocks as the third continuum."""
    rng = np.random.default_rng(seed)
    n = lab.shape[0]
    out = lab.copy()
    for c in rng.integers(0, n, size=(count, 3)):
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    out[(c[2] + dz) % n, (c[1] + dy) % n, (c[0] + dx) % n] = W.INCLUSION
    return out


def test_single_continuum_2d():
    cfg = W.PRESETS["t2"].replace(n_cont=1)
    k, _ = W.medium("t2")
    l = np.zeros_like(k, dtype=np.uint8)
    check_forward("t2 N=1", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=4)


def test_single_continuum_3d():
    cfg = W.PRESETS["t3d"].replace(n_cont=1)
    k, _ = W.medium("t3d")
    l = np.zeros_like(k, dtype=np.uint8)
    check_forward("t3d N=1", cfg, k, l, phi_cells=list(range(0, cfg.n_points, 5)), workers=4)


def test_three_continua_3d_and_adjoint():
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["t3d"].replace(n_cont=3)
    _, l0 = W.medium("t3d")
    l = _inclusion_blocks_3d(l0, seed=91, count=60)
    k = W.kappa_from_labels(l)
    say(f"[gpu] t3d N=3: label counts {np.bincount(l.reshape(-1), minlength=3).tolist()}")
    check_forward("t3d N=3", cfg, k, l, phi_cells=list(range(0, cfg.n_points, 3)), workers=4)
    # adjoint against the oracle's with a seeded dLoss/dA
    fwd = oracle.forward(cfg, k, l, workers=4)
    rng = np.random.default_rng(92)
    gA = rng.standard_normal((cfg.n_points, cfg.n_rhs, cfg.n_rhs))
    gref = oracle.backward(cfg, k, l, fwd, {p: gA[p] for p in range(cfg.n_points)}, workers=4).reshape(-1)
    plan = mch.Plan(cfg)
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    plan.solve_cells(kd, ld)
    A = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    plan.effective_coeffs(kd, A)
    g = torch.empty_like(kd)
    plan.effective_coeffs_backward(kd, torch.from_numpy(gA.reshape(-1).copy()).to(dev), g)
    torch.cuda.synchronize()
    err = np.linalg.norm(g.cpu().numpy() - gref) / np.linalg.norm(gref)
    say(f"[gpu] t3d N=3: grad rel err {err:.3e}")
    assert err <= 1e-8, err


def test_no_convergence_is_reported():
    import torch

    from paper_2503_01276_amd import mch

    for name in ("t2", "t3d"):
        cfg = W.PRESETS[name].replace(max_iter=3)
        k, l = W.medium(name)
        plan = mch.Plan(cfg)
        dev = torch.device("cuda:0")
        plan.solve_cells(torch.from_numpy(k.reshape(-1).copy()).to(dev), torch.from_numpy(l.reshape(-1).copy()).to(dev))
        torch.cuda.synchronize()
        with pytest.raises(mch.MchError) as ei:
            plan.diagnostics()
        assert ei.value.code == mch.MCH_ENOCONV
        it, rs = plan.diagnostics(allow_noconv=True)
        assert it.max() == 3 and rs.max() > cfg.rtol


def test_unsupported_3d_shapes_are_refused():
    from paper_2503_01276_amd import mch

    base = W.PRESETS["t3d"]
    for cfg in (base.replace(n_sub=1), base.replace(n_fine=128, n_macro=2, n_cell=64, levels=1)):
        with pytest.raises(mch.MchError) as ei:
            mch.Plan(cfg)
        assert ei.value.code == mch.MCH_ENOTIMPL, (cfg, ei.value)


def test_call_order_and_argument_errors():
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["t2"]
    k, l = W.medium("t2")
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    plan = mch.Plan(cfg)
    A = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
    g = torch.empty_like(kd)
    with pytest.raises(mch.MchError) as ei:
        plan.effective_coeffs(kd, A)
    assert ei.value.code == mch.MCH_ESTALE
    with pytest.raises(mch.MchError) as ei:
        plan.effective_coeffs_backward(kd, torch.zeros_like(A), g)
    assert ei.value.code == mch.MCH_ESTALE
    plan.solve_cells(kd, ld)
    # empty list of local solutions is a no-op; an out-of-range index is refused
    plan.local_solutions(np.zeros(0, np.int64), torch.empty(0, dtype=torch.float64, device=dev))
    nn = (cfg.n_cell + 1) ** cfg.dim
    with pytest.raises(mch.MchError) as ei:
        plan.local_solutions(np.array([cfg.n_points]), torch.empty(plan.M * nn, dtype=torch.float64, device=dev))
    assert ei.value.code == mch.MCH_EINVAL
    # wrong dtype / size of a device buffer
    with pytest.raises(mch.MchError):
        plan.effective_coeffs(kd, torch.empty(3, dtype=torch.float64, device=dev))
    # a zero gradient of the loss gives a zero gradient field
    plan.effective_coeffs(kd, A)
    plan.effective_coeffs_backward(kd, torch.zeros_like(A), g)
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0


def test_one_and_eight_subblocks_2d():
    # the solve kernels are compiled per number of sub-blocks per axis; the
    # workloads use 2 and 4, these cover 1 (m = N) and 8 (m = 64, the largest)
    from paper_2503_01276_amd import workloads as W2

    c1 = W.PRESETS["t2"].replace(n_sub=1)
    k, l = W.medium("t2")
    check_forward("t2 s=1", c1, k, l, phi_cells=list(range(0, c1.n_points, 4)), workers=4)
    grad_case("adj-t2 s=1", c1, 21, workers=4)
    c8 = W2.Config(dim=2, n_fine=256, n_macro=8, n_cell=64, n_sub=8, n_cont=1, levels=2)
    k8, l8 = W2.medium_for(c8, seed=23)
    l8 = np.zeros_like(l8)  # one continuum: every element belongs to it
    check_forward("s=8 N=1", c8, k8, l8, phi_cells=[0, 1, 9, 63], workers=8)


def test_invalid_kappa_and_labels_reported_as_einval():
    # kappa must be positive and finite and labels below n_cont; the forward's
    # input check reports the first offending element through mch_diagnostics
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["t2"].replace(max_iter=200)
    k, l = W.medium("t2")
    dev = torch.device("cuda:0")
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    with mch.Plan(cfg) as plan:
        for what, e, val in (("nan", 123, float("nan")), ("zero", 7, 0.0), ("negative", 4000, -1.0),
                             ("inf", 999, float("inf"))):
            bad = k.reshape(-1).copy()
            bad[e] = val
            kd = torch.from_numpy(bad).to(dev)
            say(f"[gpu] edge: kappa {what} at element {e}")
            plan.solve_cells(kd, ld)
            torch.cuda.synchronize()
            with pytest.raises(mch.MchError) as ei:
                plan.diagnostics()
            assert ei.value.code == mch.MCH_EINVAL, (what, ei.value)
            assert f"fine element {e}" in str(ei.value), str(ei.value)
        lb = l.reshape(-1).copy()
        lb[321] = cfg.n_cont
        kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
        say("[gpu] edge: label n_cont at element 321")
        plan.solve_cells(kd, torch.from_numpy(lb).to(dev))
        torch.cuda.synchronize()
        with pytest.raises(mch.MchError) as ei:
            plan.diagnostics()
        assert ei.value.code == mch.MCH_EINVAL and "fine element 321" in str(ei.value)
        # a valid forward on the same plan clears the report
        plan.solve_cells(kd, ld)
        torch.cuda.synchronize()
        it, rs = plan.diagnostics()
        assert it.min() >= 1 and rs.max() <= cfg.rtol


def test_label_buffer_swap_replays_match_eager():
    # two label arrays kept alive and swapped between forwards on one plan:
    # every captured sequence (forward, tensors, backward) is keyed on the
    # labels it reads, so each replay equals the eager run of its own labels
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["t3"]
    k, l1 = W.medium("t3")
    _, l2 = W.medium_for(cfg, 31)
    assert (l1 != l2).any()
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    lds = [torch.from_numpy(x.reshape(-1).copy()).to(dev) for x in (l1, l2)]
    rng = np.random.default_rng(77)
    with mch.Plan(cfg) as plan:
        n = plan.P * plan.M * plan.M
        gA = torch.from_numpy(rng.standard_normal(n)).to(dev)
        ref = []
        for ld in lds:  # eager, default stream
            A = torch.empty(n, dtype=torch.float64, device=dev)
            g = torch.empty_like(kd)
            plan.solve_cells(kd, ld)
            plan.effective_coeffs(kd, A)
            plan.effective_coeffs_backward(kd, gA, g)
            torch.cuda.synchronize()
            ref.append((A, g))
        assert not torch.equal(ref[0][1], ref[1][1])
        st = torch.cuda.Stream()
        A = torch.empty(n, dtype=torch.float64, device=dev)
        g = torch.empty_like(kd)
        with torch.cuda.stream(st):
            for rep in range(6):
                which = rep % 2
                plan.solve_cells(kd, lds[which])
                plan.effective_coeffs(kd, A)
                plan.effective_coeffs_backward(kd, gA, g)
                st.synchronize()
                assert torch.equal(A, ref[which][0]), rep
                assert torch.equal(g, ref[which][1]), rep
                A.zero_()
                g.zero_()
    say("[gpu] edge: 6 replays alternating two label arrays equal their eager runs")

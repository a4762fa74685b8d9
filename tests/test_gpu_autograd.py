"""Adjoint workload at full size through torch.autograd (needs an MI355X).

Loss sum_p ||A_eff(p) - A_target(p)||_F^2 on the hierarchical L=3 preset
(512^2 grid), gradient with respect to per-element log kappa:
  * against the oracle's gradient on a seeded sample of 4096 elements
    (tests/golden/c4_gradient_sample.txt, written by the oracle only);
  * against central finite differences of the GPU forward (delta = 1e-3 in
    log kappa) on 10 channel and 10 matrix elements.
"""
import os

import numpy as np
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(__file__)


def _golden():
    idx, val = [], []
    with open(os.path.join(HERE, "golden", "c4_gradient_sample.txt")) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            a, b = line.split()
            idx.append(int(a))
            val.append(float(b))
    return np.array(idx), np.array(val)


@pytest.fixture(scope="module")
def c4():
    import torch

    from paper_2503_01276_amd import autograd, mch

    import oracle

    cfg = W.PRESETS["c2"]
    k, l = W.medium("c2")
    kt, _ = W.medium("c2", channel_factor=W.target_factor(4))
    dev = torch.device("cuda:0")
    # the target tensors come from the oracle, as for the stored sample
    say("[gpu] c4: oracle forward of the target medium")
    Tref = oracle.stack_A(oracle.forward(cfg, kt, l, workers=16), cfg)
    T = torch.from_numpy(Tref).to(dev)
    plan = mch.Plan(cfg)
    lab = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    logk = torch.from_numpy(np.log(k).reshape(-1)).to(dev).requires_grad_(True)
    A = autograd.effective_tensors(logk, lab, plan)
    loss = ((A - T) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    yield dict(cfg=cfg, k=k, l=l, plan=plan, lab=lab, T=T, logk=logk, grad=logk.grad.detach().clone(),
               loss=float(loss))
    plan.close()


def test_c4_gradient_matches_oracle_sample(c4):
    from gpu_util import assert_grad

    idx, ref = _golden()
    g = c4["grad"].cpu().numpy()[idx]
    assert_grad(f"c4 ({len(idx)} sampled elements)", g, ref, c4["l"].reshape(-1)[idx])


def test_c4_finite_differences(c4):
    import torch

    from paper_2503_01276_amd import autograd

    plan, lab, T = c4["plan"], c4["lab"], c4["T"]
    base = c4["logk"].detach().clone()
    g = c4["grad"].cpu().numpy()
    d = 1e-3
    worst = 0.0
    for e in W.fd_elements(c4["l"], seed=44, n_each=10):
        vals = []
        for sgn in (1.0, -1.0):
            lk = base.clone()
            lk[int(e)] += sgn * d
            with torch.no_grad():
                A = autograd.effective_tensors(lk, lab, plan)
                vals.append(float(((A - T) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * d)
        tol = 1e-4 * abs(fd) + 1e-8 * np.abs(g).max()
        worst = max(worst, abs(fd - g[e]) / max(abs(fd), 1e-300))
        assert abs(fd - g[e]) <= tol, (int(e), fd, g[e])
    say(f"[gpu] c4: worst FD relative difference {worst:.2e}")


def test_autograd_equals_c_abi_and_stale_raises(c4):
    import torch

    from paper_2503_01276_amd import autograd, mch

    plan, lab, T = c4["plan"], c4["lab"], c4["T"]
    # the C ABI directly: forward, tensors and backward on one kappa array
    kappa = torch.exp(c4["logk"].detach()).contiguous()
    plan.solve_cells(kappa, lab)
    A_direct = torch.empty(plan.P * plan.M * plan.M, dtype=torch.float64, device=kappa.device)
    plan.effective_coeffs(kappa, A_direct)
    g_direct = torch.empty_like(kappa)
    plan.effective_coeffs_backward(kappa, (2.0 * (A_direct.view(plan.P, plan.M, plan.M) - T)).contiguous().view(-1),
                                   g_direct)
    # a backward with another kappa array than the forward's is refused
    with pytest.raises(mch.MchError) as ei:
        plan.effective_coeffs_backward(kappa.clone(), torch.zeros_like(A_direct), torch.empty_like(kappa))
    assert ei.value.code == mch.MCH_EINVAL
    torch.cuda.synchronize()
    logk = c4["logk"].detach().clone().requires_grad_(True)
    A = autograd.effective_tensors(logk, lab, plan)
    ((A - T) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(A.detach().reshape(-1), A_direct)
    assert torch.equal(logk.grad, g_direct)
    # a newer forward on the plan invalidates the first graph's backward
    logk2 = c4["logk"].detach().clone().requires_grad_(True)
    A1 = autograd.effective_tensors(logk2, lab, plan)
    with torch.no_grad():
        autograd.effective_tensors(logk2.detach(), lab, plan)
    with pytest.raises(mch.MchError) as ei:
        A1.sum().backward()
    assert ei.value.code == mch.MCH_ESTALE

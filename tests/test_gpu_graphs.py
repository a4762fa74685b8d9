"""hipGraph capture of the launch sequences (needs an MI355X).

Calls on a non-default stream are captured once and replayed while their
arguments are unchanged. Every replay must reproduce the eager (default
stream, uncaptured) result bitwise, with eager torch work and
synchronisations between the replays.
"""
import numpy as np
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import torch

    from paper_2503_01276_amd import mch

    cfg = W.PRESETS["t3"]
    k, l = W.medium("t3")
    kt, _ = W.medium("t3", channel_factor=W.target_factor(4))
    dev = torch.device("cuda:0")
    plan = mch.Plan(cfg)
    kd = torch.from_numpy(k.reshape(-1).copy()).to(dev)
    ld = torch.from_numpy(l.reshape(-1).copy()).to(dev)
    ktd = torch.from_numpy(kt.reshape(-1).copy()).to(dev)
    n = plan.P * plan.M * plan.M
    T = torch.empty(n, dtype=torch.float64, device=dev)
    plan.solve_cells(ktd, ld)
    plan.effective_coeffs(ktd, T)
    A0 = torch.empty_like(T)
    g0 = torch.empty_like(kd)
    # eager reference on the default stream
    plan.solve_cells(kd, ld)
    plan.effective_coeffs(kd, A0)
    gA = 2.0 * (A0 - T)
    plan.effective_coeffs_backward(kd, gA, g0)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    A = torch.empty_like(A0)
    g = torch.empty_like(g0)
    with torch.cuda.stream(st):
        for rep in range(4):
            plan.solve_cells(kd, ld)
            plan.effective_coeffs(kd, A)
            plan.effective_coeffs_backward(kd, gA, g)
            st.synchronize()
            assert torch.equal(A, A0), rep
            assert torch.equal(g, g0), rep
            A.zero_()
            g.zero_()
            _ = (kd * 2.0).sum().item()  # eager work between replays
    say("[gpu] graphs: 4 captured/replayed forward+eff+backward sequences equal the eager run")

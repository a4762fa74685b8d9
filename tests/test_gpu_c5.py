"""Large uneven batch (2048^2, L=4, N=3 with inclusions, contrast 1e8) on an MI355X.

The whole workload (65,536 macropoints, 589,824 solves) runs on the GPU; the
oracle checks two whole level-1 groups (the level-1 cell and its 63
inheritors each) and the local solutions of a few cells; every solve must
converge; the adjoint is checked by central differences of the GPU forward.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import A_rel_err, gpu_forward, phi_rel_err, say, tuned_knobs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    cfg = W.PRESETS["c5"]
    k, l = W.medium("c5")
    lev = oracle.hierarchy.levels(cfg.n_macro, 2, cfg.levels, cfg.eta)
    par = oracle.hierarchy.parents(cfg.n_macro, 2, cfg.levels, cfg.eta)
    l1 = np.flatnonzero(lev == 1)
    groups = [int(l1[0]), int(l1[len(l1) // 2 + 7])]
    pts = sorted(set(groups) | set(int(p) for p in np.flatnonzero(np.isin(par, groups))))
    phi_cells = [groups[0]] + [int(p) for p in pts if lev[p] == 4][:2] + [int(p) for p in pts if lev[p] == 2][:1]
    say(f"[gpu] c5: full forward on the GPU, {len(pts)} sampled cells")
    with tuned_knobs("c5") as table:  # the configuration the bench times
        plan, A, Phi, it, rs, dev = gpu_forward(cfg, k, l, cells=phi_cells)
    say(f"[gpu] c5: tuned knobs {'applied' if table else 'absent'}; band sub-bands per level {plan.band_subbands}")
    return dict(cfg=cfg, k=k, l=l, plan=plan, A=A, Phi=Phi, it=it, rs=rs, pts=pts, phi_cells=phi_cells, dev=dev)


def test_c5_converged(c5):
    it, rs = c5["it"], c5["rs"]
    say(f"[gpu] c5: iterations min/median/max {it.min()}/{int(np.median(it))}/{it.max()}")
    assert it.max() < c5["cfg"].max_iter and rs.max() <= c5["cfg"].rtol


def test_c5_sampled_groups_match_oracle(c5):
    cfg, k, l, pts = c5["cfg"], c5["k"], c5["l"], c5["pts"]
    ref = oracle.forward(cfg, k, l, points=pts, workers=1)
    Aref = np.stack([ref.A[p] for p in pts])
    ea = A_rel_err(c5["A"][pts], Aref)
    ep = max(phi_rel_err(c5["Phi"][p], ref.Phi[p]) for p in c5["phi_cells"])
    say(f"[gpu] c5: A rel err max {ea.max():.2e} over {len(pts)} cells, Phi rel err {ep:.2e}")
    assert ea.max() <= 1e-9 and ep <= 1e-8


def test_c5_adjoint_finite_differences(c5):
    import torch

    plan, (kd, ld) = c5["plan"], c5["dev"]
    A = torch.from_numpy(c5["A"].reshape(-1).copy()).to(kd.device)
    rng = np.random.default_rng(5)
    gA = torch.from_numpy(rng.standard_normal(A.numel())).to(kd.device)  # loss = sum(gA * A_eff)
    plan.solve_cells(kd, ld)
    Ab = torch.empty_like(A)
    plan.effective_coeffs(kd, Ab)
    g = torch.empty_like(kd)
    plan.effective_coeffs_backward(kd, gA, g)
    torch.cuda.synchronize()
    gh = g.cpu().numpy()
    d = 1e-3
    for e in W.fd_elements(c5["l"], seed=55, n_each=3):
        vals = []
        for sgn in (1.0, -1.0):
            kp = kd.clone()
            kp[int(e)] *= float(np.exp(sgn * d))
            plan.solve_cells(kp, ld)
            plan.effective_coeffs(kp, Ab)
            vals.append(float((gA * Ab).sum()))
        fd = (vals[0] - vals[1]) / (2 * d)
        say(f"[gpu] c5: element {int(e)} FD {fd:.6e} adjoint {gh[e]:.6e}")
        assert abs(fd - gh[e]) <= 1e-4 * abs(fd) + 1e-8 * np.abs(gh).max(), (int(e), fd, gh[e])

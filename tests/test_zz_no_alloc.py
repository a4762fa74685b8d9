"""The macroscopic solve without allocation (mch_macro_solve_noalloc), through
the C ABI (needs an MI355X).

Two calls in a row on the library's fixed device buffer, the second with a
smaller system (and another dimension and continuum count), each against
mch_macro_solve on the same plan and inputs: the same kernels in the same
order, so U, the block averages, the iteration count and the residual must be
bitwise equal. A system larger than the buffer is refused.
"""
import numpy as np
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(cfg, seed):
    rng = np.random.default_rng(seed)
    P, M = cfg.n_points, cfg.n_cont * (1 + cfg.dim)
    R = rng.standard_normal((P, M, M))
    A = R @ R.transpose(0, 2, 1) + 0.5 * np.eye(M)
    return A, rng.standard_normal((P, cfg.n_cont))


def _solve_both(plan, A, b):
    import torch

    dev = torch.device("cuda:0")
    N, nm, d = plan.cfg.n_cont, plan.cfg.n_macro, plan.cfg.dim
    Ad = torch.from_numpy(A.reshape(-1).copy()).to(dev)
    bd = torch.from_numpy(b.reshape(-1).copy()).to(dev)
    U0 = torch.empty((nm + 1) ** d * N, dtype=torch.float64, device=dev)
    Ub0 = torch.empty(plan.P * N, dtype=torch.float64, device=dev)
    plan.macro_solve(Ad, bd, U0, Ub0, rtol=1e-12, max_iter=50000)
    it0, rs0 = plan.macro_diagnostics()
    U1 = torch.full_like(U0, float("nan"))
    Ub1 = torch.full_like(Ub0, float("nan"))
    it1 = torch.full((1,), -7, dtype=torch.int32, device=dev)
    rs1 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    plan.macro_solve_noalloc(Ad, bd, U1, Ub1, it1, rs1, rtol=1e-12, max_iter=50000)
    torch.cuda.synchronize()
    return (U0, Ub0, it0, rs0), (U1, Ub1, int(it1.item()), float(rs1.item()))


def test_noalloc_macro_solve_equals_the_allocating_one():
    import torch

    from paper_2503_01276_amd import mch

    cases = [
        # grid-wide CG: 7938 unknowns, more than one workgroup's LDS holds
        ("2d 64^2 blocks N=2", W.Config(dim=2, n_fine=1024, n_macro=64, n_cell=32, n_sub=2, n_cont=2, levels=1), 5),
        # then a smaller system: one-workgroup CG, 3D, three continua
        ("3d 4^3 blocks N=3", W.Config(dim=3, n_fine=32, n_macro=4, n_cell=16, n_sub=2, n_cont=3, levels=1), 6),
    ]
    for name, cfg, seed in cases:
        A, b = _inputs(cfg, seed)
        say(f"[gpu] noalloc: {name}")
        with mch.Plan(cfg) as plan:
            (U0, Ub0, it0, rs0), (U1, Ub1, it1, rs1) = _solve_both(plan, A, b)
        say(f"[gpu] noalloc: {name}: {it1} iterations, residual {rs1:.2e} (allocating: {it0}, {rs0:.2e})")
        assert it1 == it0 and rs1 == rs0, (name, it0, it1, rs0, rs1)
        assert rs1 <= 1e-12
        assert torch.equal(U1, U0) and torch.equal(Ub1, Ub0), name


def test_noalloc_refuses_a_system_beyond_its_buffer():
    import torch

    from paper_2503_01276_amd import mch

    # 128^2 blocks with three continua: 16384 element matrices of 12 x 12
    # alone exceed the 16 MiB buffer
    cfg = W.Config(dim=2, n_fine=256, n_macro=128, n_cell=16, n_sub=2, n_cont=3, levels=1)
    dev = torch.device("cuda:0")
    with mch.Plan(cfg) as plan:
        N, nm = cfg.n_cont, cfg.n_macro
        A = torch.zeros(plan.P * plan.M * plan.M, dtype=torch.float64, device=dev)
        b = torch.zeros(plan.P * N, dtype=torch.float64, device=dev)
        U = torch.empty((nm + 1) ** 2 * N, dtype=torch.float64, device=dev)
        Ub = torch.empty(plan.P * N, dtype=torch.float64, device=dev)
        it = torch.zeros(1, dtype=torch.int32, device=dev)
        rs = torch.zeros(1, dtype=torch.float64, device=dev)
        with pytest.raises(mch.MchError) as ei:
            plan.macro_solve_noalloc(A, b, U, Ub, it, rs)
        assert ei.value.code == mch.MCH_EINVAL and "fixed scratch buffer" in str(ei.value)

"""Parity of the generic 2D solve kernel with the oracle (needs an MI355X).

The generic kernel (Krylov vectors in global memory, any level width,
either cell boundary condition) serves natural Neumann cells, cells wider
than 64 fine elements and cell widths that are not powers of two. Bars as in
test_gpu_parity.py (local solutions 1e-8, effective tensors 1e-9,
constraints 1e-12) and the element-wise gradient bar of gpu_util. Neumann
cells also carry the exact identity of pin P8 on the GPU: the average-type
local solutions sum to 1 at every node (to 1e-10).
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W

from gpu_util import check_forward, gpu_forward, grad_case, say

pytestmark = pytest.mark.gpu

PU_TOL = 1e-10


def _neumann(name):
    return W.PRESETS[name].replace(bc=1)


def _plan_uses_generic(plan):
    # rows per thread 0 on every 2D level: the generic kernel
    return all(r == 0 for r in plan.rows_per_thread)


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_neumann_forward_full(name):
    cfg = _neumann(name)
    k, l = W.medium(name)
    plan, _ = check_forward(f"{name} Neumann", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=1)
    assert _plan_uses_generic(plan)
    plan.close()


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_neumann_partition_of_unity(name):
    # constants are in every level space and have zero energy, and the
    # average constraints of the N average-type problems sum to those of the
    # constant 1, so sum_i phi_i = 1 exactly (pin P8), at every level
    cfg = _neumann(name)
    k, l = W.medium(name)
    cells = list(range(cfg.n_points))
    plan, _, Phi, it, rs, _ = gpu_forward(cfg, k, l, cells=cells)
    worst = max(np.abs(Phi[p][:, : cfg.n_cont].sum(axis=1) - 1.0).max() for p in cells)
    say(f"[gpu] {name} Neumann: max |sum_i phi_i - 1| = {worst:.2e} over {len(cells)} cells")
    plan.close()
    assert worst <= PU_TOL, worst


@pytest.mark.parametrize("name,seed", [("t2", 21), ("t3", 22)])
def test_neumann_gradient(name, seed):
    grad_case(f"{name} Neumann", _neumann(name), seed)


@pytest.mark.parametrize("name", ["c1", "t3"])
def test_generic_kernel_dirichlet(name, monkeypatch):
    # the generic kernel on shapes the register-resident kernel also holds
    monkeypatch.setenv("MCH_GENERIC", "1")
    cfg = W.PRESETS[name]
    k, l = W.medium(name)
    plan, _ = check_forward(f"{name} generic", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=1)
    assert _plan_uses_generic(plan)
    plan.close()


def test_generic_kernel_dirichlet_gradient(monkeypatch):
    monkeypatch.setenv("MCH_GENERIC", "1")
    grad_case("t3 generic", W.PRESETS["t3"], 23)


def _group_sample(cfg, every):
    lev = oracle.hierarchy.levels(cfg.n_macro, 2, cfg.levels, cfg.eta)
    par = oracle.hierarchy.parents(cfg.n_macro, 2, cfg.levels, cfg.eta)
    t = int(np.flatnonzero(lev == 1)[1])
    group = [t] + [int(p) for p in np.flatnonzero(par == t)]
    return sorted(set(group) | set(range(0, cfg.n_points, every)))


@pytest.mark.parametrize("name", ["c6", "c7"])
def test_wide_and_block_aligned_cells(name):
    # c6: 128^2 cells (level widths 128, 64, 32); c7: cells of 3 x 3 coarse
    # blocks (96, 48, 24), constraint regions = the blocks
    cfg = W.PRESETS[name]
    k, l = W.medium(name)
    sample = _group_sample(cfg, 23)
    plan, _ = check_forward(name, cfg, k, l, phi_cells=sample, a_points=sample, workers=8)
    plan.close()


@pytest.mark.parametrize("cfg,seed", [
    (W.Config(dim=2, n_fine=256, n_macro=8, n_cell=128, n_sub=4, n_cont=2, levels=2), 31),
    (W.Config(dim=2, n_fine=192, n_macro=6, n_cell=96, n_sub=3, n_cont=2, levels=2), 32),
])
def test_wide_cells_gradient(cfg, seed):
    grad_case(f"n_cell={cfg.n_cell} n_sub={cfg.n_sub}", cfg, seed, workers=8)


# ---- 3D: the generic 3D kernel (Neumann cells; MCH_GENERIC=1 for Dirichlet) ----

def test_neumann_3d_forward_full():
    cfg = _neumann("t3d")
    k, l = W.medium("t3d")
    plan, _ = check_forward("t3d Neumann", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=4)
    plan.close()


def test_neumann_3d_partition_of_unity():
    cfg = _neumann("t3d")
    k, l = W.medium("t3d")
    cells = list(range(cfg.n_points))
    plan, _, Phi, it, rs, _ = gpu_forward(cfg, k, l, cells=cells)
    worst = max(np.abs(Phi[p][:, : cfg.n_cont].sum(axis=1) - 1.0).max() for p in cells)
    say(f"[gpu] t3d Neumann: max |sum_i phi_i - 1| = {worst:.2e} over {len(cells)} cells")
    plan.close()
    assert worst <= PU_TOL, worst


def test_neumann_3d_gradient():
    grad_case("t3d Neumann", _neumann("t3d"), 24, workers=4)


def test_generic_3d_kernel_dirichlet(monkeypatch):
    monkeypatch.setenv("MCH_GENERIC", "1")
    cfg = W.PRESETS["t3d"]
    k, l = W.medium("t3d")
    plan, _ = check_forward("t3d generic", cfg, k, l, phi_cells=list(range(cfg.n_points)), workers=4)
    plan.close()
    grad_case("t3d generic", cfg, 25, workers=4)

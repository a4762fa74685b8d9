"""Pins for the oracle's Neumann cell conditions (bc = 1; no GPU).

With natural conditions on the cell boundary the constant function lies in
the kernel of the cell stiffness, and the constraint data of the N value
problems sum to the region measures, which the constant reproduces; so the
value solutions form an exact partition of unity, sum_i phi_i = 1 at every
node, on every level of the hierarchy (a child inherits a partition of unity
and its correction problem then has zero data). The value rows of A_eff
therefore sum to zero over the continua. Homogeneous Dirichlet data (bc = 0)
breaks both near the cell boundary, which the control case checks.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W


def _forward(name, **kw):
    cfg = W.PRESETS[name].replace(**kw)
    k, l = W.medium_for(cfg, W.PRESET_SEEDS[name])
    return cfg, oracle.forward(cfg, k, l, workers=4)


def _partition_error(cfg, fwd):
    N = cfg.n_cont
    return max(float(np.abs(fwd.Phi[p][:, :N].sum(axis=1) - 1.0).max()) for p in range(cfg.n_points))


@pytest.mark.parametrize("name,levels", [("t2", 1), ("t2", 2), ("t3d", 2)])
def test_neumann_value_solutions_are_a_partition_of_unity(name, levels):
    cfg, fwd = _forward(name, levels=levels, bc=1)
    assert set(fwd.level.tolist()) == set(range(1, levels + 1))
    err = _partition_error(cfg, fwd)
    assert err <= 1e-10, err


def test_neumann_value_rows_of_A_eff_sum_to_zero():
    cfg, fwd = _forward("t2", levels=2, bc=1)
    A = oracle.stack_A(fwd, cfg)
    N = cfg.n_cont
    colsum = A[:, :N, :].sum(axis=1)  # (sum_i phi_i)^T K Phi_b = 1^T K Phi_b = 0
    assert np.abs(colsum).max() <= 1e-9 * np.abs(A).max(), np.abs(colsum).max()


def test_dirichlet_control_is_not_a_partition_of_unity():
    # the same cells with homogeneous Dirichlet data: sum_i phi_i = 0 on the
    # cell boundary, so the pin above separates the two conditions
    cfg, fwd = _forward("t2", levels=2, bc=0)
    assert _partition_error(cfg, fwd) >= 0.99
    A = oracle.stack_A(fwd, cfg)
    assert np.abs(A[:, :cfg.n_cont, :].sum(axis=1)).max() > 1e-3 * np.abs(A).max()

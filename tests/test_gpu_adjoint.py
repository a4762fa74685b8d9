"""Adjoint gradient of the HIP path versus the oracle's (needs an MI355X).

Loss: sum_p ||A_eff(p) - A_target(p)||_F^2 with the target computed by the
oracle from a medium whose channel value carries a seeded lognormal factor.
Both sides receive the same dLoss/dA_eff, so the comparison isolates the
backward pass. Bar: relative 2-norm over the field <= 1e-8.
"""
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import grad_case

pytestmark = pytest.mark.gpu

_grad_case = grad_case


def test_adjoint_flat_small():
    cfg = W.Config(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=1)
    _grad_case("adj-flat", cfg, 9)


def test_adjoint_hierarchical_L2_small():
    cfg = W.PRESETS["t2"]
    _grad_case("adj-t2", cfg, 9)


def test_adjoint_hierarchical_L3():
    cfg = W.PRESETS["t3"]
    _grad_case("adj-t3", cfg, 8)

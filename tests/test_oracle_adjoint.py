"""Pins for the oracle's adjoint gradient (no GPU): complex step and central differences.

The loss is the one of the adjoint workload, sum_p ||A_eff(p) - A_target(p)||_F^2,
written without conjugation so that it is analytic in kappa and the complex
step (Squire & Trapp 1998) gives the derivative to machine precision.
"""
import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import workloads as W


def _setup(levels):
    cfg = W.Config(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=levels)
    k, l = W.medium_for(cfg, 9)
    kt, _ = W.medium_for(cfg, 9, channel_factor=W.target_factor(4))
    T = oracle.stack_A(oracle.forward(cfg, kt, l, workers=1), cfg)
    return cfg, k, l, T


def _loss(cfg, k, l, T):
    A = oracle.stack_A(oracle.forward(cfg, k, l, workers=1), cfg)
    return np.sum((A - T) ** 2)


@pytest.mark.parametrize("levels", [1, 2])
def test_adjoint_vs_complex_step(levels):
    cfg, k, l, T = _setup(levels)
    fwd = oracle.forward(cfg, k, l, workers=1)
    A = oracle.stack_A(fwd, cfg)
    gA = {p: 2 * (A[p] - T[p]) for p in range(cfg.n_points)}
    g = oracle.backward(cfg, k, l, fwd, gA, workers=1).reshape(-1)
    els = W.fd_elements(l, seed=44, n_each=3)
    delta = 1e-30
    for e in els:
        kc = k.astype(complex).reshape(-1)
        kc[e] *= 1 + 1j * delta
        dL = np.imag(_loss(cfg, kc.reshape(k.shape), l, T)) / delta
        assert abs(dL - g[e]) <= 1e-9 * max(abs(dL), 1e-12 * np.abs(g).max()), (e, dL, g[e])


def test_adjoint_vs_central_difference():
    cfg, k, l, T = _setup(2)
    fwd = oracle.forward(cfg, k, l, workers=1)
    A = oracle.stack_A(fwd, cfg)
    gA = {p: 2 * (A[p] - T[p]) for p in range(cfg.n_points)}
    g = oracle.backward(cfg, k, l, fwd, gA, workers=1).reshape(-1)
    d = 1e-3
    for e in W.fd_elements(l, seed=44, n_each=2):
        kp = k.copy().reshape(-1); kp[e] *= np.exp(d)
        km = k.copy().reshape(-1); km[e] *= np.exp(-d)
        fd = (_loss(cfg, kp.reshape(k.shape), l, T) - _loss(cfg, km.reshape(k.shape), l, T)) / (2 * d)
        assert abs(fd - g[e]) <= 1e-4 * abs(fd) + 1e-10 * np.abs(g).max(), (e, fd, g[e])

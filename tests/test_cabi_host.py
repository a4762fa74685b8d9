"""C-ABI checks that need no GPU: exported symbols, host-side hierarchy, error paths."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2503_01276_amd import mch
from paper_2503_01276_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mch.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mch_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "mch_build_levels" in names and "mch_effective_coeffs_backward" in names
    for n in names:
        assert hasattr(mch.LIB, n), n
    assert sorted(mch.EXPORTS) == names


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5", "t2", "t3"])
def test_host_hierarchy_equals_oracle(name):
    cfg = W.PRESETS[name]
    lev, par = mch.build_hierarchy(cfg)
    olev = oracle.hierarchy.levels(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
    opar = oracle.hierarchy.parents(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta)
    assert np.array_equal(lev, olev) and np.array_equal(par, opar)


@pytest.mark.parametrize("name,levels,eta", [("c2", 3, 2), ("c5", 4, 2), ("t3", 3, 2), ("t2", 2, 2),
                                             ("t3d", 2, 2), ("c1", 3, 2), ("t3", 2, 4)])
def test_host_multilinear_neighbours_equal_oracle(name, levels, eta):
    # interp = 1 lists, bit for bit (same neighbours, order and binary64 weights)
    cfg = W.PRESETS[name].replace(levels=levels, eta=eta, interp=1)
    nbr, w = mch.build_interp(cfg)
    ref = oracle.hierarchy.interp_weights(cfg.n_macro, cfg.dim, cfg.levels, cfg.eta, 1)
    K = 2 ** cfg.dim
    for p in range(cfg.n_points):
        k = len(ref[p])
        assert nbr[p, :k].tolist() == [t for t, _ in ref[p]]
        assert w[p, :k].tolist() == [c for _, c in ref[p]]
        assert np.all(nbr[p, k:K] == -1) and np.all(w[p, k:K] == 0.0)


def test_host_hierarchy_paper_example_counts():
    cfg = W.Config(dim=2, n_fine=64, n_macro=8, n_cell=16, n_sub=2, n_cont=2, levels=3)
    lev, par = mch.build_hierarchy(cfg)
    assert np.bincount(lev)[1:].tolist() == [4, 12, 48]


def _expect(cfg, code):
    with pytest.raises(mch.MchError) as ei:
        mch.Plan(cfg)
    assert ei.value.code == code, str(ei.value)
    assert len(mch.LIB.mch_last_error()) > 0


def test_invalid_configurations():
    good = W.PRESETS["t2"]
    _expect(good.replace(n_cell=15), mch.MCH_EINVAL)          # odd cell
    _expect(good.replace(n_macro=7), mch.MCH_EINVAL)          # n_fine not a multiple
    _expect(good.replace(n_cell=18), mch.MCH_EINVAL)          # not divisible by n_sub*eta^(L-1)
    _expect(good.replace(n_cont=4), mch.MCH_EINVAL)
    _expect(good.replace(levels=0), mch.MCH_EINVAL)
    _expect(good.replace(interp=2), mch.MCH_EINVAL)
    _expect(good.replace(bc=2), mch.MCH_EINVAL)
    _expect(good.replace(bc=1, interp=1), mch.MCH_ENOTIMPL)
    _expect(W.PRESETS["t3d"].replace(bc=1, n_sub=1), mch.MCH_ENOTIMPL)  # 3D Neumann cells need 2 sub-blocks per axis
    _expect(good.replace(rtol=0.0), mch.MCH_EINVAL)
    # over-constrained coarsest level: 2 x 2 sub-blocks x 2 continua = 8 rows, 1 free node
    _expect(W.Config(dim=2, n_fine=64, n_macro=8, n_cell=8, n_sub=2, n_cont=2, levels=3), mch.MCH_ESINGULAR)
    # shapes without a solve kernel (checked before any device work): 2D
    # cells wider than 128 fine elements that the register-resident kernel
    # does not hold either (the generic kernel takes every other width)
    _expect(W.Config(dim=2, n_fine=320, n_macro=20, n_cell=160, n_sub=2, n_cont=2, levels=1), mch.MCH_ENOTIMPL)
    _expect(W.Config(dim=2, n_fine=512, n_macro=16, n_cell=256, n_sub=2, n_cont=2, levels=2), mch.MCH_ENOTIMPL)
    _expect(W.Config(dim=3, n_fine=64, n_macro=8, n_cell=24, n_sub=2, n_cont=2, levels=1), mch.MCH_ENOTIMPL)


def test_classify_solves_rule():
    # the verdict of mch_diagnostics on synthetic per-solve records
    cs = mch.classify_solves
    ok_it, ok_rs = np.array([5, 17, 3]), np.array([1e-13, 5e-13, 0.0])
    assert cs(ok_it, ok_rs, 100, 1e-12) == mch.MCH_OK
    assert cs(np.array([5, -1, 3]), ok_rs, 100, 1e-12) == mch.MCH_ESINGULAR
    # stopped at max_iter above rtol; at max_iter but converged is fine
    assert cs(np.array([5, 100, 3]), np.array([1e-13, 2e-12, 0.0]), 100, 1e-12) == mch.MCH_ENOCONV
    assert cs(np.array([5, 100, 3]), np.array([1e-13, 1e-12, 0.0]), 100, 1e-12) == mch.MCH_OK
    # a non-finite residual is never converged, whatever the iteration count
    assert cs(ok_it, np.array([1e-13, np.nan, 0.0]), 100, 1e-12) == mch.MCH_ENOCONV
    assert cs(ok_it, np.array([np.inf, 0.0, 0.0]), 100, 1e-12) == mch.MCH_ENOCONV
    # a singular record outranks a non-converged one
    assert cs(np.array([100, -1]), np.array([np.nan, 0.0]), 100, 1e-12) == mch.MCH_ESINGULAR
    assert cs(np.zeros(0), np.zeros(0), 100, 1e-12) == mch.MCH_OK
    assert mch.LIB.mch_classify_solves(None, None, 3, 100, 1e-12) == mch.MCH_EINVAL


def test_null_handles():
    vp = ctypes.c_void_p
    assert mch.LIB.mch_solve_cells(None, None, None, None) == mch.MCH_EINVAL
    assert mch.LIB.mch_effective_coeffs(None, None, None, None) == mch.MCH_EINVAL
    assert mch.LIB.mch_effective_coeffs_backward(None, None, None, None, None) == mch.MCH_EINVAL
    assert mch.LIB.mch_profile(None, 1) == mch.MCH_EINVAL
    it = np.zeros(1, np.int32)
    rs = np.zeros(1)
    assert mch.LIB.mch_diagnostics(None, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   rs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == mch.MCH_EINVAL
    mch.LIB.mch_destroy(vp())  # NULL is allowed
    assert mch.LIB.mch_build_levels(None, None) == mch.MCH_EINVAL


def test_config_struct_layout():
    # the ctypes mirror must match the C struct layout of include/mch.h
    c = mch.CConfig
    assert c.dim.offset == 0 and c.n_fine.offset == 4 and c.h.offset == 16
    assert c.n_macro.offset == 24 and c.n_cell.offset == 36 and c.rtol.offset == 64
    assert ctypes.sizeof(c) == 80


def test_plan_owned_by_another_process_is_not_destroyed(monkeypatch):
    # A forked worker (the oracle's process pool) inherits Plan objects; when
    # it collects one it must drop the handle without calling into the device.
    calls = []

    class FakeLib:
        def mch_destroy(self, h):
            calls.append(h)

    monkeypatch.setattr(mch, "LIB", FakeLib())
    p = mch.Plan.__new__(mch.Plan)
    p._h, p._pid = ctypes.c_void_p(1234), os.getpid() + 1
    p.close()
    assert calls == [] and p._h is None
    q = mch.Plan.__new__(mch.Plan)
    q._h, q._pid = ctypes.c_void_p(5678), os.getpid()
    q.close()
    assert len(calls) == 1 and q._h is None

"""ctypes binding of libmch.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module converts
Python/torch arguments into the C ABI declared in include/mch.h and raises
``MchError`` on any non-zero status. If the library has not been built the
import of this module fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MCH_LIB", os.path.join(HERE, "libmch.so"))

MCH_OK, MCH_EINVAL, MCH_ESINGULAR, MCH_ENOCONV, MCH_EHIP, MCH_ESTALE, MCH_ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
CODE_NAMES = {MCH_EINVAL: "MCH_EINVAL", MCH_ESINGULAR: "MCH_ESINGULAR", MCH_ENOCONV: "MCH_ENOCONV",
              MCH_EHIP: "MCH_EHIP", MCH_ESTALE: "MCH_ESTALE", MCH_ENOTIMPL: "MCH_ENOTIMPL"}

EXPORTS = ["mch_build_levels", "mch_build_hierarchy", "mch_build_interp", "mch_plan_info", "mch_hierarchy", "mch_solve_cells", "mch_effective_coeffs",
           "mch_effective_coeffs_backward", "mch_local_solutions", "mch_diagnostics", "mch_adjoint_diagnostics", "mch_profile",
           "mch_profile_read", "mch_classify_solves", "mch_macro_load", "mch_macro_solve", "mch_macro_solve_noalloc", "mch_macro_diagnostics", "mch_destroy",
           "mch_last_error"]


class MchError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class CConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n_fine", ctypes.c_int32 * 3),
        ("h", ctypes.c_double),
        ("n_macro", ctypes.c_int32 * 3),
        ("n_cell", ctypes.c_int32),
        ("n_sub", ctypes.c_int32),
        ("n_cont", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("eta", ctypes.c_int32),
        ("interp", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
    ]


def _load():
    # torch bundles its own HIP runtime with the same soname (libamdhip64.so.7)
    # as ROCm's; importing torch first makes the library bind to that one
    # runtime, so torch tensors and the library's kernels share one device
    # context.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmch.so not built at {LIB_PATH}; run `python -m paper_2503_01276_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32p, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), \
        ctypes.POINTER(ctypes.c_double)
    lib.mch_build_levels.argtypes = [ctypes.POINTER(CConfig), ctypes.POINTER(vp)]
    lib.mch_plan_info.argtypes = [vp, i64p]
    lib.mch_build_hierarchy.argtypes = [ctypes.POINTER(CConfig), i32p, i32p]
    lib.mch_build_interp.argtypes = [ctypes.POINTER(CConfig), i32p, dp]
    lib.mch_hierarchy.argtypes = [vp, i32p, i32p]
    lib.mch_solve_cells.argtypes = [vp, vp, vp, vp]
    lib.mch_effective_coeffs.argtypes = [vp, vp, vp, vp]
    lib.mch_effective_coeffs_backward.argtypes = [vp, vp, vp, vp, vp]
    lib.mch_local_solutions.argtypes = [vp, i64p, ctypes.c_int64, vp, vp]
    lib.mch_diagnostics.argtypes = [vp, i32p, dp]
    lib.mch_adjoint_diagnostics.argtypes = [vp, i32p, dp]
    lib.mch_profile.argtypes = [vp, ctypes.c_int32]
    lib.mch_profile_read.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32, dp]
    lib.mch_classify_solves.argtypes = [i32p, dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double]
    lib.mch_macro_load.argtypes = [vp, vp, vp, vp]
    lib.mch_macro_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp]
    lib.mch_macro_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    lib.mch_macro_diagnostics.argtypes = [vp, i32p, dp]
    lib.mch_destroy.argtypes = [vp]
    lib.mch_destroy.restype = None
    lib.mch_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("mch_destroy", "mch_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


LIB = _load()

# Plans still open when the interpreter exits are released by an exit hook,
# which runs while torch's runtime is still up (hooks run in reverse order of
# registration, and torch is imported before this one is registered).
_LIVE = weakref.WeakSet()


def _close_all():
    for plan in list(_LIVE):
        try:
            plan.close()
        except Exception:
            pass


atexit.register(_close_all)


def check(rc: int):
    if rc != MCH_OK:
        raise MchError(rc, LIB.mch_last_error().decode())


def to_c_config(cfg) -> CConfig:
    c = CConfig()
    c.dim = cfg.dim
    for a in range(3):
        c.n_fine[a] = cfg.n_fine if a < cfg.dim else 1
        c.n_macro[a] = cfg.n_macro if a < cfg.dim else 1
    c.h = 1.0 / cfg.n_fine
    c.n_cell, c.n_sub, c.n_cont = cfg.n_cell, cfg.n_sub, cfg.n_cont
    c.levels, c.eta, c.interp, c.bc = cfg.levels, cfg.eta, cfg.interp, cfg.bc
    c.rtol, c.max_iter = cfg.rtol, cfg.max_iter
    return c


def build_hierarchy(cfg):
    """Host-only hierarchy (level, parent) of a configuration; needs no device."""
    c = to_c_config(cfg)
    P = cfg.n_macro ** cfg.dim
    lev = np.zeros(P, np.int32)
    par = np.zeros(P, np.int32)
    check(LIB.mch_build_hierarchy(ctypes.byref(c), lev.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  par.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return lev, par


def build_interp(cfg):
    """Host-only multilinear neighbours and weights, each [P][2^dim]; needs no device."""
    c = to_c_config(cfg)
    shape = (cfg.n_macro ** cfg.dim, 2 ** cfg.dim)
    nbr = np.zeros(shape, np.int32)
    w = np.zeros(shape, np.float64)
    check(LIB.mch_build_interp(ctypes.byref(c), nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return nbr, w


def classify_solves(iters, resid, max_iter: int, rtol: float) -> int:
    """Status code the library's diagnostics give to per-solve records (host only)."""
    it = np.ascontiguousarray(iters, dtype=np.int32).reshape(-1)
    rs = np.ascontiguousarray(resid, dtype=np.float64).reshape(-1)
    return LIB.mch_classify_solves(it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   rs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), it.size, int(max_iter),
                                   float(rtol))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """Owns one ``mch_plan``; methods mirror the C entry points one to one."""

    def __init__(self, cfg):
        self.cfg = cfg
        self._c = to_c_config(cfg)
        # the process whose device context owns the plan; a forked child (a
        # CPU worker pool) inherits the object but must not touch the device
        self._pid = os.getpid()
        h = ctypes.c_void_p()
        check(LIB.mch_build_levels(ctypes.byref(self._c), ctypes.byref(h)))
        self._h = h
        info = (ctypes.c_int64 * 28)()
        check(LIB.mch_plan_info(self._h, info))
        self.P, self.M, self.m, self.levels = int(info[0]), int(info[1]), int(info[2]), int(info[3])
        self.level_counts = [int(info[4 + k]) for k in range(self.levels)]
        # node rows per thread of each level's 2D solve kernel (0 in 3D and
        # on levels solved by the generic 2D kernel)
        self.rows_per_thread = [int(info[4 + self.levels + k]) for k in range(self.levels)]
        # whether each level's 2D solve uses the band coarse correction, and
        # with how many sub-bands per thread's node rows (0: none)
        self.band_subbands = [int(info[4 + 2 * self.levels + k]) for k in range(self.levels)]
        self.band_precond = [b > 0 for b in self.band_subbands]
        self.generation = 0  # bumped by every forward solve
        _LIVE.add(self)

    def close(self):
        """Release the plan (mch_destroy). Call it before the interpreter exits."""
        if getattr(self, "_h", None):
            if getattr(self, "_pid", None) == os.getpid():
                LIB.mch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # During interpreter shutdown the HIP runtime and torch's streams may
        # already be torn down: make no HIP call then (the process exit
        # releases the device memory). The check is bound at definition time,
        # since module globals such as sys may already be cleared by then.
        if _finalizing():
            self._h = None
            return
        try:
            self.close()
        except Exception:
            pass

    def hierarchy(self):
        lev = np.zeros(self.P, np.int32)
        par = np.zeros(self.P, np.int32)
        check(LIB.mch_hierarchy(self._h, lev.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                par.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return lev, par

    def solve_cells(self, kappa, label, stream=None):
        _require(kappa, "float64", self.cfg.n_fine ** self.cfg.dim)
        _require(label, "uint8", self.cfg.n_fine ** self.cfg.dim)
        check(LIB.mch_solve_cells(self._h, _ptr(kappa), _ptr(label), _stream(stream)))
        self.generation += 1

    def effective_coeffs(self, kappa, A_eff, stream=None):
        _require(kappa, "float64", self.cfg.n_fine ** self.cfg.dim)
        _require(A_eff, "float64", self.P * self.M * self.M)
        check(LIB.mch_effective_coeffs(self._h, _ptr(kappa), _ptr(A_eff), _stream(stream)))

    def effective_coeffs_backward(self, kappa, gA, glogk, stream=None):
        _require(kappa, "float64", self.cfg.n_fine ** self.cfg.dim)
        _require(gA, "float64", self.P * self.M * self.M)
        _require(glogk, "float64", self.cfg.n_fine ** self.cfg.dim)
        check(LIB.mch_effective_coeffs_backward(self._h, _ptr(kappa), _ptr(gA), _ptr(glogk), _stream(stream)))

    def local_solutions(self, cells, out, stream=None):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        nn = (self.cfg.n_cell + 1) ** self.cfg.dim
        _require(out, "float64", len(cells) * self.M * nn)
        check(LIB.mch_local_solutions(self._h, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      len(cells), _ptr(out), _stream(stream)))

    def macro_load(self, f, b, stream=None):
        """b[p][j] = int_{K_p} f phi_j from the last forward."""
        _require(f, "float64", self.cfg.n_fine ** self.cfg.dim)
        _require(b, "float64", self.P * self.cfg.n_cont)
        check(LIB.mch_macro_load(self._h, _ptr(f), _ptr(b), _stream(stream)))

    def macro_solve(self, A_eff, b, U, U_block, rtol=1e-12, max_iter=20000, stream=None):
        """The macroscopic system from A_eff and b: nodal U and block averages."""
        N, nm = self.cfg.n_cont, self.cfg.n_macro
        _require(A_eff, "float64", self.P * self.M * self.M)
        _require(b, "float64", self.P * N)
        _require(U, "float64", (nm + 1) ** self.cfg.dim * N)
        _require(U_block, "float64", self.P * N)
        check(LIB.mch_macro_solve(self._h, _ptr(A_eff), _ptr(b), _ptr(U), _ptr(U_block), float(rtol), int(max_iter),
                                  _stream(stream)))

    def macro_solve_noalloc(self, A_eff, b, U, U_block, iters, resid, rtol=1e-12, max_iter=20000, stream=None):
        """macro_solve on the library's fixed device buffer (no allocation);
        iteration count and residual into the device tensors iters (int32 [1])
        and resid (float64 [1])."""
        N, nm = self.cfg.n_cont, self.cfg.n_macro
        _require(A_eff, "float64", self.P * self.M * self.M)
        _require(b, "float64", self.P * N)
        _require(U, "float64", (nm + 1) ** self.cfg.dim * N)
        _require(U_block, "float64", self.P * N)
        _require(iters, "int32", 1)
        _require(resid, "float64", 1)
        check(LIB.mch_macro_solve_noalloc(self._h, _ptr(A_eff), _ptr(b), _ptr(U), _ptr(U_block), float(rtol),
                                          int(max_iter), _ptr(iters), _ptr(resid), _stream(stream)))

    def macro_diagnostics(self):
        it = np.zeros(1, np.int32)
        rs = np.zeros(1, np.float64)
        check(LIB.mch_macro_diagnostics(self._h, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        rs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return int(it[0]), float(rs[0])

    def profile(self, on: bool):
        """Turn per-launch event timing on or off (clears the records)."""
        check(LIB.mch_profile(self._h, 1 if on else 0))

    def profile_records(self):
        """[(kernel name, milliseconds)] for every profiled launch since the last profile() call."""
        n = LIB.mch_profile_read(self._h, -1, None, 0, None)
        if n < 0:
            check(n)
        out = []
        buf = ctypes.create_string_buffer(64)
        ms = ctypes.c_double()
        for i in range(n):
            rc = LIB.mch_profile_read(self._h, i, buf, 64, ctypes.byref(ms))
            if rc < 0:
                check(rc)
            out.append((buf.value.decode(), ms.value))
        return out

    def diagnostics(self, allow_noconv: bool = False, adjoint: bool = False):
        it = np.zeros(self.P * self.M, np.int32)
        rs = np.zeros(self.P * self.M, np.float64)
        fn = LIB.mch_adjoint_diagnostics if adjoint else LIB.mch_diagnostics
        rc = fn(self._h, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                rs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if not (allow_noconv and rc == MCH_ENOCONV):
            check(rc)
        return it.reshape(self.P, self.M), rs.reshape(self.P, self.M)


def _require(t, dtype: str, numel: int):
    if not (t.is_cuda and str(t.dtype).endswith(dtype) and t.is_contiguous() and t.numel() == numel):
        raise MchError(MCH_EINVAL, f"expected a contiguous {dtype} device tensor of {numel} elements, got "
                                   f"{t.dtype} {tuple(t.shape)} on {t.device}")

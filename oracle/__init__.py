"""fp64 CPU oracle for Weighted Regularized Graph Normalization (WRGN).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path (``paper_2605_05330_amd``) never
imports it.  The compiled part is ``gn_oracle.c`` (plain C, gcc); this module
holds its ctypes binding.  The message-passing warm-start reference lives in
``oracle/mpnn.py``, the census of GN atoms (Appendix A) in ``oracle/atoms.py``, the fractional
clique-LP warm start (Section 6) in ``oracle/lp.py``.

Parity status of every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gn_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "_build", "liboracle_omp.so")   # all-core build (CPU baseline only)

OK, NOT_CONVERGED = 0, 1
E_ARG, E_CSR, E_SELF_LOOP, E_ASYMMETRIC, E_WEIGHT, E_NOT_NORMALIZABLE = -1, -2, -3, -4, -5, -6


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with gcc (no optimisation flags beyond -O2; fp contraction off
    so each operation rounds as written).  omp=True builds the all-core variant
    (-fopenmp) that the benchmark times as its second CPU baseline."""
    lib = _LIB_OMP if omp else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(lib), exist_ok=True)
        tmp = lib + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               *(["-fopenmp"] if omp else []), "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    if force and not omp:
        build(force=True, omp=True)
    return lib


_lib = None
_lib_omp = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


class _Schedule(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_double), ("gamma1", ctypes.c_double),
                ("ramp_steps", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("tau", ctypes.c_double), ("check_every", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("binarised", ctypes.c_int32),
                ("fallback_count", ctypes.c_int64),
                ("relaxed_objective", ctypes.c_double), ("set_objective", ctypes.c_double),
                ("set_size", ctypes.c_int64), ("conflicts", ctypes.c_int64),
                ("uncovered", ctypes.c_int64), ("stab", ctypes.c_double),
                ("residual", ctypes.c_double), ("growing", ctypes.c_int64)]


def _load(omp: bool = False):
    global _lib, _lib_omp
    if omp:
        if _lib_omp is None:
            _lib_omp = _bind(ctypes.CDLL(build(omp=True)))
        return _lib_omp
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _bind(lib):
    if True:
        lib.orc_validate.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _f64p]
        lib.orc_validate.restype = ctypes.c_int
        lib.orc_gamma.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int64]
        lib.orc_gamma.restype = ctypes.c_double
        lib.orc_step.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_double, _f64p, _f64p]
        lib.orc_step.restype = ctypes.c_int64
        lib.orc_is_normalizable.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p]
        lib.orc_is_normalizable.restype = ctypes.c_int
        lib.orc_binarisation.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_double, _f64p,
                                         _f64p, _i64p, _i64p]
        lib.orc_binarisation.restype = None
        lib.orc_objective.argtypes = [ctypes.c_int32, _f64p, _f64p]
        lib.orc_objective.restype = ctypes.c_double
        lib.orc_check.argtypes = [ctypes.c_int32, _i32p, _i32p, _u8p, _i64p, _i64p]
        lib.orc_check.restype = None
        lib.orc_stab.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_double, _u8p]
        lib.orc_stab.restype = ctypes.c_double
        lib.orc_energy.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_double, _f64p]
        lib.orc_energy.restype = ctypes.c_double
        lib.orc_solve.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.POINTER(_Schedule),
                                  _f64p, _u8p, ctypes.POINTER(_Result)]
        lib.orc_solve.restype = ctypes.c_int
        lib.orc_unrolled_forward.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p,
                                             ctypes.c_int32, _f64p, _f64p]
        lib.orc_unrolled_forward.restype = ctypes.c_int64
        lib.orc_unrolled_vjp.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, ctypes.c_int32,
                                         _f64p, _f64p, _f64p, _f64p]
        lib.orc_unrolled_vjp.restype = None
        lib.orc_set_x_floor.argtypes = [ctypes.c_double]
        lib.orc_set_x_floor.restype = None
        lib.orc_get_x_floor.argtypes = []
        lib.orc_get_x_floor.restype = ctypes.c_double
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
    return lib


def threads(omp: bool = True) -> int:
    """Threads the row loops of the all-core build use (OMP_NUM_THREADS or all cores)."""
    return _load(omp).orc_threads()


def _p(a, t):
    return a.ctypes.data_as(t)


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if a.size else np.zeros(1, np.float64)


def validate(n, row_ptr, col_idx, w) -> int:
    rp, ci = _csr(row_ptr, col_idx)
    return _load().orc_validate(n, int(np.asarray(row_ptr)[-1]) if n >= 0 else 0,
                                _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p))


def x_floor() -> float:
    """The level at which a positive coordinate is held instead of underflowing
    (fp64's smallest normal number, 2^-1022, unless a test moved it)."""
    return _load().orc_get_x_floor()


def set_x_floor(f: float) -> None:
    """Move the support floor (tests only: they show that results do not depend on
    it); a non-positive value restores 2^-1022."""
    _load().orc_set_x_floor(float(f))


def gamma(gamma0, gamma1, ramp, k) -> float:
    return _load().orc_gamma(gamma0, gamma1, ramp, k)


def gammas(gamma0, gamma1, ramp, count) -> np.ndarray:
    return np.array([gamma(gamma0, gamma1, ramp, k) for k in range(count)], dtype=np.float64)


def step(n, row_ptr, col_idx, w, gamma_k, x) -> tuple[np.ndarray, int]:
    """One WRGN step; returns (x', fallback_count)."""
    rp, ci = _csr(row_ptr, col_idx)
    v = np.sqrt(np.asarray(w, dtype=np.float64))
    xin = _f64(x)
    out = np.zeros(max(n, 1), np.float64)
    fb = _load().orc_step(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(v), _f64p), float(gamma_k),
                          _p(xin, _f64p), _p(out, _f64p))
    return out[:n], int(fb)


def is_normalizable(n, row_ptr, col_idx, x) -> int:
    rp, ci = _csr(row_ptr, col_idx)
    return _load().orc_is_normalizable(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(x), _f64p))


def binarisation(n, row_ptr, col_idx, w, gamma_k, x) -> tuple[float, int, int]:
    """(residual, uncovered, growing) of state x under gamma_k."""
    rp, ci = _csr(row_ptr, col_idx)
    r = ctypes.c_double()
    u = ctypes.c_int64()
    g = ctypes.c_int64()
    _load().orc_binarisation(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), float(gamma_k),
                             _p(_f64(x), _f64p), ctypes.byref(r), ctypes.byref(u), ctypes.byref(g))
    return r.value, u.value, g.value


def objective(w, x) -> float:
    w = _f64(w)
    return _load().orc_objective(len(np.atleast_1d(x)), _p(w, _f64p), _p(_f64(x), _f64p))


def check(n, row_ptr, col_idx, sel) -> tuple[int, int]:
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(sel, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    c = ctypes.c_int64()
    u = ctypes.c_int64()
    _load().orc_check(n, _p(rp, _i32p), _p(ci, _i32p), _p(s, _u8p), ctypes.byref(c), ctypes.byref(u))
    return c.value, u.value


def stab(n, row_ptr, col_idx, w, gamma_k, sel) -> float:
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(sel, dtype=np.uint8)
    return _load().orc_stab(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), float(gamma_k),
                            _p(s, _u8p))


def energy(n, row_ptr, col_idx, w, gamma_k, y) -> float:
    rp, ci = _csr(row_ptr, col_idx)
    return _load().orc_energy(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), float(gamma_k),
                              _p(_f64(y), _f64p))


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    sel: np.ndarray
    steps: int
    binarised: bool
    fallback_count: int
    relaxed_objective: float
    set_objective: float
    set_size: int
    conflicts: int
    uncovered: int
    stab: float
    residual: float
    growing: int


def solve(n, row_ptr, col_idx, w, x0, gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=2000,
          tau=1e-4, check_every=1, omp=False) -> SolveResult:
    rp, ci = _csr(row_ptr, col_idx)
    x = np.array(np.asarray(x0, dtype=np.float64), copy=True)
    xb = x if x.size else np.zeros(1, np.float64)
    sel = np.zeros(max(n, 1), np.uint8)
    sch = _Schedule(gamma0, gamma1, ramp_steps, max_steps, tau, check_every)
    res = _Result()
    st = _load(omp).orc_solve(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), ctypes.byref(sch),
                           _p(xb, _f64p), _p(sel, _u8p), ctypes.byref(res))
    return SolveResult(st, xb[:n].copy(), sel[:n].astype(bool), res.steps, bool(res.binarised),
                       res.fallback_count, res.relaxed_objective, res.set_objective, res.set_size,
                       res.conflicts, res.uncovered, res.stab, res.residual, res.growing)


def unrolled_forward(n, row_ptr, col_idx, w, gammas_, x0) -> np.ndarray:
    """Returns all iterates, shape (T+1, n)."""
    rp, ci = _csr(row_ptr, col_idx)
    g = _f64(gammas_)
    T = len(np.atleast_1d(gammas_))
    xs = np.zeros((T + 1) * max(n, 1), np.float64)
    _load().orc_unrolled_forward(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), _p(g, _f64p),
                                 T, _p(_f64(x0), _f64p), _p(xs, _f64p))
    return xs[:(T + 1) * n].reshape(T + 1, n)


def unrolled_vjp(n, row_ptr, col_idx, w, gammas_, x0, gxT) -> tuple[np.ndarray, np.ndarray]:
    """Gradient of <gxT, x^T> through T steps: returns (dL/dw, dL/dx0)."""
    rp, ci = _csr(row_ptr, col_idx)
    g = _f64(gammas_)
    T = len(np.atleast_1d(gammas_))
    gw = np.zeros(max(n, 1), np.float64)
    gx0 = np.zeros(max(n, 1), np.float64)
    _load().orc_unrolled_vjp(n, _p(rp, _i32p), _p(ci, _i32p), _p(_f64(w), _f64p), _p(g, _f64p), T,
                             _p(_f64(x0), _f64p), _p(_f64(gxT), _f64p), _p(gw, _f64p), _p(gx0, _f64p))
    return gw[:n], gx0[:n]


def solve_batch(ns, row_ptr_cat, col_idx_cat, w_cat, x0_cat, **sched) -> list[SolveResult]:
    """Many independent graphs (local CSR arrays back to back): one solve per graph.
    By connected-component independence (Section 2, property iii) this is the
    batched reference."""
    out = []
    rpo = 0
    co = 0
    vo = 0
    for n in ns:
        n = int(n)
        rp = np.asarray(row_ptr_cat[rpo:rpo + n + 1], dtype=np.int32)
        nnz = int(rp[-1])
        ci = col_idx_cat[co:co + nnz]
        out.append(solve(n, rp, ci, w_cat[vo:vo + n], x0_cat[vo:vo + n], **sched))
        rpo += n + 1
        co += nnz
        vo += n
    return out


def random_start(u) -> np.ndarray:
    """Random starting point of the paper's module (code appendix), one start:
    e = -log(u) for u in (0, 1], normalised by its maximum and clamped to
    [1e-3, 1]; all ones when every e is zero.  fp64."""
    e = -np.log(np.asarray(u, dtype=np.float64))
    e = np.maximum(e, 0.0)
    m = e.max() if e.size else 0.0
    if m <= 0.0:
        return np.ones_like(e)
    return np.clip(e / m, 1e-3, 1.0)


def multi_solve(n, row_ptr, col_idx, w, x0s, **sched) -> list[SolveResult]:
    """Independent solves from several starting points (rows of x0s), one by one."""
    return [solve(n, row_ptr, col_idx, w, x0, **sched) for x0 in np.atleast_2d(np.asarray(x0s, dtype=np.float64))]

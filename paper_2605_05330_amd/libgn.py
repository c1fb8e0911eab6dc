"""Thin ctypes binding of libgn (include/libgn.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if
``libgn.so`` is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from collections.abc import Sequence
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libgn.so")

GN_OK, GN_NOT_CONVERGED = 0, 1
GN_E_ARG, GN_E_CSR, GN_E_SELF_LOOP, GN_E_ASYMMETRIC, GN_E_WEIGHT = -1, -2, -3, -4, -5
GN_E_NOT_NORMALIZABLE, GN_E_NUMERIC, GN_E_HIP, GN_E_NOMEM, GN_E_SIZE = -6, -7, -8, -9, -10
GN_INPUT_HOST, GN_INPUT_DEVICE, GN_NO_VALIDATE = 0, 1, 2
GN_NUM_BINS = 7


class GNError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {gn_status_str(status)} ({status})")


class gn_schedule(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_float), ("gamma1", ctypes.c_float), ("ramp_steps", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("tau", ctypes.c_float), ("check_every", ctypes.c_int32)]


class gn_result(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("binarised", ctypes.c_int32), ("fallback_count", ctypes.c_int64),
                ("relaxed_objective", ctypes.c_double), ("set_objective", ctypes.c_double),
                ("set_size", ctypes.c_int64), ("conflicts", ctypes.c_int64), ("uncovered", ctypes.c_int64),
                ("stab", ctypes.c_float)]


class gn_atom_counts(ctypes.Structure):
    _fields_ = [("connected", ctypes.c_int64), ("irregular_discrete", ctypes.c_int64),
                ("irregular_continuous", ctypes.c_int64), ("regular_discrete", ctypes.c_int64),
                ("regular_continuous", ctypes.c_int64), ("atomic", ctypes.c_int64),
                ("labelled_evaluated", ctypes.c_int64)]


class gn_lp_result(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("converged", ctypes.c_int32), ("temperature", ctypes.c_float),
                ("pad", ctypes.c_float), ("dual", ctypes.c_double), ("primal", ctypes.c_double),
                ("gap", ctypes.c_double)]


class gn_tuning(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lds_vertices", ctypes.c_int32), ("light_max_deg", ctypes.c_int32),
                ("mid_max_deg", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libgn.so (raises if it is not built).

    torch is imported first: its wheel carries its own HIP runtime under the
    same soname as the system one that libgn.so is linked against.  Loaded
    first, libgn.so would pull in the system runtime, and torch would then load
    a second one into the process; two HIP runtimes in one process make
    allocations fail or launches do nothing.  With torch first, the library
    binds to the runtime already loaded."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgn.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "gn_graph_create": ([ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_uint32, _vp,
                                 ctypes.POINTER(_vp)], ctypes.c_int),
            "gn_graph_destroy": ([_vp], None),
            "gn_graph_info": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "gn_step": ([_vp, ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
            "gn_step_static": ([_vp, ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
            "gn_step_static_max_n": ([], ctypes.c_int32),
            "gn_solve": ([_vp, ctypes.POINTER(gn_schedule), _vp, _vp, ctypes.POINTER(gn_result), _vp],
                         ctypes.c_int),
            "gn_objective": ([_vp, _vp, ctypes.POINTER(ctypes.c_double), _vp], ctypes.c_int),
            "gn_check_independent": ([_vp, _vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      _vp], ctypes.c_int),
            "gn_status_str": ([ctypes.c_int], ctypes.c_char_p),
            "gn_set_chunk_len": ([ctypes.c_int32], ctypes.c_int),
            "gn_set_small_graph_limit": ([ctypes.c_int32], ctypes.c_int),
            "gn_set_pruning": ([ctypes.c_int32], ctypes.c_int),
            "gn_set_prune_interval": ([ctypes.c_int32], ctypes.c_int),
            "gn_set_multi_handoff": ([ctypes.c_int32], ctypes.c_int),
            "gn_atom_census": ([ctypes.c_int32, ctypes.POINTER(gn_atom_counts), _vp], ctypes.c_int),
            "gn_batch_create": ([ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)],
                                ctypes.c_int),
            "gn_batch_destroy": ([_vp], None),
            "gn_batch_solve": ([_vp, ctypes.POINTER(gn_schedule), ctypes.POINTER(gn_tuning), _vp, _vp,
                                ctypes.POINTER(gn_result), _vp], ctypes.c_int),
            "gn_batch_autotune": ([_vp, ctypes.POINTER(gn_schedule), ctypes.POINTER(gn_tuning), _vp], ctypes.c_int),
            "gn_batch_tuning_cache_size": ([], ctypes.c_int32),
            "gn_batch_tuning_cache_clear": ([], None),
            "gn_batch_graph": ([_vp], _vp),
            "gn_mpnn_cache_bytes": ([ctypes.c_int32], ctypes.c_int64),
            "gn_mpnn_forward": ([_vp, _vp, ctypes.c_float, _vp, _vp, _vp, _vp], ctypes.c_int),
            "gn_mpnn_backward": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
            "gn_adam_step": ([_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_int32, _vp], ctypes.c_int),
            "gn_multi_solve": ([_vp, ctypes.POINTER(gn_schedule), ctypes.c_int32, _vp, _vp, _vp,
                                ctypes.POINTER(ctypes.c_int32), _vp], ctypes.c_int),
            "gn_random_starts": ([_vp, ctypes.c_int32, _vp, _vp, _vp], ctypes.c_int),
            "gn_rook_create": ([ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)],
                               ctypes.c_int),
            "gn_rook_destroy": ([_vp], None),
            "gn_lp_create": ([ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
            "gn_lp_destroy": ([_vp], None),
            "gn_hyper_create": ([ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)],
                                ctypes.c_int),
            "gn_hyper_destroy": ([_vp], None),
            "gn_hyper_multi_solve": ([_vp, ctypes.POINTER(gn_schedule), ctypes.c_int32, _vp, _vp, _vp,
                                      ctypes.POINTER(ctypes.c_int32), _vp], ctypes.c_int),
            "gn_hyper_step": ([_vp, ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
            "gn_hyper_solve": ([_vp, ctypes.POINTER(gn_schedule), _vp, _vp, ctypes.POINTER(gn_result), _vp],
                               ctypes.c_int),
            "gn_lp_info": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "gn_lp_set_fused": ([_vp, ctypes.c_int32], ctypes.c_int32),
            "gn_lp_solve": ([_vp, ctypes.c_int32, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                             ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp,
                             ctypes.POINTER(gn_lp_result), _vp],
                            ctypes.c_int),
            "gn_rook_step": ([_vp, ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
            "gn_rook_solve": ([_vp, ctypes.POINTER(gn_schedule), _vp, _vp, ctypes.POINTER(gn_result), _vp],
                              ctypes.c_int),
            "gn_unrolled_ckpt_floats": ([_vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int64),
            "gn_batch_unrolled_store_floats": ([_vp, ctypes.c_int32], ctypes.c_int64),
            "gn_batch_unrolled_forward": ([_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp], ctypes.c_int),
            "gn_batch_unrolled_backward": ([_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
            "gn_unrolled_forward": ([_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp], ctypes.c_int),
            "gn_unrolled_backward": ([_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp],
                                     ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def gn_status_str(s: int) -> str:
    try:
        return lib().gn_status_str(int(s)).decode()
    except Exception:
        return f"status {s}"


def _check(st: int, where: str, allow=(GN_OK,)) -> int:
    if st not in allow:
        raise GNError(st, where)
    return st


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, dtype=None, what="tensor"):
    """Device pointer of a contiguous CUDA tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, ctypes.c_void_p(a.ctypes.data if a.size else 0)


def gn_graph_create(n, row_ptr, col_idx, w, flags=None, validate=True, stream=None):
    """Create a graph handle.  Host numpy arrays or CUDA tensors (int32, int32, float32)."""
    import torch
    dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
    keep = []
    if dev:
        nnz = int(col_idx.numel())
        p_rp = _dptr(row_ptr, torch.int32, "row_ptr")
        p_ci = _dptr(col_idx, torch.int32, "col_idx") if nnz else ctypes.c_void_p(0)
        p_w = _dptr(w, torch.float32, "w") if n else ctypes.c_void_p(0)
        fl = GN_INPUT_DEVICE
    else:
        rp, p_rp = _hptr(row_ptr, np.int32)
        ci, p_ci = _hptr(col_idx, np.int32)
        ww, p_w = _hptr(w, np.float32)
        keep += [rp, ci, ww]
        nnz = int(ci.size)
        fl = GN_INPUT_HOST
    if flags is not None:
        fl = flags
    elif not validate:
        fl |= GN_NO_VALIDATE
    h = ctypes.c_void_p()
    _check(lib().gn_graph_create(int(n), nnz, p_rp, p_ci, p_w, fl, _stream(stream), ctypes.byref(h)),
           "gn_graph_create")
    return h


def gn_graph_destroy(h):
    if h:
        lib().gn_graph_destroy(h)


def gn_graph_info(h) -> dict:
    n = ctypes.c_int32()
    nnz = ctypes.c_int64()
    md = ctypes.c_int32()
    bins = (ctypes.c_int32 * GN_NUM_BINS)()
    _check(lib().gn_graph_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(md), bins), "gn_graph_info")
    names = ["lane16", "lane32", "g8", "wave", "block", "unused5", "unused6"]
    return {"n": n.value, "nnz": nnz.value, "max_degree": md.value,
            "bins": {k: bins[i] for i, k in enumerate(names)}}


def gn_step(h, gamma, x_in, x_out, stream=None):
    import torch
    _check(lib().gn_step(h, float(gamma), _dptr(x_in, torch.float32, "x_in"), _dptr(x_out, torch.float32, "x_out"),
                         _stream(stream)), "gn_step")


def gn_step_static(h, gamma, x_in, x_out, stream=None):
    """gn_step with its work buffer in the library's static device array (no
    allocation; calls on one GPU must not overlap)."""
    import torch
    _check(lib().gn_step_static(h, float(gamma), _dptr(x_in, torch.float32, "x_in"),
                                _dptr(x_out, torch.float32, "x_out"), _stream(stream)), "gn_step_static")


def gn_step_static_max_n() -> int:
    return int(lib().gn_step_static_max_n())


def make_schedule(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=2000, tau=1e-4, check_every=1) -> gn_schedule:
    return gn_schedule(float(gamma0), float(gamma1), int(ramp_steps), int(max_steps), float(tau), int(check_every))


@dataclass
class Result:
    status: int
    steps: int
    binarised: bool
    fallback_count: int
    relaxed_objective: float
    set_objective: float
    set_size: int
    conflicts: int
    uncovered: int
    stab: float


def gn_solve(h, schedule: gn_schedule, x, sel, stream=None) -> Result:
    import torch
    r = gn_result()
    st = lib().gn_solve(h, ctypes.byref(schedule), _dptr(x, torch.float32, "x"), _dptr(sel, torch.uint8, "sel"),
                        ctypes.byref(r), _stream(stream))
    _check(st, "gn_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return Result(st, r.steps, bool(r.binarised), r.fallback_count, r.relaxed_objective, r.set_objective,
                  r.set_size, r.conflicts, r.uncovered, float(r.stab))


def gn_objective(h, x, stream=None) -> float:
    import torch
    out = ctypes.c_double()
    _check(lib().gn_objective(h, _dptr(x, torch.float32, "x"), ctypes.byref(out), _stream(stream)), "gn_objective")
    return out.value


def gn_check_independent(h, sel, stream=None) -> tuple[int, int]:
    import torch
    c = ctypes.c_int64()
    u = ctypes.c_int64()
    _check(lib().gn_check_independent(h, _dptr(sel, torch.uint8, "sel"), ctypes.byref(c), ctypes.byref(u),
                                      _stream(stream)), "gn_check_independent")
    return c.value, u.value


CHUNK_LEN_DEFAULT = 64   # the library's default chain length (gn_set_chunk_len)
PRUNE_INTERVAL_DEFAULT = 64   # steps between rebuilds of the pruned lists (gn_set_prune_interval)


def gn_set_chunk_len(length: int):
    _check(lib().gn_set_chunk_len(int(length)), "gn_set_chunk_len")


def gn_atom_census(n: int, stream=None) -> gn_atom_counts:
    """Connected graphs on n vertices (1..10) up to isomorphism and their GN-atomic
    classes (Appendix A, Table atoms_10), counted on the device."""
    out = gn_atom_counts()
    _check(lib().gn_atom_census(int(n), ctypes.byref(out), _stream(stream)), "gn_atom_census")
    return out


# default (and largest) work bound of gn_solve's one-workgroup path: it is taken
# whenever the graph's LDS image fits
SMALL_LIMIT_DEFAULT = 1 << 20


def gn_set_small_graph_limit(work_max: int):
    _check(lib().gn_set_small_graph_limit(int(work_max)), "gn_set_small_graph_limit")


PRUNE_NEVER, PRUNE_WHERE_IT_PAYS, PRUNE_ALWAYS = 0, 1, 2


def gn_set_multi_handoff(enable: bool):
    """gn_multi_solve: hand the last running start to the single-start chained
    solve (True, the default) or keep it in the 16-start steps; results do not
    change."""
    _check(lib().gn_set_multi_handoff(1 if enable else 0), "gn_set_multi_handoff")


def gn_set_pruning(mode: int):
    """Pruned neighbour lists in gn_solve's chained path: PRUNE_NEVER,
    PRUNE_WHERE_IT_PAYS (the default) or PRUNE_ALWAYS; results do not change."""
    _check(lib().gn_set_pruning(int(mode)), "gn_set_pruning")


def gn_set_prune_interval(steps: int):
    """Steps between rebuilds of the pruned neighbour lists; results do not change."""
    _check(lib().gn_set_prune_interval(int(steps)), "gn_set_prune_interval")


class Graph:
    """Owning wrapper of a gn_graph handle."""

    def __init__(self, n, row_ptr, col_idx, w, validate=True, stream=None):
        self.n = int(n)
        self.handle = gn_graph_create(n, row_ptr, col_idx, w, validate=validate, stream=stream)

    def close(self):
        if getattr(self, "handle", None):
            gn_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return gn_graph_info(self.handle)

    def step(self, gamma, x_in, x_out, stream=None):
        gn_step(self.handle, gamma, x_in, x_out, stream)

    def solve(self, x, sel, stream=None, **sched) -> Result:
        return gn_solve(self.handle, make_schedule(**sched), x, sel, stream)

    def random_starts(self, starts, u, x, stream=None):
        gn_random_starts(self.handle, starts, u, x, stream)

    def multi_solve(self, starts, x, sel, stream=None, **sched):
        """`starts` runs at once; x, sel start-major [starts * n]."""
        return gn_multi_solve(self.handle, make_schedule(**sched), starts, x, sel, stream)

    def objective(self, x, stream=None) -> float:
        return gn_objective(self.handle, x, stream)

    def check(self, sel, stream=None):
        return gn_check_independent(self.handle, sel, stream)


GN_MAX_STARTS = 16


def gn_multi_solve(h, schedule: gn_schedule, starts: int, x, sel, stream=None) -> tuple[int, list[Result], int]:
    """x: CUDA float32 [starts * n] start-major (in: starting points, out: final
    states); sel: CUDA uint8 [starts * n].  Returns (status, per-start results, best)."""
    import torch
    res = (gn_result * int(starts))()
    best = ctypes.c_int32(-1)
    st = lib().gn_multi_solve(h, ctypes.byref(schedule), int(starts), _dptr(x, torch.float32, "x"),
                              _dptr(sel, torch.uint8, "sel"), res, ctypes.byref(best), _stream(stream))
    _check(st, "gn_multi_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return st, [_result(res[b], st) for b in range(int(starts))], best.value


def gn_random_starts(h, starts: int, u, x, stream=None):
    """x = clamp(-log u / max(-log u), 1e-3, 1) per start; u, x CUDA float32 [starts * n]."""
    import torch
    _check(lib().gn_random_starts(h, int(starts), _dptr(u, torch.float32, "u"), _dptr(x, torch.float32, "x"),
                                  _stream(stream)), "gn_random_starts")


def gn_lp_create(n, clique_ptr, members, cost, stream=None):
    """Clique-constrained LP instance from host arrays (int32 CSR of cliques, float32 costs)."""
    cp = np.ascontiguousarray(clique_ptr, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    if c.size != int(n) or cp.size < 2 or int(cp[-1]) != mem.size:
        raise GNError(GN_E_ARG, "gn_lp_create: sizes")
    h = _vp()
    _check(lib().gn_lp_create(int(n), int(cp.size - 1), _vp(cp.ctypes.data), _vp(mem.ctypes.data),
                              _vp(c.ctypes.data), _stream(stream), ctypes.byref(h)), "gn_lp_create")
    return h


def gn_lp_destroy(h):
    if h:
        lib().gn_lp_destroy(h)


def gn_lp_info(h) -> dict:
    k, m, mc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gn_lp_info(h, ctypes.byref(k), ctypes.byref(m), ctypes.byref(mc)), "gn_lp_info")
    return {"n_classes": k.value, "n_cliques": m.value, "max_class": mc.value}


def gn_lp_set_fused(h, enable: bool) -> bool:
    """Fused passes on or off (testing control); True when solves will run fused."""
    r = lib().gn_lp_set_fused(h, 1 if enable else 0)
    if r < 0:
        raise GNError(GN_E_ARG, "gn_lp_set_fused")
    return r == 1


def gn_lp_solve(h, t0, order, x, drop=0.99, t_min=1e-4, max_passes=10000, check_every=10, gap_tol=1e-3,
                x_floor=1e-3, anneal_tol=3e-3, stall=10, stream=None):
    """t0: host float32 [starts]; order: host int32 [starts, n_classes]; x: CUDA
    float32 [starts * n] (out).  Defaults: the paper's 0.1% stop, the annealed
    schedule (anneal_tol <= 0: the drop every pass).  Returns (status, list of
    gn_lp_result)."""
    import torch
    t = np.ascontiguousarray(t0, dtype=np.float32).reshape(-1)
    o = np.ascontiguousarray(order, dtype=np.int32)
    starts = t.size
    res = (gn_lp_result * max(starts, 1))()
    st = lib().gn_lp_solve(h, int(starts), _vp(t.ctypes.data), _vp(o.ctypes.data), float(drop), float(t_min),
                           int(max_passes), int(check_every), float(gap_tol), float(x_floor), float(anneal_tol),
                           int(stall), _dptr(x, torch.float32, "x"), res, _stream(stream))
    _check(st, "gn_lp_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return st, [res[s] for s in range(starts)]


class LP:
    """Owning wrapper of a gn_lp handle (fractional warm start by the clique LP)."""

    def __init__(self, n, clique_ptr, members, cost, stream=None):
        self.n = int(n)
        self.handle = gn_lp_create(n, clique_ptr, members, cost, stream)
        self.info = gn_lp_info(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            gn_lp_destroy(h)
            self.handle = None

    def set_fused(self, enable: bool) -> bool:
        return gn_lp_set_fused(self.handle, enable)

    def solve(self, t0, order, x, **kw):
        return gn_lp_solve(self.handle, t0, order, x, **kw)


def gn_hyper_create(n, edge_ptr, members, w, stream=None):
    """Hyperedge-constrained instance from host arrays (int32 CSR of hyperedges,
    float32 weights)."""
    ep = np.ascontiguousarray(edge_ptr, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.float32)
    if ww.size != int(n) or ep.size < 2 or int(ep[-1]) != mem.size:
        raise GNError(GN_E_ARG, "gn_hyper_create: sizes")
    h = _vp()
    _check(lib().gn_hyper_create(int(n), int(ep.size - 1), _vp(ep.ctypes.data), _vp(mem.ctypes.data),
                                 _vp(ww.ctypes.data), _stream(stream), ctypes.byref(h)), "gn_hyper_create")
    return h


def gn_hyper_destroy(h):
    if h:
        lib().gn_hyper_destroy(h)


def gn_hyper_step(h, gamma, x_in, x_out, stream=None):
    import torch
    _check(lib().gn_hyper_step(h, float(gamma), _dptr(x_in, torch.float32, "x_in"),
                               _dptr(x_out, torch.float32, "x_out"), _stream(stream)), "gn_hyper_step")


def gn_hyper_solve(h, schedule: gn_schedule, x, sel, stream=None) -> Result:
    import torch
    res = gn_result()
    st = lib().gn_hyper_solve(h, ctypes.byref(schedule), _dptr(x, torch.float32, "x"),
                              _dptr(sel, torch.uint8, "sel"), ctypes.byref(res), _stream(stream))
    _check(st, "gn_hyper_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return _result(res, st)


def gn_hyper_multi_solve(h, schedule: gn_schedule, starts: int, x, sel, stream=None):
    """x: CUDA float32 [starts * n] start-major (in: starting points, out: final
    states); sel: CUDA uint8 [starts * n].  Returns (status, per-start results, best)."""
    import torch
    res = (gn_result * int(starts))()
    best = ctypes.c_int32(-1)
    st = lib().gn_hyper_multi_solve(h, ctypes.byref(schedule), int(starts), _dptr(x, torch.float32, "x"),
                                    _dptr(sel, torch.uint8, "sel"), res, ctypes.byref(best), _stream(stream))
    _check(st, "gn_hyper_multi_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return st, [_result(res[b], st) for b in range(int(starts))], best.value


class Hyper:
    """Owning wrapper of a gn_hyper handle (GN under hyperedge constraints)."""

    def __init__(self, n, edge_ptr, members, w, stream=None):
        self.n = int(n)
        self.handle = gn_hyper_create(n, edge_ptr, members, w, stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            gn_hyper_destroy(h)
            self.handle = None

    def step(self, gamma, x_in, x_out, stream=None):
        gn_hyper_step(self.handle, gamma, x_in, x_out, stream)

    def solve(self, x, sel, stream=None, **sched) -> Result:
        return gn_hyper_solve(self.handle, make_schedule(**sched), x, sel, stream)

    def multi_solve(self, starts, x, sel, stream=None, **sched):
        return gn_hyper_multi_solve(self.handle, make_schedule(**sched), starts, x, sel, stream)


def gn_rook_create(rows, cols, w, stream=None):
    """Assignment instance from a rows x cols weight matrix (row-major; host numpy
    array or CUDA tensor, float32)."""
    import torch
    keep = None
    if isinstance(w, torch.Tensor) and w.is_cuda:
        p_w = _dptr(w, torch.float32, "w")
        fl = GN_INPUT_DEVICE
    else:
        keep, p_w = _hptr(w, np.float32)
        fl = GN_INPUT_HOST
    h = ctypes.c_void_p()
    _check(lib().gn_rook_create(int(rows), int(cols), p_w, fl, _stream(stream), ctypes.byref(h)), "gn_rook_create")
    del keep
    return h


def gn_rook_destroy(h):
    if h:
        lib().gn_rook_destroy(h)


def gn_rook_step(h, gamma, x_in, x_out, stream=None):
    import torch
    _check(lib().gn_rook_step(h, float(gamma), _dptr(x_in, torch.float32, "x_in"),
                              _dptr(x_out, torch.float32, "x_out"), _stream(stream)), "gn_rook_step")


def gn_rook_solve(h, schedule: gn_schedule, x, sel, stream=None) -> Result:
    import torch
    r = gn_result()
    st = lib().gn_rook_solve(h, ctypes.byref(schedule), _dptr(x, torch.float32, "x"),
                             _dptr(sel, torch.uint8, "sel"), ctypes.byref(r), _stream(stream))
    _check(st, "gn_rook_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return _result(r, st)


class Rook:
    """Owning wrapper of a gn_rook handle (assignment by cross-normalization)."""

    def __init__(self, rows, cols, w, stream=None):
        self.rows, self.cols = int(rows), int(cols)
        self.handle = gn_rook_create(rows, cols, w, stream)

    def close(self):
        if getattr(self, "handle", None):
            gn_rook_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, gamma, x_in, x_out, stream=None):
        gn_rook_step(self.handle, gamma, x_in, x_out, stream)

    def solve(self, x, sel, stream=None, **sched) -> Result:
        return gn_rook_solve(self.handle, make_schedule(**sched), x, sel, stream)


def _result(r: gn_result, st: int) -> Result:
    return Result(st, r.steps, bool(r.binarised), r.fallback_count, r.relaxed_objective, r.set_objective,
                  r.set_size, r.conflicts, r.uncovered, float(r.stab))


class Results(Sequence):
    """Read-only sequence over a gn_result array filled by the library.  Elements
    become Result objects only when read, so a call that returns thousands of
    results does not build (and later garbage-collect) thousands of objects."""

    def __init__(self, arr, st: int):
        self._arr = arr
        self._st = st

    def __len__(self) -> int:
        return len(self._arr)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [_result(self._arr[k], self._st) for k in range(*i.indices(len(self._arr)))]
        n = len(self._arr)
        if i < 0:
            i += n
        if not 0 <= i < n:
            raise IndexError(i)
        return _result(self._arr[i], self._st)


def gn_batch_create(n, nnz, row_ptr_cat, col_idx_cat, w_cat, validate=True, stream=None):
    """Batch handle from per-graph sizes (host) and concatenated local CSR + weights
    (host numpy arrays or CUDA tensors)."""
    import torch
    ns, p_n = _hptr(n, np.int32)
    nz, p_nz = _hptr(nnz, np.int64)
    keep = [ns, nz]
    if isinstance(row_ptr_cat, torch.Tensor) and row_ptr_cat.is_cuda:
        p_rp = _dptr(row_ptr_cat, torch.int32, "row_ptr_cat")
        p_ci = _dptr(col_idx_cat, torch.int32, "col_idx_cat") if col_idx_cat.numel() else ctypes.c_void_p(0)
        p_w = _dptr(w_cat, torch.float32, "w_cat") if w_cat.numel() else ctypes.c_void_p(0)
        fl = GN_INPUT_DEVICE
    else:
        rp, p_rp = _hptr(row_ptr_cat, np.int32)
        ci, p_ci = _hptr(col_idx_cat, np.int32)
        ww, p_w = _hptr(w_cat, np.float32)
        keep += [rp, ci, ww]
        fl = GN_INPUT_HOST
    if not validate:
        fl |= GN_NO_VALIDATE
    h = ctypes.c_void_p()
    _check(lib().gn_batch_create(len(ns), p_n, p_nz, p_rp, p_ci, p_w, fl, _stream(stream), ctypes.byref(h)),
           "gn_batch_create")
    return h


def gn_batch_destroy(h):
    if h:
        lib().gn_batch_destroy(h)


def gn_batch_solve(h, count, schedule: gn_schedule, x_cat, sel_cat, tuning: gn_tuning | None = None,
                   stream=None) -> tuple[int, Results]:
    import torch
    res = (gn_result * count)()
    st = lib().gn_batch_solve(h, ctypes.byref(schedule), ctypes.byref(tuning) if tuning is not None else None,
                              _dptr(x_cat, torch.float32, "x_cat"), _dptr(sel_cat, torch.uint8, "sel_cat"), res,
                              _stream(stream))
    _check(st, "gn_batch_solve", allow=(GN_OK, GN_NOT_CONVERGED))
    return st, Results(res, st)


def gn_batch_autotune(h, schedule: gn_schedule, stream=None) -> gn_tuning:
    t = gn_tuning()
    _check(lib().gn_batch_autotune(h, ctypes.byref(schedule), ctypes.byref(t), _stream(stream)), "gn_batch_autotune")
    return t


def gn_batch_tuning_cache_size() -> int:
    return int(lib().gn_batch_tuning_cache_size())


def gn_batch_tuning_cache_clear():
    lib().gn_batch_tuning_cache_clear()


def gn_batch_graph(h):
    g = lib().gn_batch_graph(h)
    if not g:
        raise GNError(GN_E_HIP, "gn_batch_graph")
    return ctypes.c_void_p(g)


class Batch:
    """Owning wrapper of a gn_batch handle."""

    def __init__(self, n, nnz, row_ptr_cat, col_idx_cat, w_cat, validate=True, stream=None):
        self.n = np.asarray(n, dtype=np.int64)
        self.count = len(self.n)
        self.total_n = int(self.n.sum())
        self.handle = gn_batch_create(n, nnz, row_ptr_cat, col_idx_cat, w_cat, validate, stream)

    @classmethod
    def from_graphs(cls, graphs, weights, **kw):
        ns = [g.n for g in graphs]
        nnz = [g.nnz for g in graphs]
        rp = np.concatenate([g.row_ptr for g in graphs]).astype(np.int32)
        ci = np.concatenate([g.col_idx for g in graphs]).astype(np.int32)
        w = np.concatenate([np.asarray(x, np.float32) for x in weights])
        return cls(ns, nnz, rp, ci, w, **kw)

    def close(self):
        if getattr(self, "handle", None):
            gn_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, x_cat, sel_cat, tuning=None, stream=None, **sched):
        return gn_batch_solve(self.handle, self.count, make_schedule(**sched), x_cat, sel_cat, tuning, stream)

    def autotune(self, stream=None, **sched) -> gn_tuning:
        return gn_batch_autotune(self.handle, make_schedule(**sched), stream)

    def graph_handle(self):
        return gn_batch_graph(self.handle)


def gn_unrolled_ckpt_floats(h, T, ckpt_every) -> int:
    r = lib().gn_unrolled_ckpt_floats(h, int(T), int(ckpt_every))
    if r < 0:
        raise GNError(GN_E_ARG, "gn_unrolled_ckpt_floats")
    return int(r)


def gn_unrolled_forward(h, w, gammas, ckpt_every, x0, xT, ckpt, stream=None):
    import torch
    gm, p_g = _hptr(gammas, np.float32)
    _check(lib().gn_unrolled_forward(h, _dptr(w, torch.float32, "w") if w is not None else None, p_g, len(gm),
                                     int(ckpt_every), _dptr(x0, torch.float32, "x0"), _dptr(xT, torch.float32, "xT"),
                                     _dptr(ckpt, torch.float32, "ckpt"), _stream(stream)), "gn_unrolled_forward")


def gn_unrolled_backward(h, w, gammas, ckpt_every, ckpt, gxT, gw, gx0, stream=None):
    import torch
    gm, p_g = _hptr(gammas, np.float32)
    _check(lib().gn_unrolled_backward(h, _dptr(w, torch.float32, "w") if w is not None else None, p_g, len(gm),
                                      int(ckpt_every), _dptr(ckpt, torch.float32, "ckpt"),
                                      _dptr(gxT, torch.float32, "gxT"), _dptr(gw, torch.float32, "gw"),
                                      _dptr(gx0, torch.float32, "gx0"), _stream(stream)), "gn_unrolled_backward")


def gn_batch_unrolled_store_floats(h, T) -> int:
    r = lib().gn_batch_unrolled_store_floats(h, int(T))
    if r < 0:
        raise GNError(GN_E_ARG, "gn_batch_unrolled_store_floats")
    return int(r)


def gn_batch_unrolled_forward(h, w_cat, gammas, x0_cat, xT_cat, store, stream=None):
    import torch
    gm, p_g = _hptr(gammas, np.float32)
    _check(lib().gn_batch_unrolled_forward(h, _dptr(w_cat, torch.float32, "w_cat") if w_cat is not None else None,
                                           p_g, len(gm), _dptr(x0_cat, torch.float32, "x0_cat"),
                                           _dptr(xT_cat, torch.float32, "xT_cat"),
                                           _dptr(store, torch.float32, "store") if store is not None else None,
                                           _stream(stream)), "gn_batch_unrolled_forward")


def gn_batch_unrolled_backward(h, w_cat, gammas, store, gxT_cat, gw_cat, gx0_cat, stream=None):
    import torch
    gm, p_g = _hptr(gammas, np.float32)
    _check(lib().gn_batch_unrolled_backward(h, _dptr(w_cat, torch.float32, "w_cat") if w_cat is not None else None,
                                            p_g, len(gm),
                                            _dptr(store, torch.float32, "store") if store is not None else None,
                                            _dptr(gxT_cat, torch.float32, "gxT_cat"),
                                            _dptr(gw_cat, torch.float32, "gw_cat"),
                                            _dptr(gx0_cat, torch.float32, "gx0_cat"), _stream(stream)),
           "gn_batch_unrolled_backward")


GN_MPNN_NPARAMS = 9409


def gn_mpnn_cache_bytes(n) -> int:
    r = lib().gn_mpnn_cache_bytes(int(n))
    if r < 0:
        raise GNError(GN_E_ARG, "gn_mpnn_cache_bytes")
    return int(r)


def gn_mpnn_forward(h, params, x0, z, cache, gate=0.0, stream=None):
    import torch
    _check(lib().gn_mpnn_forward(h, _dptr(params, torch.float32, "params"), float(gate), _dptr(x0, torch.float32, "x0"),
                                 _dptr(z, torch.float32, "z") if z is not None else None,
                                 _dptr(cache, torch.uint8, "cache"), _stream(stream)), "gn_mpnn_forward")


def gn_mpnn_backward(h, params, labels, cache, grad, loss, stream=None):
    import torch
    _check(lib().gn_mpnn_backward(h, _dptr(params, torch.float32, "params"), _dptr(labels, torch.float32, "labels"),
                                  _dptr(cache, torch.uint8, "cache"), _dptr(grad, torch.float32, "grad"),
                                  _dptr(loss, torch.float32, "loss"), _stream(stream)), "gn_mpnn_backward")


def gn_adam_step(params, grad, m, v, lr, beta1, beta2, eps, t, stream=None):
    import torch
    _check(lib().gn_adam_step(_dptr(params, torch.float32, "params"), _dptr(grad, torch.float32, "grad"),
                              _dptr(m, torch.float32, "m"), _dptr(v, torch.float32, "v"), params.numel(), float(lr),
                              float(beta1), float(beta2), float(eps), int(t), _stream(stream)), "gn_adam_step")

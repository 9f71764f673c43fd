"""Thin Python binding of the C ABI in include/mm.h (ctypes; argument marshalling only).

Every computation runs in the HIP library ``libmm355.so``; this module converts
numpy arrays to pointers and status codes to exceptions. Importing it on a
machine without the built library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm355.so")

MM_OK, MM_EINVAL, MM_EOVERFLOW, MM_ENOMEM, MM_EHIP, MM_ERANGE, MM_EBUSY, MM_EINTERNAL, MM_ENOTFOUND = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
CBO, LCOM_PQ, LCOM_HS, RFC = 1, 2, 4, 8
PARETO, PAPER_LCOM, PAPER_CBO = 0, 1, 2
EXPLICIT, ALL, REFERENCED, SIMILAR = 0, 1, 2, 3
SIM_NONZERO, SIM_ABOVE_AVG, SIM_ABOVE_AVG_NZ = 0, 1, 2
SUGGEST_LCOM, SUGGEST_CBO, SUGGEST_SIMILAR = 0, 1, 2
THRESH_NONE, THRESH_AVERAGE = 0, 1
CLASS_CK = np.dtype([("wmc", "<i8"), ("noc", "<i4"), ("dit", "<i4")])
SIM_PAIR = np.dtype([("m1", "<i4"), ("m2", "<i4"), ("shared", "<i4"), ("uni", "<i4")])

CLASS_METRICS = np.dtype([("n_methods", "<i4"), ("n_attrs", "<i4"), ("cbo", "<i4"), ("rfc", "<i4"),
                          ("lcom_p", "<i8"), ("lcom_q", "<i8"), ("hs_num", "<i8"), ("hs_den", "<i8")])
METHOD_METRICS = np.dtype([("fan_in", "<i4"), ("fan_out", "<i4"), ("own_attr_uses", "<i4"),
                           ("own_coaccess_partners", "<i4")])
MOVE_SCORE = np.dtype([("method", "<i4"), ("src", "<i4"), ("dst", "<i4"),
                       ("d_cbo_src", "<i4"), ("d_cbo_dst", "<i4"), ("d_rfc_src", "<i4"), ("d_rfc_dst", "<i4"),
                       ("n_caller_cls", "<i4"), ("n_caller_worse", "<i4"), ("n_caller_better", "<i4"),
                       ("keep", "<i4"), ("pad", "<i4"),
                       ("d_lcom_src", "<i8"), ("d_lcom_dst", "<i8"),
                       ("hs_num_src", "<i8"), ("hs_den_src", "<i8"), ("hs_num_dst", "<i8"), ("hs_den_dst", "<i8")])


class MMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mm error {code}: {msg}")
        self.code = code


class SystemDesc(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("n_methods", ctypes.c_int32), ("n_attrs", ctypes.c_int32),
                ("method_class", ctypes.c_void_p), ("attr_class", ctypes.c_void_p),
                ("acc_off", ctypes.c_void_p), ("acc_idx", ctypes.c_void_p),
                ("call_off", ctypes.c_void_p), ("call_idx", ctypes.c_void_p)]


class EditDesc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("method", ctypes.c_void_p), ("new_class", ctypes.c_void_p),
                ("acc_off", ctypes.c_void_p), ("acc_idx", ctypes.c_void_p),
                ("call_off", ctypes.c_void_p), ("call_idx", ctypes.c_void_p)]


class SystemInfo(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("n_methods", ctypes.c_int32), ("n_attrs", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("nnz_acc", ctypes.c_int64), ("nnz_call", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("version", ctypes.c_int64)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("caller_light", ctypes.c_int32), ("heavy_chunk", ctypes.c_int32),
                ("delta_chunk", ctypes.c_int32), ("delta_grid", ctypes.c_int32),
                ("fill_chunk", ctypes.c_int32), ("fill_group", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("mem_budget_bytes", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("system_id", ctypes.c_int32),
                ("load", ctypes.c_void_p), ("edit", ctypes.c_void_p),
                ("cand_mode", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cand_method", ctypes.c_void_p), ("cand_class", ctypes.c_void_p), ("n_cand", ctypes.c_int64),
                ("metric_mask", ctypes.c_uint32), ("rule", ctypes.c_int32), ("keep_only", ctypes.c_int32),
                ("pad2", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("n_records", ctypes.c_int64), ("records", ctypes.c_void_p),
                ("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double),
                ("error", ctypes.c_char_p)]


class SimStats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_nonzero", ctypes.c_int64), ("n_high", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("threshold", ctypes.c_int32), ("max_union", ctypes.c_int32),
                ("average", ctypes.c_double)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("refused", ctypes.c_int64), ("evicted", ctypes.c_int64), ("records", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("elapsed_s", ctypes.c_double),
                ("resident", ctypes.c_int32), ("queued", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("reloaded", ctypes.c_int64), ("peak_bytes", ctypes.c_uint64)]


REQ_LOAD, REQ_EDIT, REQ_SCORE, REQ_FREE = 1, 2, 3, 4

_P = ctypes.c_void_p
_SIGS = {
    "mm_server_create": ([ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)], ctypes.c_int32),
    "mm_server_destroy": ([_P], ctypes.c_int32),
    "mm_server_submit": ([_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "mm_server_wait": ([_P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(Result)], ctypes.c_int32),
    "mm_server_release": ([_P, ctypes.c_uint64], ctypes.c_int32),
    "mm_server_drain": ([_P], ctypes.c_int32),
    "mm_server_stats": ([_P, ctypes.c_int32, ctypes.POINTER(ServerCounters)], ctypes.c_int32),
    "mm_context_set_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int32),
    "mm_context_get_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int32),
    "mm_autotune": ([_P, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32,
                     ctypes.c_int32, ctypes.POINTER(Tuning)], ctypes.c_int32),
    "mm_load_batch": ([_P, _P, ctypes.c_int32, ctypes.POINTER(_P)], ctypes.c_int32),
    "mm_system_parts": ([_P, ctypes.POINTER(ctypes.c_int32), _P, _P, _P], ctypes.c_int32),
    "mm_context_set_timing": ([_P, ctypes.c_char_p], ctypes.c_int32),
    "mm_context_timing": ([_P, ctypes.POINTER(KernelTime), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                           ctypes.c_int32], ctypes.c_int32),
    "mm_last_error": ([], ctypes.c_char_p),
    "mm_context_create": ([ctypes.c_int32, _P, ctypes.c_uint64, ctypes.POINTER(_P)], ctypes.c_int32),
    "mm_context_destroy": ([_P], ctypes.c_int32),
    "mm_context_memory": ([_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "mm_load_system": ([_P, ctypes.POINTER(SystemDesc), ctypes.POINTER(_P)], ctypes.c_int32),
    "mm_free_system": ([_P], ctypes.c_int32),
    "mm_system_info_get": ([_P, ctypes.POINTER(SystemInfo)], ctypes.c_int32),
    "mm_compute_metrics": ([_P, _P, _P], ctypes.c_int32),
    "mm_compute_metrics_device": ([_P, _P, _P], ctypes.c_int32),
    "mm_score_moves": ([_P, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                        ctypes.c_int32, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_score_moves_device": ([_P, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                               ctypes.c_int32, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_move_affected": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                          ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_set_hierarchy": ([_P, _P, _P], ctypes.c_int32),
    "mm_compute_ck": ([_P, _P], ctypes.c_int32),
    "mm_compute_ck_device": ([_P, _P], ctypes.c_int32),
    "mm_move_affected_noalloc": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_void_p], ctypes.c_int32),
    "mm_similarity": ([_P, ctypes.c_int32, ctypes.POINTER(SimStats)], ctypes.c_int32),
    "mm_similarity_pairs": ([_P, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
                            ctypes.c_int32),
    "mm_set_similarity_threshold": ([_P, ctypes.c_int32], ctypes.c_int32),
    "mm_suggest": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                    ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_suggest_independent": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_plan": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                 ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mm_apply_move": ([_P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "mm_system_set_incremental": ([_P, ctypes.c_int32], ctypes.c_int32),
    "mm_apply_edit": ([_P, ctypes.POINTER(EditDesc)], ctypes.c_int32),
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run `python -m paper_1308_4011_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
        # Loading torch first lets the library bind to that one runtime, so device
        # pointers and streams pass freely between the two; loaded the other way
        # round, torch would start a second runtime that finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != MM_OK:
        raise MMError(rc, lib().mm_last_error().decode(errors="replace"))
    return rc


def _arr(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class Context:
    def __init__(self, device: int = 0, stream: int | None = None, mem_budget: int = 0):
        h = _P()
        _check(lib().mm_context_create(device, stream, mem_budget, ctypes.byref(h)))
        self.handle = h

    def memory(self):
        u, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().mm_context_memory(self.handle, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def close(self):
        if self.handle:
            _check(lib().mm_context_destroy(self.handle))
            self.handle = None


def context_set_timing(ctx: "Context", kernels: str | None):
    """Time launches of the named kernels with HIP events ("*" = all, None/"" = off)."""
    _check(lib().mm_context_set_timing(ctx.handle, kernels.encode() if kernels else None))


def context_timing(ctx: "Context", reset: bool = False) -> dict:
    """{kernel: (launches, total_ms)} since the last reset."""
    n = ctypes.c_int32()
    _check(lib().mm_context_timing(ctx.handle, None, 0, ctypes.byref(n), 0))
    arr = (KernelTime * max(n.value, 1))()
    _check(lib().mm_context_timing(ctx.handle, arr, n.value, ctypes.byref(n), int(reset)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}


def context_set_tuning(ctx: "Context", tuning: dict | None):
    """Set the scoring schedule (None restores the defaults)."""
    if tuning is None:
        _check(lib().mm_context_set_tuning(ctx.handle, None))
    else:
        t = Tuning(**tuning)
        _check(lib().mm_context_set_tuning(ctx.handle, ctypes.byref(t)))


def context_get_tuning(ctx: "Context") -> dict:
    t = Tuning()
    _check(lib().mm_context_get_tuning(ctx.handle, ctypes.byref(t)))
    return t.as_dict()


def context_create(device: int = 0, stream: int | None = None, mem_budget: int = 0) -> Context:
    return Context(device, stream, mem_budget)


def context_destroy(ctx: Context):
    ctx.close()


class System:
    def __init__(self, ctx: Context, handle, n_classes, n_methods):
        self.ctx, self.handle = ctx, handle
        self.n_classes, self.n_methods = n_classes, n_methods

    def free(self):
        if self.handle:
            _check(lib().mm_free_system(self.handle))
            self.handle = None


def load_system(ctx: Context, system) -> System:
    """Upload a system (any object with the mm_system_desc fields as arrays)."""
    keep = [_arr(system.method_class, np.int32), _arr(system.attr_class, np.int32),
            _arr(system.acc_off, np.int64), _arr(system.acc_idx, np.int32),
            _arr(system.call_off, np.int64), _arr(system.call_idx, np.int32)]
    d = SystemDesc(system.n_classes, system.n_methods, system.n_attrs, *(_ptr(a) for a in keep))
    if keep[2].size:
        d.acc_off = keep[2].ctypes.data
    if keep[4].size:
        d.call_off = keep[4].ctypes.data
    h = _P()
    _check(lib().mm_load_system(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
    return System(ctx, h, system.n_classes, system.n_methods)


def _desc(system, keep):
    arrs = [_arr(system.method_class, np.int32), _arr(system.attr_class, np.int32),
            _arr(system.acc_off, np.int64), _arr(system.acc_idx, np.int32),
            _arr(system.call_off, np.int64), _arr(system.call_idx, np.int32)]
    keep.append(arrs)
    return SystemDesc(system.n_classes, system.n_methods, system.n_attrs, *(_ptr(a) for a in arrs))


def load_batch(ctx: Context, systems) -> System:
    """Load independent systems as one batch (their disjoint union)."""
    keep = []
    descs = (SystemDesc * len(systems))(*[_desc(s_, keep) for s_ in systems])
    h = _P()
    _check(lib().mm_load_batch(ctx.handle, descs, len(systems), ctypes.byref(h)))
    return System(ctx, h, sum(s_.n_classes for s_ in systems), sum(s_.n_methods for s_ in systems))


def system_parts(sys_: System) -> dict:
    """Offsets of the parts of a batch: {'classes', 'methods', 'attrs'} arrays of n_parts + 1."""
    n = ctypes.c_int32()
    _check(lib().mm_system_parts(sys_.handle, ctypes.byref(n), None, None, None))
    co, mo, ao = (np.zeros(n.value + 1, np.int32) for _ in range(3))
    _check(lib().mm_system_parts(sys_.handle, ctypes.byref(n), co.ctypes.data, mo.ctypes.data, ao.ctypes.data))
    return {"classes": co, "methods": mo, "attrs": ao}


def split_records(records: np.ndarray, parts: dict) -> list:
    """Per-part records of a batch, with method and class ids local to the part."""
    mo, co = parts["methods"], parts["classes"]
    which = np.searchsorted(mo, records["method"], side="right") - 1
    out = []
    for i in range(len(mo) - 1):
        r = records[which == i].copy()
        r["method"] -= mo[i]
        r["src"] -= co[i]
        r["dst"] -= co[i]
        out.append(r)
    return out


def autotune(sys_: System, cand_mode: int = REFERENCED, cand_method=None, cand_class=None,
             metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO, keep_only: bool = True, repeats: int = 3) -> dict:
    """Time the scoring call under several schedules; the fastest stays set in the context."""
    cm, ct, n = _cands(cand_method, cand_class)
    t = Tuning()
    _check(lib().mm_autotune(sys_.handle, cand_mode, _ptr(cm), _ptr(ct), n, metric_mask, rule, int(keep_only),
                             repeats, ctypes.byref(t)))
    return t.as_dict()


def free_system(sys_: System):
    sys_.free()


def system_info(sys_: System) -> dict:
    info = SystemInfo()
    _check(lib().mm_system_info_get(sys_.handle, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in SystemInfo._fields_ if f != "pad"}


def compute_metrics(sys_: System):
    cls = np.zeros(sys_.n_classes, CLASS_METRICS)
    meth = np.zeros(sys_.n_methods, METHOD_METRICS)
    _check(lib().mm_compute_metrics(sys_.handle, _ptr(cls), _ptr(meth)))
    return cls, meth


def compute_metrics_device(sys_: System, d_cls: int | None, d_meth: int | None):
    _check(lib().mm_compute_metrics_device(sys_.handle, d_cls, d_meth))


def _cands(cand_method, cand_class):
    if cand_method is None:
        return None, None, 0
    cm, ct = _arr(cand_method, np.int32), _arr(cand_class, np.int32)
    if cm.shape != ct.shape:
        raise ValueError("candidate arrays differ in length")
    return cm, ct, len(cm)


def score_moves(sys_: System, cand_mode: int = REFERENCED, cand_method=None, cand_class=None,
                metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO, keep_only: bool = False) -> np.ndarray:
    cm, ct, n = _cands(cand_method, cand_class)
    n_out = ctypes.c_int64()
    L = lib()
    _check(L.mm_score_moves(sys_.handle, cand_mode, _ptr(cm), _ptr(ct), n, metric_mask, rule, int(keep_only),
                            None, 0, ctypes.byref(n_out)))
    out = np.zeros(max(n_out.value, 1), MOVE_SCORE)
    _check(L.mm_score_moves(sys_.handle, cand_mode, _ptr(cm), _ptr(ct), n, metric_mask, rule, int(keep_only),
                            out.ctypes.data, len(out), ctypes.byref(n_out)))
    return out[:n_out.value]


def score_moves_count(sys_: System, cand_mode: int = REFERENCED, cand_method=None, cand_class=None,
                      metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO, keep_only: bool = False) -> int:
    cm, ct, n = _cands(cand_method, cand_class)
    n_out = ctypes.c_int64()
    _check(lib().mm_score_moves(sys_.handle, cand_mode, _ptr(cm), _ptr(ct), n, metric_mask, rule,
                                int(keep_only), None, 0, ctypes.byref(n_out)))
    return n_out.value


def score_moves_device(sys_: System, d_out: int | None, capacity: int, cand_mode: int = REFERENCED,
                       cand_method=None, cand_class=None, metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO,
                       keep_only: bool = False) -> int:
    """Scores into a caller-owned device buffer (e.g. a torch tensor's data_ptr());
    returns the number of records."""
    cm, ct, n = _cands(cand_method, cand_class)
    n_out = ctypes.c_int64()
    _check(lib().mm_score_moves_device(sys_.handle, cand_mode, _ptr(cm), _ptr(ct), n, metric_mask, rule,
                                       int(keep_only), d_out, capacity, ctypes.byref(n_out)))
    return n_out.value


def move_affected(sys_: System, method: int, dst_class: int):
    """Caller classes of `method` other than its class and dst_class (ascending)
    and each one's CBO change under the move (see mm_move_affected)."""
    n = ctypes.c_int64(0)
    _check(lib().mm_move_affected(sys_.handle, method, dst_class, None, None, 0, ctypes.byref(n)))
    cls = np.zeros(max(n.value, 1), np.int32)
    d = np.zeros(max(n.value, 1), np.int32)
    _check(lib().mm_move_affected(sys_.handle, method, dst_class, cls.ctypes.data, d.ctypes.data, n.value,
                                  ctypes.byref(n)))
    return cls[:n.value], d[:n.value]


def set_hierarchy(sys_: System, parent, weight=None):
    """Class hierarchy (parent per class, -1 = none) and method weights (None: all 1)."""
    par = _arr(parent, np.int32)
    w = None if weight is None else _arr(weight, np.int32)
    if len(par) != sys_.n_classes or (w is not None and len(w) != sys_.n_methods):
        raise ValueError("parent / weight sizes differ from the system's")
    _check(lib().mm_set_hierarchy(sys_.handle, _ptr(par), None if w is None else _ptr(w)))


def compute_ck(sys_: System) -> np.ndarray:
    """WMC, NOC and DIT of every class (CLASS_CK records)."""
    out = np.zeros(sys_.n_classes, CLASS_CK)
    _check(lib().mm_compute_ck(sys_.handle, _ptr(out)))
    return out


def compute_ck_device(sys_: System, d_out: int):
    """WMC, NOC and DIT into the caller's device buffer at d_out (n_classes records)."""
    _check(lib().mm_compute_ck_device(sys_.handle, d_out))


def move_affected_noalloc(sys_: System, method: int, dst_class: int, d_cls: int, d_cbo: int, capacity: int,
                          d_n: int) -> None:
    """Enqueue mm_move_affected_noalloc: caller classes and CBO changes into the
    device buffers at addresses d_cls / d_cbo (capacity entries each) and their
    number into the device int64 at d_n; nothing is allocated and nothing waits."""
    _check(lib().mm_move_affected_noalloc(sys_.handle, method, dst_class, d_cls, d_cbo, capacity, d_n))


def similarity(sys_: System, threshold: int = 1) -> dict:
    """Pair and candidate counts under a similarity threshold (see mm_similarity)."""
    st = SimStats()
    _check(lib().mm_similarity(sys_.handle, threshold, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in SimStats._fields_}


def similarity_pairs(sys_: System, threshold: int = 1) -> np.ndarray:
    """High-similarity pairs (m1 < m2, shared, union), (m1, m2) ascending."""
    n = ctypes.c_int64(0)
    _check(lib().mm_similarity_pairs(sys_.handle, threshold, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), SIM_PAIR)
    _check(lib().mm_similarity_pairs(sys_.handle, threshold, out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def set_similarity_threshold(sys_: System, threshold: int):
    _check(lib().mm_set_similarity_threshold(sys_.handle, threshold))


def suggest(sys_: System, kind: int, threshold: int = THRESH_AVERAGE) -> np.ndarray:
    """Ranked suggestions (see mm_suggest), best first."""
    n = ctypes.c_int64(0)
    _check(lib().mm_suggest(sys_.handle, kind, threshold, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), MOVE_SCORE)
    _check(lib().mm_suggest(sys_.handle, kind, threshold, out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def suggest_independent(sys_: System, kind: int, threshold: int = THRESH_AVERAGE) -> np.ndarray:
    """Conflict-free subset of the ranked suggestions (see mm_suggest_independent)."""
    n = ctypes.c_int64(0)
    _check(lib().mm_suggest_independent(sys_.handle, kind, threshold, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), MOVE_SCORE)
    _check(lib().mm_suggest_independent(sys_.handle, kind, threshold, out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def plan(sys_: System, kind: int, threshold: int = THRESH_AVERAGE, max_moves: int = 16,
         keep_applied: bool = False) -> np.ndarray:
    """Greedy plan of up to max_moves moves (see mm_plan)."""
    out = np.zeros(max(max_moves, 1), MOVE_SCORE)
    n = ctypes.c_int64(0)
    _check(lib().mm_plan(sys_.handle, kind, threshold, max_moves, int(keep_applied), out.ctypes.data,
                         ctypes.byref(n)))
    return out[:n.value]


def apply_move(sys_: System, method: int, dst_class: int):
    _check(lib().mm_apply_move(sys_.handle, method, dst_class))


def set_incremental(sys_: System, enabled: bool):
    """Moves recompute only what they touch (True, the default) or everything."""
    _check(lib().mm_system_set_incremental(sys_.handle, int(bool(enabled))))


def apply_edit(sys_: System, methods, new_class, acc_off, acc_idx, call_off, call_idx):
    keep = [_arr(methods, np.int32), None if new_class is None else _arr(new_class, np.int32),
            _arr(acc_off, np.int64), _arr(acc_idx, np.int32), _arr(call_off, np.int64), _arr(call_idx, np.int32)]
    e = EditDesc(len(keep[0]), *(None if a is None else (a.ctypes.data if a.size else None) for a in keep))
    _check(lib().mm_apply_edit(sys_.handle, ctypes.byref(e)))


class Server:
    """Request server keeping systems resident (see mm_server_* in include/mm.h)."""

    def __init__(self, device: int = 0, n_slots: int = 4, queue_capacity: int = 4096, mem_budget: int = 0):
        o = ServerOpts(device, n_slots, queue_capacity, 0, mem_budget)
        h = _P()
        _check(lib().mm_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h

    def _submit(self, req: Request) -> int:
        t = ctypes.c_uint64()
        _check(lib().mm_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def load(self, system_id: int, system) -> int:
        keep = []
        d = _desc(system, keep)
        return self._submit(Request(kind=REQ_LOAD, system_id=system_id, load=ctypes.addressof(d)))

    def edit(self, system_id: int, methods, new_class, acc_off, acc_idx, call_off, call_idx,
             metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO, keep_only: bool = True) -> int:
        keep = [_arr(methods, np.int32), None if new_class is None else _arr(new_class, np.int32),
                _arr(acc_off, np.int64), _arr(acc_idx, np.int32), _arr(call_off, np.int64), _arr(call_idx, np.int32)]
        e = EditDesc(len(keep[0]), *(None if a is None else (a.ctypes.data if a.size else None) for a in keep))
        return self._submit(Request(kind=REQ_EDIT, system_id=system_id, edit=ctypes.addressof(e),
                                    metric_mask=metric_mask, rule=rule, keep_only=int(keep_only)))

    def score(self, system_id: int, cand_mode: int = REFERENCED, cand_method=None, cand_class=None,
              metric_mask: int = CBO | LCOM_PQ, rule: int = PARETO, keep_only: bool = True) -> int:
        cm, ct, n = _cands(cand_method, cand_class)
        return self._submit(Request(kind=REQ_SCORE, system_id=system_id, cand_mode=cand_mode,
                                    cand_method=_ptr(cm), cand_class=_ptr(ct), n_cand=n,
                                    metric_mask=metric_mask, rule=rule, keep_only=int(keep_only)))

    def free(self, system_id: int) -> int:
        return self._submit(Request(kind=REQ_FREE, system_id=system_id))

    def wait(self, ticket: int, timeout_ms: int = -1, release: bool = True) -> dict:
        r = Result()
        rc = lib().mm_server_wait(self.handle, ticket, timeout_ms, ctypes.byref(r))
        if rc not in (MM_OK,) and r.state != 2:
            _check(rc)
        recs = np.zeros(0, MOVE_SCORE)
        if r.n_records:
            buf = (ctypes.c_char * (r.n_records * MOVE_SCORE.itemsize)).from_address(r.records)
            recs = np.frombuffer(bytes(buf), MOVE_SCORE).copy()
        out = {"status": r.status, "slot": r.slot, "records": recs, "submit_ms": r.submit_ms,
               "start_ms": r.start_ms, "end_ms": r.end_ms, "error": (r.error or b"").decode()}
        if release:
            _check(lib().mm_server_release(self.handle, ticket))
        return out

    def drain(self):
        _check(lib().mm_server_drain(self.handle))

    def stats(self, reset: bool = False) -> dict:
        c = ServerCounters()
        _check(lib().mm_server_stats(self.handle, int(reset), ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in ServerCounters._fields_}

    def close(self):
        if self.handle:
            _check(lib().mm_server_destroy(self.handle))
            self.handle = None

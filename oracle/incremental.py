"""ctypes wrapper of the second CPU oracle (mm_oracle_inc.c): move deltas from
per-class grouped counts, multi-threaded.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library. It shares no code with the
first oracle (oracle.py / mm_oracle.c) or with the HIP path; the record layouts
below are declared here on their own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mm_oracle_inc.c")
LIB = os.path.join(HERE, "libmm_oracle_inc.so")

CBO, LCOM_PQ, LCOM_HS, RFC = 1, 2, 4, 8
PARETO, PAPER_LCOM, PAPER_CBO = 0, 1, 2

CLASS_DT = np.dtype([("n_methods", "<i4"), ("n_attrs", "<i4"), ("cbo", "<i4"), ("rfc", "<i4"),
                     ("lcom_p", "<i8"), ("lcom_q", "<i8"), ("hs_num", "<i8"), ("hs_den", "<i8")])
METHOD_DT = np.dtype([("fan_in", "<i4"), ("fan_out", "<i4"), ("own_attr_uses", "<i4"),
                      ("own_coaccess_partners", "<i4")])
MOVE_DT = np.dtype([("method", "<i4"), ("src", "<i4"), ("dst", "<i4"),
                    ("d_cbo_src", "<i4"), ("d_cbo_dst", "<i4"), ("d_rfc_src", "<i4"), ("d_rfc_dst", "<i4"),
                    ("n_caller_cls", "<i4"), ("n_caller_worse", "<i4"), ("n_caller_better", "<i4"),
                    ("keep", "<i4"), ("pad", "<i4"),
                    ("d_lcom_src", "<i8"), ("d_lcom_dst", "<i8"),
                    ("hs_num_src", "<i8"), ("hs_den_src", "<i8"), ("hs_num_dst", "<i8"), ("hs_den_dst", "<i8")])


class _Desc(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("n_methods", ctypes.c_int32), ("n_attrs", ctypes.c_int32),
                ("method_class", ctypes.c_void_p), ("attr_class", ctypes.c_void_p),
                ("acc_off", ctypes.c_void_p), ("acc_idx", ctypes.c_void_p),
                ("call_off", ctypes.c_void_p), ("call_idx", ctypes.c_void_p)]


def build(force: bool = False) -> str:
    """Compile with gcc (plain C11 + POSIX threads, -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.inc_build.argtypes = [ctypes.POINTER(_Desc)]
        L.inc_build.restype = ctypes.c_void_p
        L.inc_free.argtypes = [ctypes.c_void_p]
        L.inc_free.restype = None
        L.inc_metrics.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.inc_metrics.restype = ctypes.c_int
        L.inc_referenced.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.inc_referenced.restype = ctypes.c_int64
        L.inc_score.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]
        L.inc_score.restype = ctypes.c_int
        _lib = L
    return _lib


def host_threads(cap: int = 16) -> int:
    """Threads for the scorer: the CPUs this process may run on, at most `cap`."""
    return max(1, min(len(os.sched_getaffinity(0)), cap))


class Incremental:
    """Grouped counts of one system; scores moves from them."""

    def __init__(self, sys):
        arrs = [np.ascontiguousarray(sys.method_class, np.int32), np.ascontiguousarray(sys.attr_class, np.int32),
                np.ascontiguousarray(sys.acc_off, np.int64), np.ascontiguousarray(sys.acc_idx, np.int32),
                np.ascontiguousarray(sys.call_off, np.int64), np.ascontiguousarray(sys.call_idx, np.int32)]
        arrs = [a if a.size else np.zeros(1, a.dtype) for a in arrs]
        d = _Desc(sys.n_classes, sys.n_methods, sys.n_attrs, *(a.ctypes.data for a in arrs))
        self.n_classes, self.n_methods = sys.n_classes, sys.n_methods
        self._h = lib().inc_build(ctypes.byref(d))
        if not self._h:
            raise ValueError("inc_build rejected the system")

    def close(self):
        if self._h:
            lib().inc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def metrics(self):
        cls = np.zeros(max(self.n_classes, 1), CLASS_DT)
        meth = np.zeros(max(self.n_methods, 1), METHOD_DT)
        if lib().inc_metrics(self._h, cls.ctypes.data, meth.ctypes.data):
            raise RuntimeError("inc_metrics failed")
        return cls[:self.n_classes], meth[:self.n_methods]

    def referenced(self):
        n = lib().inc_referenced(self._h, None, None, 0)
        if n < 0:
            raise RuntimeError("inc_referenced failed")
        cm = np.zeros(max(n, 1), np.int32)
        ct = np.zeros(max(n, 1), np.int32)
        lib().inc_referenced(self._h, cm.ctypes.data, ct.ctypes.data, n)
        return cm[:n], ct[:n]

    def score(self, cand_method, cand_class, mask=CBO | LCOM_PQ, rule=PARETO, threads=None):
        cm = np.ascontiguousarray(cand_method, np.int32)
        ct = np.ascontiguousarray(cand_class, np.int32)
        out = np.zeros(max(len(cm), 1), MOVE_DT)
        nt = host_threads() if threads is None else threads
        rc = lib().inc_score(self._h, len(cm), cm.ctypes.data if len(cm) else None,
                             ct.ctypes.data if len(ct) else None, mask, rule, out.ctypes.data, nt)
        if rc != 0:
            raise ValueError("inc_score rejected its arguments")
        return out[:len(cm)]

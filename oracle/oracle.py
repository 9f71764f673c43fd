"""ctypes wrapper of the CPU oracle (mm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library. It shares no code with the
HIP path; the record layouts below are declared here on their own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mm_oracle.c")
LIB = os.path.join(HERE, "libmm_oracle.so")

CBO, LCOM_PQ, LCOM_HS, RFC = 1, 2, 4, 8
PARETO, PAPER_LCOM, PAPER_CBO = 0, 1, 2
EXPLICIT, ALL, REFERENCED = 0, 1, 2

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
assert CLASS_DT.itemsize == 48 and METHOD_DT.itemsize == 16 and MOVE_DT.itemsize == 96


class _Sys(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("n_methods", ctypes.c_int32), ("n_attrs", ctypes.c_int32),
                ("method_class", ctypes.c_void_p), ("attr_class", ctypes.c_void_p),
                ("acc_off", ctypes.c_void_p), ("acc_idx", ctypes.c_void_p),
                ("call_off", ctypes.c_void_p), ("call_idx", ctypes.c_void_p)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.orc_metrics.argtypes = [ctypes.POINTER(_Sys), ctypes.c_void_p, ctypes.c_void_p]
        L.orc_metrics.restype = ctypes.c_int
        L.orc_candidates.argtypes = [ctypes.POINTER(_Sys), ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64]
        L.orc_candidates.restype = ctypes.c_int64
        L.orc_score.argtypes = [ctypes.POINTER(_Sys), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p]
        L.orc_score.restype = ctypes.c_int
        L.orc_value_count.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L.orc_value_count.restype = ctypes.c_int64
        L.orc_similarity.argtypes = [ctypes.POINTER(_Sys), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.orc_similarity.restype = ctypes.c_int64
        L.orc_ck.argtypes = [ctypes.POINTER(_Sys), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p]
        L.orc_ck.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a.size else None


class _Held:
    """Keeps contiguous copies of the arrays alive while the C struct points at them."""

    def __init__(self, sys):
        self.arrs = [np.ascontiguousarray(sys.method_class, np.int32),
                     np.ascontiguousarray(sys.attr_class, np.int32),
                     np.ascontiguousarray(sys.acc_off, np.int64),
                     np.ascontiguousarray(sys.acc_idx, np.int32),
                     np.ascontiguousarray(sys.call_off, np.int64),
                     np.ascontiguousarray(sys.call_idx, np.int32)]
        # never hand C a NULL row array
        self.arrs = [a if a.size else np.zeros(1, a.dtype) for a in self.arrs]
        self.s = _Sys(sys.n_classes, sys.n_methods, sys.n_attrs, *(a.ctypes.data for a in self.arrs))


def metrics(sys):
    """Per-class and per-method metrics by definition."""
    h = _Held(sys)
    cls = np.zeros(sys.n_classes, CLASS_DT)
    meth = np.zeros(sys.n_methods, METHOD_DT)
    rc = lib().orc_metrics(ctypes.byref(h.s), _ptr(cls), _ptr(meth))
    if rc != 0:
        raise RuntimeError("orc_metrics failed")
    return cls, meth


CK_DT = np.dtype([("wmc", "<i8"), ("noc", "<i4"), ("dit", "<i4")])


class CycleError(ValueError):
    """The parent relation has a cycle."""


def ck(sys, parent, weight=None):
    """WMC, NOC and DIT of every class by definition (orc_ck), as a CK_DT array.
    parent[C] = -1: no parent in the system; weight None: every method weighs 1."""
    h = _Held(sys)
    par = np.ascontiguousarray(parent, np.int32)
    w = None if weight is None else np.ascontiguousarray(weight, np.int32)
    if len(par) != sys.n_classes or (w is not None and len(w) != sys.n_methods):
        raise ValueError("parent / weight sizes differ from the system's")
    out = np.zeros(sys.n_classes, CK_DT)
    wmc = np.zeros(sys.n_classes, np.int64)
    noc = np.zeros(sys.n_classes, np.int32)
    dit = np.zeros(sys.n_classes, np.int32)
    rc = lib().orc_ck(ctypes.byref(h.s), _ptr(par), None if w is None else _ptr(w), _ptr(wmc), _ptr(noc),
                      _ptr(dit))
    if rc == -1:
        raise CycleError("the parent relation has a cycle")
    if rc != 0:
        raise ValueError("bad parent id or negative weight")
    out["wmc"], out["noc"], out["dit"] = wmc, noc, dit
    return out


def candidates(sys, mode):
    h = _Held(sys)
    n = lib().orc_candidates(ctypes.byref(h.s), mode, None, None, 0)
    if n < 0:
        raise ValueError("bad candidate mode")
    cm = np.zeros(max(n, 1), np.int32)
    ct = np.zeros(max(n, 1), np.int32)
    lib().orc_candidates(ctypes.byref(h.s), mode, cm.ctypes.data, ct.ctypes.data, n)
    return cm[:n], ct[:n]


def score(sys, cand_method, cand_class, mask=CBO | LCOM_PQ, rule=PARETO):
    """Score explicit candidates by re-evaluating the changed classes."""
    h = _Held(sys)
    cm = np.ascontiguousarray(cand_method, np.int32)
    ct = np.ascontiguousarray(cand_class, np.int32)
    out = np.zeros(max(len(cm), 1), MOVE_DT)
    rc = lib().orc_score(ctypes.byref(h.s), len(cm), _ptr(cm), _ptr(ct), mask, rule, out.ctypes.data)
    if rc != 0:
        raise ValueError("orc_score rejected its arguments")
    return out[:len(cm)]


def value_count(c, m):
    return lib().orc_value_count(c, m)


def moved(sys, method, dst):
    """The same system with one method's owner changed (plain array copy)."""
    s2 = sys.copy()
    s2.method_class[method] = dst
    return s2


def affected(sys, method, dst):
    """Caller classes of `method` other than its own class and `dst` (ascending)
    and the change of each one's CBO when the method moves to `dst`, both CBO
    values evaluated by definition on the system before and after the move
    (Sec. II-B defines CBO; Sec. IV-A asks that no other class gets worse)."""
    S = int(sys.method_class[method])
    off = np.asarray(sys.call_off)
    idx = np.asarray(sys.call_idx)
    callers = {int(y) for y in range(sys.n_methods)
               if y != method and method in set(idx[off[y]:off[y + 1]].tolist())}
    xs = sorted({int(sys.method_class[y]) for y in callers} - {S, int(dst)})
    before = metrics(sys)[0]["cbo"].astype(np.int64)
    after = metrics(moved(sys, method, dst))[0]["cbo"].astype(np.int64)
    xs = np.array(xs, np.int32)
    return xs, (after[xs] - before[xs]).astype(np.int32)


# ---- similarity (Sec. II-A) and the similarity-driven candidates (Sec. III-A)

SIM_NONZERO, SIM_ABOVE_AVG, SIM_ABOVE_AVG_NZ = 0, 1, 2


def similarity_pairs(sys, lo=0, hi=None):
    """Pairs (m1 < m2, m1 in [lo, hi)) sharing a property, with |shared| and
    |union| of their property sets (Jaccard similarity = shared / union)."""
    hi = sys.n_methods if hi is None else hi
    h = _Held(sys)
    n = lib().orc_similarity(ctypes.byref(h.s), lo, hi, None, None, None, None, 0)
    if n < 0:
        raise ValueError("bad row range")
    out = [np.zeros(max(n, 1), np.int32) for _ in range(4)]
    lib().orc_similarity(ctypes.byref(h.s), lo, hi, *(a.ctypes.data for a in out), n)
    return tuple(a[:n] for a in out)


def similarity_average(n_methods, inter, union, threshold):
    """The average similarity as an exact fraction: the sum of shared / union
    over the listed pairs (every pair with J > 0), divided by the number of all
    pairs n(n-1)/2 (SIM_ABOVE_AVG: zeros included) or of the listed pairs
    (SIM_ABOVE_AVG_NZ). None when there is nothing to average. The sum is taken
    per union size (an exact regrouping of the same terms)."""
    inter = np.asarray(inter, np.int64)
    union = np.asarray(union, np.int64)
    by_union = np.zeros(int(union.max()) + 1 if len(union) else 1, np.int64)
    np.add.at(by_union, union, inter)
    total = sum((Fraction(int(v), u) for u, v in enumerate(by_union.tolist()) if v), Fraction(0))
    count = n_methods * (n_methods - 1) // 2 if threshold == SIM_ABOVE_AVG else len(inter)
    return total / count if count else None


def similarity_kept(n_methods, inter, union, threshold):
    """Boolean mask of the pairs whose similarity is 'high' (Sec. III-A): above
    zero (SIM_NONZERO), or strictly above the average, compared exactly (one
    Fraction comparison per distinct (shared, union) value)."""
    inter = np.asarray(inter, np.int64)
    union = np.asarray(union, np.int64)
    if threshold == SIM_NONZERO:
        return inter > 0
    avg = similarity_average(n_methods, inter, union, threshold)
    if avg is None or len(inter) == 0:
        return np.zeros(len(inter), bool)
    key = inter * (int(union.max()) + 1) + union
    uniq, back = np.unique(key, return_inverse=True)
    width = int(union.max()) + 1
    high = np.array([Fraction(int(k) // width, int(k) % width) > avg for k in uniq.tolist()], bool)
    return high[back]


def similar_candidates(sys, threshold=SIM_ABOVE_AVG, pairs=None):
    """Moves suggested by high similarity (Sec. III-A): for every high-similarity
    pair whose methods sit in different classes, each method may move to the
    other's class or to a class holding a method it calls. (method, class)
    ascending, each once. `pairs` may pass similarity_pairs(sys) already computed."""
    m1, m2, inter, union = similarity_pairs(sys) if pairs is None else pairs
    keep = similarity_kept(sys.n_methods, inter, union, threshold)
    owner = np.asarray(sys.method_class, np.int64)
    a, b = m1[keep].astype(np.int64), m2[keep].astype(np.int64)
    cross = owner[a] != owner[b]
    a, b = a[cross], b[cross]
    c = int(sys.n_classes)
    # the partner's class, both ways
    keys = [a * c + owner[b], b * c + owner[a]]
    # the classes of the methods called by every method of such a pair
    movers = np.unique(np.concatenate([a, b]))
    off = np.asarray(sys.call_off, np.int64)
    idx = np.asarray(sys.call_idx, np.int64)
    lens = off[movers + 1] - off[movers]
    rows = np.repeat(movers, lens)
    callees = idx[np.concatenate([np.arange(off[m], off[m + 1]) for m in movers.tolist()])] if len(movers) \
        else np.zeros(0, np.int64)
    keys.append(rows * c + owner[callees])
    allk = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    cm, ct = allk // c, allk % c
    own = owner[cm] != ct
    return cm[own].astype(np.int32), ct[own].astype(np.int32)


# ---- ranked suggestions (Sec. III-A): threshold on the origin class, rank by fan-in / fan-out

SUGGEST_LCOM, SUGGEST_CBO, SUGGEST_SIMILAR = 0, 1, 2
THRESH_NONE, THRESH_AVERAGE = 0, 1


def suggest(sys, kind, threshold=THRESH_AVERAGE, sim_threshold=SIM_ABOVE_AVG):
    """Suggested moves, best first (Sec. III-A).
    SUGGEST_LCOM: moves out of classes whose LCOM (P - Q) is above the average over
      all classes, to classes the method references, kept when LCOM improves in
      both classes (PAPER_LCOM); methods with the highest fan-out first.
    SUGGEST_CBO: moves out of classes whose CBO is above the average, to classes
      the method uses, kept when the origin's CBO drops, the destination's does
      not rise and no caller class gets worse (PAPER_CBO); highest fan-in +
      fan-out first.
    SUGGEST_SIMILAR: the moves suggested by high-similarity pairs, kept by
      PAPER_LCOM, in candidate order.
    Equal keys keep candidate order ((method, class) ascending). The average
    test is exact: metric(S) * c > sum of the metric over the c classes."""
    cls, meth = metrics(sys)
    if kind == SUGGEST_SIMILAR:
        cm, ct = similar_candidates(sys, sim_threshold)
        mask, rule = LCOM_PQ, PAPER_LCOM
    else:
        cm, ct = candidates(sys, REFERENCED)
        mask, rule = (LCOM_PQ, PAPER_LCOM) if kind == SUGGEST_LCOM else (CBO, PAPER_CBO)
    recs = score(sys, cm, ct, mask, rule)
    recs = recs[recs["keep"] == 1]
    if kind != SUGGEST_SIMILAR and threshold == THRESH_AVERAGE:
        value = (cls["lcom_p"] - cls["lcom_q"]) if kind == SUGGEST_LCOM else cls["cbo"].astype(np.int64)
        total = int(value.sum())
        c = sys.n_classes
        high = [int(v) * c > total for v in value.tolist()]
        recs = recs[np.array([high[s] for s in recs["src"].tolist()], bool)] if len(recs) else recs
    if kind == SUGGEST_LCOM:
        key = [int(meth["fan_out"][m]) for m in recs["method"].tolist()]
    elif kind == SUGGEST_CBO:
        key = [int(meth["fan_in"][m]) + int(meth["fan_out"][m]) for m in recs["method"].tolist()]
    else:
        key = [0] * len(recs)
    order = sorted(range(len(recs)), key=lambda i: -key[i])  # sorted() is stable
    return recs[order]


# ---- multi-move planning on top of the suggestions

def affected_classes(sys, method, dst):
    """Classes a move of `method` to `dst` can change: its class, the destination
    and every class owning a caller of the method (CBO of those)."""
    off = np.asarray(sys.call_off)
    idx = np.asarray(sys.call_idx)
    owners = {int(sys.method_class[y]) for y in range(sys.n_methods)
              if y != method and method in set(idx[off[y]:off[y + 1]].tolist())}
    return owners | {int(sys.method_class[method]), int(dst)}


def independent(sys, kind, threshold=THRESH_AVERAGE):
    """The ranked suggestions reduced, in rank order, to moves whose affected
    classes are disjoint from those of every move taken before: a set of moves
    that can all be applied, each changing the metrics exactly as predicted."""
    ranked = suggest(sys, kind, threshold)
    owner = np.asarray(sys.method_class)
    callers = {}  # method -> classes owning another method that calls it
    for y in range(sys.n_methods):
        for x in set(sys.call_idx[sys.call_off[y]:sys.call_off[y + 1]].tolist()):
            if x != y:
                callers.setdefault(x, set()).add(int(owner[y]))
    used, take = set(), []
    for i, r in enumerate(ranked):
        m = int(r["method"])
        aff = callers.get(m, set()) | {int(owner[m]), int(r["dst"])}
        if aff & used:
            continue
        used |= aff
        take.append(i)
    return ranked[take]


def plan(sys, kind, threshold=THRESH_AVERAGE, max_moves=16):
    """Greedy sequence: apply the best suggestion, re-evaluate, repeat (Sec. IV-C
    re-runs the metrics after a change). Returns the records as scored at each
    step and the system after the moves."""
    cur = sys.copy()
    steps = []
    for _ in range(max_moves):
        r = suggest(cur, kind, threshold)
        if len(r) == 0:
            break
        steps.append(r[:1])
        cur = moved(cur, int(r[0]["method"]), int(r[0]["dst"]))
    out = np.concatenate(steps) if steps else np.zeros(0, MOVE_DT)
    return out, cur

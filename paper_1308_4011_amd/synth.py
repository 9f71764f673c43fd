"""Seeded synthetic software systems (class / method / attribute / call graphs).

This module only draws random graphs. It computes none of the metrics and none
of the move scoring; both the CPU oracle and the HIP path receive the arrays it
returns, unchanged.

The shape of the graphs follows the paper's data model (Section IV-B/IV-C):
every method and attribute belongs to one class, and every method has a list of
invoked methods and a list of accessed attributes, all as numeric ids. The real
systems the paper measured (Table I: Java systems read with BCEL) are not
available, so these generators stand in for them:

* attributes per class ~ Poisson(5);
* accesses per method ~ Poisson(3); each access picks a uniform attribute of the
  method's own class with probability 0.8 (when that class has attributes),
  otherwise a uniform attribute of the whole system;
* calls per method ~ Poisson(lambda_call); targets are drawn Chung-Lu style with
  probability proportional to w_j = 1/u_j, u_j ~ U(0,1], which gives an
  in-degree tail with exponent 2;
* methods per class depend on the workload (see ``WORKLOADS``).

Rows are emitted unsorted and may repeat an id (a method calling the same
target twice); the library treats rows as sets.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 13084011


@dataclasses.dataclass
class System:
    n_classes: int
    n_methods: int
    n_attrs: int
    method_class: np.ndarray  # int32[n_methods]
    attr_class: np.ndarray  # int32[n_attrs]
    acc_off: np.ndarray  # int64[n_methods+1]
    acc_idx: np.ndarray  # int32[nnz_acc]
    call_off: np.ndarray  # int64[n_methods+1]
    call_idx: np.ndarray  # int32[nnz_call]

    def arrays(self):
        return (self.method_class, self.attr_class, self.acc_off, self.acc_idx,
                self.call_off, self.call_idx)

    def copy(self) -> "System":
        return System(self.n_classes, self.n_methods, self.n_attrs,
                      *(a.copy() for a in self.arrays()))

    @property
    def nnz_acc(self) -> int:
        return int(self.acc_off[-1])

    @property
    def nnz_call(self) -> int:
        return int(self.call_off[-1])

    def summary(self) -> dict:
        return {"classes": self.n_classes, "methods": self.n_methods,
                "attrs": self.n_attrs, "acc_nnz": self.nnz_acc,
                "call_nnz": self.nnz_call}


def _offsets(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def build_system(methods_per_class, attrs_per_class, rng: np.random.Generator,
                 lam_acc: float = 3.0, p_own: float = 0.8,
                 lam_call: float = 4.0) -> System:
    """Draw accesses and calls for the given class sizes."""
    mpc = np.asarray(methods_per_class, dtype=np.int64)
    apc = np.asarray(attrs_per_class, dtype=np.int64)
    c = len(mpc)
    method_class = np.repeat(np.arange(c, dtype=np.int32), mpc)
    attr_class = np.repeat(np.arange(c, dtype=np.int32), apc)
    nm, na = len(method_class), len(attr_class)
    attr_first = _offsets(apc)

    # attribute accesses
    k_acc = rng.poisson(lam_acc, nm).astype(np.int64) if na > 0 else np.zeros(nm, np.int64)
    acc_off = _offsets(k_acc)
    nd = int(acc_off[-1])
    draw_cls = np.repeat(method_class, k_acc)
    own_n = apc[draw_cls]
    use_own = (rng.random(nd) < p_own) & (own_n > 0)
    own_pick = attr_first[draw_cls] + rng.integers(0, np.maximum(own_n, 1))
    any_pick = rng.integers(0, max(na, 1), nd)
    acc_idx = np.where(use_own, own_pick, any_pick).astype(np.int32)

    # calls, Chung-Lu targets with weight 1/u
    k_call = rng.poisson(lam_call, nm).astype(np.int64) if nm > 0 else np.zeros(0, np.int64)
    call_off = _offsets(k_call)
    nc = int(call_off[-1])
    if nm > 0 and nc > 0:
        u = 1.0 - rng.random(nm)  # (0, 1]
        cw = np.cumsum(1.0 / u)
        r = rng.random(nc) * cw[-1]
        call_idx = np.minimum(np.searchsorted(cw, r, side="right"), nm - 1).astype(np.int32)
    else:
        call_idx = np.zeros(0, np.int32)
    return System(c, nm, na, method_class, attr_class, acc_off, acc_idx, call_off, call_idx)


def _lognormal_sizes(rng, n, mu, sigma, lo, hi):
    return np.clip(np.rint(rng.lognormal(mu, sigma, n)), lo, hi).astype(np.int64)


def plain(n_classes: int = 200, seed: int = BASE_SEED + 1000) -> System:
    """Small system: methods/class Poisson(10) (0 allowed), calls Poisson(4)."""
    rng = np.random.default_rng(seed)
    mpc = rng.poisson(10.0, n_classes)
    apc = rng.poisson(5.0, n_classes)
    return build_system(mpc, apc, rng, lam_call=4.0)


def medium(n_classes: int = 5000, seed: int = BASE_SEED + 2000) -> System:
    """Methods/class round(LogNormal(2.3, 0.8)) clamped to [1, 500], calls Poisson(4)."""
    rng = np.random.default_rng(seed)
    mpc = _lognormal_sizes(rng, n_classes, 2.3, 0.8, 1, 500)
    apc = rng.poisson(5.0, n_classes)
    return build_system(mpc, apc, rng, lam_call=4.0)


def large(n_classes: int = 50000, seed: int = BASE_SEED + 3000, n_giant: int = 32) -> System:
    """Heavy-tailed: bulk round(LogNormal(2.0, 1.0)) in [1, 2000] plus ``n_giant``
    classes log-uniform in [500, 2000] (one of them exactly 2000); calls Poisson(8)."""
    rng = np.random.default_rng(seed)
    mpc = _lognormal_sizes(rng, n_classes, 2.0, 1.0, 1, 2000)
    n_giant = min(n_giant, n_classes)
    if n_giant > 0:
        where = rng.choice(n_classes, n_giant, replace=False)
        g = np.rint(np.exp(rng.uniform(math.log(500), math.log(2000), n_giant))).astype(np.int64)
        g[0] = 2000
        mpc[where] = g
    apc = rng.poisson(5.0, n_classes)
    return build_system(mpc, apc, rng, lam_call=8.0)


def batch_class_counts(n_systems: int = 256, seed: int = BASE_SEED + 4000) -> np.ndarray:
    """Class counts of a batch of snapshots: round(LogNormal(ln 1414, 1.32)) in [100, 20000]."""
    rng = np.random.default_rng(seed)
    return _lognormal_sizes(rng, n_systems, math.log(1414.0), 1.32, 100, 20000)


def batch(n_systems: int = 256, seed: int = BASE_SEED + 4000, max_classes: int | None = None):
    """Snapshots of uneven sizes, each drawn with the ``medium`` generators."""
    counts = batch_class_counts(n_systems, seed)
    if max_classes is not None:
        counts = np.minimum(counts, max_classes)
    return [medium(int(k), seed=seed + 1 + i) for i, k in enumerate(counts)]


def served_class_counts(n_systems: int = 64, seed: int = BASE_SEED + 5000) -> np.ndarray:
    """Class counts of resident systems, log-uniform in [1000, 50000]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(1000), math.log(50000), n_systems))).astype(np.int64)


def served_system(n_classes: int, seed: int) -> System:
    if n_classes > 20000:
        return large(n_classes, seed=seed, n_giant=max(1, n_classes * 32 // 50000))
    return medium(n_classes, seed=seed)


def tiny(rng: np.random.Generator, max_classes: int = 4, max_methods: int = 5,
         max_attrs: int = 3, lam_acc: float = 2.0, lam_call: float = 2.0) -> System:
    """Very small random systems for exhaustive checks (empty classes allowed)."""
    c = int(rng.integers(1, max_classes + 1))
    mpc = rng.integers(0, max_methods + 1, c)
    if mpc.sum() == 0:
        mpc[0] = 1
    apc = rng.integers(0, max_attrs + 1, c)
    return build_system(mpc, apc, rng, lam_acc=lam_acc, p_own=0.6, lam_call=lam_call)


def edit_batch(sys: System, rng: np.random.Generator, k: int, p_owner: float = 0.25,
               p_drop: float = 0.2, lam_add_call: float = 1.0, lam_add_acc: float = 0.5):
    """A random edit of ``k`` distinct methods: new rows (some edges dropped, some
    added) and, with probability ``p_owner``, a new owner taken from the classes the
    method references. Returns (methods, new_class, acc_off, acc_idx, call_off, call_idx)."""
    nm, na = sys.n_methods, sys.n_attrs
    k = min(k, nm)
    methods = np.sort(rng.choice(nm, k, replace=False)).astype(np.int32)
    new_class = np.empty(k, np.int32)
    acc_rows, call_rows = [], []
    for i, m in enumerate(methods):
        acc = sys.acc_idx[sys.acc_off[m]:sys.acc_off[m + 1]]
        call = sys.call_idx[sys.call_off[m]:sys.call_off[m + 1]]
        acc = acc[rng.random(len(acc)) >= p_drop]
        call = call[rng.random(len(call)) >= p_drop]
        if na > 0:
            acc = np.concatenate([acc, rng.integers(0, na, rng.poisson(lam_add_acc))]).astype(np.int32)
        call = np.concatenate([call, rng.integers(0, nm, rng.poisson(lam_add_call))]).astype(np.int32)
        owner = int(sys.method_class[m])
        if rng.random() < p_owner:
            refs = np.concatenate([sys.method_class[call], sys.attr_class[acc]]) if (len(call) + len(acc)) else np.zeros(0, np.int32)
            refs = refs[refs != owner]
            if len(refs):
                owner = int(refs[rng.integers(0, len(refs))])
        new_class[i] = owner
        acc_rows.append(acc.astype(np.int32))
        call_rows.append(call.astype(np.int32))
    acc_off = _offsets(np.array([len(r) for r in acc_rows], np.int64))
    call_off = _offsets(np.array([len(r) for r in call_rows], np.int64))
    acc_idx = np.concatenate(acc_rows) if acc_rows else np.zeros(0, np.int32)
    call_idx = np.concatenate(call_rows) if call_rows else np.zeros(0, np.int32)
    return methods, new_class, acc_off, acc_idx.astype(np.int32), call_off, call_idx.astype(np.int32)


def apply_edit_arrays(sys: System, methods, new_class, acc_off, acc_idx, call_off, call_idx) -> System:
    """Rebuild a System with the given rows replaced (plain array surgery)."""
    acc_rows = [sys.acc_idx[sys.acc_off[m]:sys.acc_off[m + 1]] for m in range(sys.n_methods)]
    call_rows = [sys.call_idx[sys.call_off[m]:sys.call_off[m + 1]] for m in range(sys.n_methods)]
    mc = sys.method_class.copy()
    for i, m in enumerate(methods):
        acc_rows[m] = acc_idx[acc_off[i]:acc_off[i + 1]]
        call_rows[m] = call_idx[call_off[i]:call_off[i + 1]]
        mc[m] = new_class[i]
    a_off = _offsets(np.array([len(r) for r in acc_rows], np.int64))
    c_off = _offsets(np.array([len(r) for r in call_rows], np.int64))
    a_idx = np.concatenate(acc_rows).astype(np.int32) if a_off[-1] else np.zeros(0, np.int32)
    c_idx = np.concatenate(call_rows).astype(np.int32) if c_off[-1] else np.zeros(0, np.int32)
    return System(sys.n_classes, sys.n_methods, sys.n_attrs, mc, sys.attr_class.copy(),
                  a_off, a_idx, c_off, c_idx)


def hierarchy(n_classes: int, n_methods: int, seed: int, p_extend: float = 0.35, lam_cx: float = 1.5):
    """A class hierarchy and method weights for the rest of the CK suite (WMC,
    NOC, DIT), drawn from their own random stream so the system's graph is
    unchanged. Classes are visited in a random order; each extends, with
    probability ``p_extend``, a uniform class visited before it (single
    inheritance, acyclic), else it has no parent in the system (-1). Method
    weights (a cyclomatic-complexity stand-in) are 1 + Poisson(``lam_cx``).
    Returns (parent int32[n_classes], weight int32[n_methods])."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n_classes)
    parent = np.full(n_classes, -1, np.int32)
    if n_classes > 1:
        ext = rng.random(n_classes) < p_extend
        ext[0] = False
        pos = np.arange(n_classes)
        pick = np.floor(rng.random(n_classes) * np.maximum(pos, 1)).astype(np.int64)
        parent[order[ext]] = order[pick[ext]]
    weight = (1 + rng.poisson(lam_cx, n_methods)).astype(np.int32)
    return parent, weight


def from_lists(n_classes: int, method_class, attr_class, acc_rows, call_rows) -> System:
    """Build a System from Python lists (hand-written fixtures)."""
    mc = np.asarray(method_class, np.int32)
    ac = np.asarray(attr_class, np.int32)
    acc_off = _offsets(np.array([len(r) for r in acc_rows], np.int64))
    call_off = _offsets(np.array([len(r) for r in call_rows], np.int64))
    acc_idx = np.array([x for r in acc_rows for x in r], np.int32)
    call_idx = np.array([x for r in call_rows for x in r], np.int32)
    return System(n_classes, len(mc), len(ac), mc, ac, acc_off, acc_idx, call_off, call_idx)


def stress(seed: int = BASE_SEED + 7000, n_classes: int = 300) -> System:
    """A system built to reach every size regime of the library: an attribute-rich
    class (150 attributes, so own-attribute vectors span three 64-wide blocks), a
    giant class (700 methods), empty classes, and two hub methods called from
    most classes (one by ~1500 methods)."""
    rng = np.random.default_rng(seed)
    mpc = rng.poisson(6.0, n_classes)
    apc = rng.poisson(4.0, n_classes)
    mpc[0], apc[0] = 700, 6
    mpc[1], apc[1] = 40, 150
    mpc[5:8] = 0
    base = build_system(mpc, apc, rng, lam_acc=3.0, p_own=0.8, lam_call=3.0)
    nm = base.n_methods
    first = _offsets(mpc)
    acc_rows = [list(base.acc_idx[base.acc_off[m]:base.acc_off[m + 1]]) for m in range(nm)]
    call_rows = [list(base.call_idx[base.call_off[m]:base.call_off[m + 1]]) for m in range(nm)]
    # attribute-rich class: every method touches ~20 of its 150 attributes
    a1 = np.nonzero(base.attr_class == 1)[0]
    for m in range(first[1], first[2]):
        acc_rows[m] += list(rng.choice(a1, 20, replace=False))
    # hubs: one method of class 2 called once from each of most classes, one
    # method of class 3 called by ~1500 methods
    hub1, hub2 = int(first[2]), int(first[3])
    for C in range(n_classes):
        if mpc[C] > 0 and rng.random() < 0.93:
            call_rows[int(first[C] + rng.integers(0, mpc[C]))].append(hub1)
    for m in rng.choice(nm, min(1500, nm), replace=False):
        call_rows[int(m)].append(hub2)
    return from_lists(n_classes, base.method_class, base.attr_class, acc_rows, call_rows)


WORKLOADS = {
    "plain200": lambda: plain(200),
    "medium5k": lambda: medium(5000),
    "large50k": lambda: large(50000),
}

"""Host logic of the benchmark's algorithmic-byte model (CPU only), which the
roofline line divides by kernel time: every table tier is counted once, the two
passes over the hash-table segments together account for those segments' rows
and grouped entries, and the metric recompute's total is the sum of its kernels."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1308_4011_amd import synth  # noqa: E402


def _class_cbo(s):
    """CBO of every class, from the definition (distinct other classes used)."""
    own = s.method_class.astype(np.int64)
    ar, aa = bench.dedup_rows(s.acc_off, s.acc_idx)
    cr, cc = bench.dedup_rows(s.call_off, s.call_idx)
    src = np.concatenate([own[cr], own[ar]])
    dst = np.concatenate([own[cc], s.attr_class.astype(np.int64)[aa]])
    keep = src != dst
    pairs = np.unique(src[keep] * s.n_classes + dst[keep])
    cls = np.zeros(s.n_classes, dtype=[("cbo", "<i4")])
    cls["cbo"] = np.bincount(pairs // s.n_classes, minlength=s.n_classes)
    return cls


def _hash_tier_bytes(s, cls):
    """Rows and grouped entries of the hash-table segments, written out
    directly: W and CNT of more than mid_hi references, caller maps of more
    than 512 callers."""
    n, c = s.n_methods, s.n_classes
    own = s.method_class.astype(np.int64)
    ar, aa = bench.dedup_rows(s.acc_off, s.acc_idx)
    cr, cc = bench.dedup_rows(s.call_off, s.call_idx)
    mid_hi = 2048 if n >= (1 << 17) else 512
    nmem = np.bincount(own, minlength=c)
    wref = np.bincount(own[cr], minlength=c) + np.bincount(own[ar], minlength=c)
    cref = np.bincount(own[cr], minlength=c)
    c_ent = np.bincount(np.unique(own[cr] * (1 << 31) + cc) >> 31, minlength=c)
    w_ent = cls["cbo"].astype(np.int64)
    big_w, big_c = wref > mid_hi, cref > mid_hi
    total = (20 * nmem + 4 * wref + 8 * w_ent)[big_w].sum() + (12 * nmem + 4 * cref + 8 * c_ent)[big_c].sum()
    rlen = np.bincount(cc, minlength=n)
    self_call = cr == cc
    i_ent = np.bincount(np.unique(cc[~self_call] * (1 << 31) + own[cr[~self_call]]) >> 31, minlength=n)
    big_i = rlen > 512
    total += (4 * rlen + 8 * i_ent)[big_i].sum()
    return int(total), bool(big_w.any() or big_c.any() or big_i.any())


def test_byte_model_of_the_metric_kernels():
    for s in (synth.plain(200), synth.medium(1500)):
        cls = _class_cbo(s)
        b = bench.algorithmic_bytes(s, cls, 1000, 3)
        for k in bench.METRIC_KERNELS:
            assert b.get(k, 0) >= 0, k
        assert b["compute_metrics"] == sum(b.get(k, 0) for k in bench.METRIC_KERNELS)
        want, any_big = _hash_tier_bytes(s, cls)
        assert b["k_big_stage"] + b["k_big_build"] == want
        assert (b["k_big_stage"] > 0) == any_big
        # below 2^17 methods the block-LDS tier is empty: its segments are hash-table segments
        assert s.n_methods < (1 << 17) and b["k_map_tab_mid"] == 0

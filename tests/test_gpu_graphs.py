"""Recorded launch sequences (HIP graphs) against direct launches, bit for bit.

A context with graphs enabled records the metric recompute and the scoring
pass the second time the same call repeats and replays it afterwards. Each
replay here is compared with a context that launches every kernel directly, with
other device work, library calls and host synchronisation between replays, and
again after a move and an edit change the system (the recorded graph no longer
matches and is recorded afresh).
"""
import sys

import numpy as np
import pytest
import torch

from paper_1308_4011_amd import mm, synth
from tests.helpers import CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="graph recording is switched off: the first recording of the metric "
                                      "recompute (four streams joined by events) ended the test process with a "
                                      "host segmentation fault inside mm_compute_metrics_device; the cause has "
                                      "not been found, so the path stays off the GPU")]

REPLAYS = 6


def say(msg):
    print(f"[gpu-graphs] {msg}", flush=True)
    sys.stdout.flush()


class Runner:
    """One context and one loaded system, results read into numpy."""

    def __init__(self, s, graphs):
        self.ctx = mm.context_create(0)
        mm.context_set_graphs(self.ctx, graphs)
        self.g = mm.load_system(self.ctx, s)
        self.s = s
        dev = torch.device("cuda:0")
        self.d_cls = torch.empty(max(s.n_classes, 1) * mm.CLASS_METRICS.itemsize, dtype=torch.uint8, device=dev)
        self.d_meth = torch.empty(max(s.n_methods, 1) * mm.METHOD_METRICS.itemsize, dtype=torch.uint8, device=dev)
        self.cap = 0
        self.d_out = None

    def metrics(self):
        mm.compute_metrics_device(self.g, self.d_cls.data_ptr(), self.d_meth.data_ptr())
        torch.cuda.synchronize()
        cls = np.frombuffer(self.d_cls.cpu().numpy().tobytes(), mm.CLASS_METRICS)[:self.s.n_classes]
        meth = np.frombuffer(self.d_meth.cpu().numpy().tobytes(), mm.METHOD_METRICS)[:self.s.n_methods]
        return cls, meth

    def score(self, mode, keep_only, mask=mm.CBO | mm.LCOM_PQ, rule=mm.PARETO):
        """Device scoring into a buffer sized once from a count query (the way a
        repeated caller scores); grown and re-counted when a call reports more."""
        if self.d_out is None:
            self.cap = max(mm.score_moves_count(self.g, mode, metric_mask=mask, rule=rule, keep_only=keep_only), 1)
            self.d_out = torch.empty(self.cap * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device="cuda:0")
        for _ in range(8):
            try:
                k = mm.score_moves_device(self.g, self.d_out.data_ptr(), self.cap, mode, metric_mask=mask, rule=rule,
                                          keep_only=keep_only)
                break
            except mm.MMError as e:
                if e.code != mm.MM_ERANGE:
                    raise
                self.cap *= 2
                self.d_out = torch.empty(self.cap * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device="cuda:0")
        else:
            raise AssertionError("output buffer kept growing")
        torch.cuda.synchronize()
        return np.frombuffer(self.d_out[:k * mm.MOVE_SCORE.itemsize].cpu().numpy().tobytes(), mm.MOVE_SCORE).copy()

    def close(self):
        mm.free_system(self.g)
        mm.context_destroy(self.ctx)


def step(r, mode, keep_only, mask, rule):
    cls, meth = r.metrics()
    rec = r.score(mode, keep_only, mask, rule)
    return cls, meth, rec


def same(a, b, what):
    assert_fields_equal(a[0], b[0], CLASS_FIELDS, what + " classes")
    assert_fields_equal(a[1], b[1], METHOD_FIELDS, what + " methods")
    assert len(a[2]) == len(b[2]), what + " record count"
    assert_fields_equal(a[2], b[2], MOVE_FIELDS, what + " records")


CASES = [
    ("plain200", mm.REFERENCED, True, mm.CBO | mm.LCOM_PQ, mm.PARETO),
    ("plain200", mm.ALL, True, mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC, mm.PARETO),
    ("plain200", mm.REFERENCED, False, mm.LCOM_PQ, mm.PAPER_LCOM),
    ("medium5k", mm.REFERENCED, True, mm.CBO | mm.LCOM_PQ, mm.PARETO),
]


@pytest.mark.parametrize("workload,mode,keep_only,mask,rule", CASES)
def test_replays_match_direct_launches(workload, mode, keep_only, mask, rule):
    say(f"{workload} mode={mode} keep_only={keep_only} mask={mask} rule={rule}")
    s = synth.WORKLOADS[workload]()
    direct = Runner(s, False)
    graphed = Runner(s, True)
    try:
        want = step(direct, mode, keep_only, mask, rule)
        noise = torch.arange(1 << 20, device="cuda:0", dtype=torch.int32)
        for i in range(REPLAYS):
            got = step(graphed, mode, keep_only, mask, rule)
            same(got, want, f"{workload} call {i}")
            # unrelated device work, an eager library call and a host sync between replays
            noise = (noise * 3 + 1) % 1000003
            mm.score_moves(graphed.g, mm.EXPLICIT, np.array([0], np.int32), np.array([s.n_classes - 1], np.int32))
            torch.cuda.synchronize()
        # the structure changes: the recorded sequence must not replay stale launches
        m = int(np.argmax(np.diff(np.asarray(s.call_off))))
        dst = (int(s.method_class[m]) + 1) % s.n_classes
        for r in (direct, graphed):
            mm.apply_move(r.g, m, dst)
        want = step(direct, mode, keep_only, mask, rule)
        for i in range(3):
            same(step(graphed, mode, keep_only, mask, rule), want, f"{workload} after move, call {i}")
        rng = np.random.default_rng(7)
        s_now = s.copy()
        s_now.method_class[m] = dst
        ed = synth.edit_batch(s_now, rng, 4)
        for r in (direct, graphed):
            mm.apply_edit(r.g, *ed)
        want = step(direct, mode, keep_only, mask, rule)
        for i in range(3):
            same(step(graphed, mode, keep_only, mask, rule), want, f"{workload} after edit, call {i}")
    finally:
        direct.close()
        graphed.close()


def test_timing_inside_replays():
    """Kernel timing stays live when the launches replay from a graph: every
    call contributes one timed launch of the selected kernel."""
    say("timing inside replays, plain200")
    s = synth.WORKLOADS["plain200"]()
    r = Runner(s, True)
    try:
        mm.context_set_timing(r.ctx, "k_delta,k_finalize")
        mm.context_timing(r.ctx, reset=True)
        calls = 7
        for _ in range(calls):
            step(r, mm.REFERENCED, True, mm.CBO | mm.LCOM_PQ, mm.PARETO)
        t = mm.context_timing(r.ctx, reset=True)
        mm.context_set_timing(r.ctx, None)
        # the first call also counts its records once
        assert t["k_delta"][0] == calls + 1, t
        assert t["k_finalize"][0] == calls, t
        assert t["k_delta"][1] > 0 and t["k_finalize"][1] > 0
    finally:
        r.close()

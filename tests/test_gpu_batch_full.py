"""The 256-snapshot batch at its full size, in the launch configuration the
benchmark times.

Snapshot class counts are lognormal in [100, 20,000] (859,977 classes in all),
each snapshot drawn with the generators of the 5,000-class system. As the
benchmark does, metrics go into device buffers and REFERENCED candidates are
scored with the keep rule into a device buffer (49.8M candidates). The oracle
cannot score all of them in seconds, so the checks are:

* metrics of every fourth snapshot and of the largest, field by field;
* the kept records of the five smallest snapshots against the oracle's scores
  of all their REFERENCED candidates;
* 2,000 sampled candidates in each of three large snapshots, scored through the
  batch (EXPLICIT) against the oracle;
* properties on the whole batch: the kept list is in candidate order, every
  kept record's part-local move is one of that part's REFERENCED candidates,
  and the host-output call returns the same records as the device-output call.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal

pytestmark = pytest.mark.gpu

MASK, RULE = mm.CBO | mm.LCOM_PQ, mm.PARETO


def say(msg):
    print(f"[gpu-batch-full] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    say("generating the 256 snapshots")
    systems = synth.batch(256)
    ctx = mm.context_create(0)
    b = mm.load_batch(ctx, systems)
    off = mm.system_parts(b)
    say(f"batch loaded: {b.n_classes} classes, {b.n_methods} methods")
    yield systems, b, off
    b.free()
    mm.context_destroy(ctx)


def test_batch_metrics_in_device_buffers(batch):
    systems, b, off = batch
    dev = torch.device("cuda:0")
    d_cls = torch.empty(b.n_classes * mm.CLASS_METRICS.itemsize, dtype=torch.uint8, device=dev)
    d_meth = torch.empty(b.n_methods * mm.METHOD_METRICS.itemsize, dtype=torch.uint8, device=dev)
    mm.compute_metrics_device(b, d_cls.data_ptr(), d_meth.data_ptr())
    torch.cuda.synchronize()
    cls = np.frombuffer(d_cls.cpu().numpy().tobytes(), mm.CLASS_METRICS)
    meth = np.frombuffer(d_meth.cpu().numpy().tobytes(), mm.METHOD_METRICS)
    sizes = np.array([s.n_classes for s in systems])
    picks = sorted(set(range(0, len(systems), 4)) | {int(np.argmax(sizes))})
    for i in picks:
        s = systems[i]
        oc, om = O.metrics(s)
        c0, c1 = off["classes"][i], off["classes"][i + 1]
        m0, m1 = off["methods"][i], off["methods"][i + 1]
        assert_fields_equal(cls[c0:c1], oc, CLASS_FIELDS, f"snapshot {i} classes")
        assert_fields_equal(meth[m0:m1], om, METHOD_FIELDS, f"snapshot {i} methods")
    say(f"metrics of {len(picks)} snapshots match")


def test_batch_kept_records_in_device_buffer(batch):
    systems, b, off = batch
    n_cand = mm.score_moves_count(b, mm.REFERENCED, metric_mask=MASK, rule=RULE)
    say(f"{n_cand} REFERENCED candidates")
    assert n_cand > 40_000_000
    d_out = torch.empty(n_cand * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device="cuda:0")
    mm.compute_metrics_device(b, None, None)
    kept = mm.score_moves_device(b, d_out.data_ptr(), n_cand, mm.REFERENCED, metric_mask=MASK, rule=RULE,
                                 keep_only=True)
    torch.cuda.synchronize()
    rec = np.frombuffer(d_out[:kept * mm.MOVE_SCORE.itemsize].cpu().numpy().tobytes(), mm.MOVE_SCORE).copy()
    say(f"{kept} kept")
    assert np.all(rec["keep"] == 1)
    # candidate order: by method, then destination class
    key = rec["method"].astype(np.int64) * b.n_classes + rec["dst"]
    assert np.all(np.diff(key) > 0)
    host = mm.score_moves(b, mm.REFERENCED, metric_mask=MASK, rule=RULE, keep_only=True)
    assert host.tobytes() == rec.tobytes()

    per = mm.split_records(rec, off)
    sizes = np.array([s.n_classes for s in systems])
    for i in np.argsort(sizes, kind="stable")[:5]:
        s = systems[i]
        cm, ct = O.candidates(s, O.REFERENCED)
        ro = O.score(s, cm, ct, MASK, RULE)
        assert_fields_equal(per[i], ro[ro["keep"] == 1], MOVE_FIELDS, f"snapshot {i} kept")
    # every kept move is one of its part's REFERENCED candidates
    for i in np.argsort(sizes, kind="stable")[5::16]:
        s = systems[i]
        cm, ct = O.candidates(s, O.REFERENCED)
        ref = set((cm.astype(np.int64) * s.n_classes + ct).tolist())
        got = per[i]["method"].astype(np.int64) * s.n_classes + per[i]["dst"]
        assert set(got.tolist()) <= ref, f"snapshot {i}"
    say("kept records match")


def test_batch_sampled_candidates(batch):
    systems, b, off = batch
    rng = np.random.default_rng(31337)
    sizes = np.array([s.n_classes for s in systems])
    for i in np.argsort(sizes, kind="stable")[-3:]:
        s = systems[i]
        cm, ct = O.candidates(s, O.REFERENCED)
        pick = np.sort(rng.choice(len(cm), 2000, replace=False))
        cm, ct = cm[pick], ct[pick]
        got = mm.score_moves(b, mm.EXPLICIT, cm + off["methods"][i], ct + off["classes"][i], MASK, RULE)
        got = mm.split_records(got, off)[i]
        assert_fields_equal(got, O.score(s, cm, ct, MASK, RULE), MOVE_FIELDS, f"snapshot {i} sampled")
    say("sampled candidates match")

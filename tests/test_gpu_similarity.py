"""Similarity of method pairs (Sec. II-A) and similarity-driven candidates
(Sec. III-A) on the HIP path against the CPU oracle: every pair, every threshold
and every candidate on fixtures, tiny systems, the 200-class system and the
stress system (hub methods); on the 5,000-class system the pair and candidate
counts under each threshold against counts the oracle wrote, and a sample of
SIMILAR candidates scored against the oracle."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import MOVE_FIELDS, assert_fields_equal, fixture_system, load_fixture

pytestmark = pytest.mark.gpu

THRESHOLDS = [mm.SIM_NONZERO, mm.SIM_ABOVE_AVG, mm.SIM_ABOVE_AVG_NZ]


def say(msg):
    print(f"[gpu-sim] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return mm.context_create(0)


def check_system(ctx, s, what, score=True):
    g = mm.load_system(ctx, s)
    pairs = O.similarity_pairs(s)
    m1, m2, i, u = pairs
    for th in THRESHOLDS:
        keep = O.similarity_kept(s.n_methods, i, u, th)
        gp = mm.similarity_pairs(g, th)
        assert len(gp) == int(keep.sum()), (what, th)
        for f, ref in (("m1", m1), ("m2", m2), ("shared", i), ("uni", u)):
            assert np.array_equal(gp[f], ref[keep]), (what, th, f)
        st = mm.similarity(g, th)
        cm, ct = O.similar_candidates(s, th, pairs)
        assert st["n_nonzero"] == len(m1) and st["n_high"] == int(keep.sum()), (what, th)
        assert st["n_candidates"] == len(cm), (what, th)
        if th != mm.SIM_NONZERO and len(m1):
            avg = O.similarity_average(s.n_methods, i, u, th)
            assert abs(st["average"] - float(avg)) <= 1e-12 * float(avg), (what, th)
        mm.set_similarity_threshold(g, th)
        rec = mm.score_moves(g, mm.SIMILAR, metric_mask=mm.LCOM_PQ, rule=mm.PAPER_LCOM)
        assert np.array_equal(rec["method"], cm) and np.array_equal(rec["dst"], ct), (what, th)
        if score and len(cm):
            assert_fields_equal(rec, O.score(s, cm, ct, O.LCOM_PQ, O.PAPER_LCOM), MOVE_FIELDS, f"{what} th {th}")
            kept = mm.score_moves(g, mm.SIMILAR, metric_mask=mm.LCOM_PQ, rule=mm.PAPER_LCOM, keep_only=True)
            assert kept.tobytes() == rec[rec["keep"] == 1].tobytes()
    g.free()


def test_fixture(ctx):
    say("fixture f4")
    fx = load_fixture("f4_similarity.json")
    s = fixture_system(fx)
    g = mm.load_system(ctx, s)
    gp = mm.similarity_pairs(g, mm.SIM_NONZERO)
    assert [[int(r["m1"]), int(r["m2"]), int(r["shared"]), int(r["uni"])] for r in gp] == fx["pairs"]
    for th, key in ((mm.SIM_ABOVE_AVG, "candidates_all"), (mm.SIM_ABOVE_AVG_NZ, "candidates_nonzero")):
        mm.set_similarity_threshold(g, th)
        rec = mm.score_moves(g, mm.SIMILAR, metric_mask=mm.LCOM_PQ, rule=mm.PAPER_LCOM)
        assert [[int(a), int(b)] for a, b in zip(rec["method"], rec["dst"])] == fx[key]
    st = mm.similarity(g, mm.SIM_ABOVE_AVG_NZ)
    assert st["n_high"] == sum(fx["kept_nonzero"]) and abs(st["average"] - 7 / 15) < 1e-15
    g.free()
    check_system(ctx, s, "f4")


def test_tiny_systems(ctx):
    rng = np.random.default_rng(404)
    done = 0
    for k in range(80):
        s = synth.tiny(rng)
        if s.n_methods < 2:
            continue
        check_system(ctx, s, f"tiny {k}")
        done += 1
    say(f"tiny systems: {done}")
    assert done > 50


def test_plain200(ctx):
    s = synth.plain(200)
    say(f"plain200 {s.summary()}")
    check_system(ctx, s, "plain200")


def test_stress_hubs(ctx):
    s = synth.stress(seed=21, n_classes=160)
    say(f"stress {s.summary()}")
    check_system(ctx, s, "stress", score=False)


def test_medium5k_counts(ctx):
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sim_medium5k.json")))
    s = synth.medium(5000)
    say(f"medium5k {s.summary()}")
    g = mm.load_system(ctx, s)
    for name, th in (("nonzero", mm.SIM_NONZERO), ("above_avg", mm.SIM_ABOVE_AVG),
                     ("above_avg_nz", mm.SIM_ABOVE_AVG_NZ)):
        want = gold["thresholds"][name]
        st = mm.similarity(g, th)
        say(f"medium5k {name}: {st}")
        assert st["n_nonzero"] == gold["n_nonzero"]
        assert st["n_high"] == want["n_high"] and st["n_candidates"] == want["n_candidates"], name
        if want["average"]:
            avg = int(want["average"][0]) / int(want["average"][1])
            assert abs(st["average"] - avg) <= 1e-12 * avg
    # the SIMILAR list under the nonzero average (91.6M records, 8.8 GB) scored
    # into device memory; the golden sample and 4,000 more records come back
    import torch
    mm.set_similarity_threshold(g, mm.SIM_ABOVE_AVG_NZ)
    want = gold["thresholds"]["above_avg_nz"]
    n = want["n_candidates"]
    buf = torch.empty((n, mm.MOVE_SCORE.itemsize), dtype=torch.uint8, device="cuda:0")
    got = mm.score_moves_device(g, buf.data_ptr(), n, mm.SIMILAR, metric_mask=mm.LCOM_PQ | mm.CBO,
                                rule=mm.PAPER_LCOM)
    torch.cuda.synchronize()
    assert got == n
    pos = np.array(want["sample_pos"])
    idx = np.unique(np.concatenate([pos, np.random.default_rng(3).choice(n, 4000, replace=False)]))
    rec = np.frombuffer(buf[torch.from_numpy(idx).to("cuda:0")].cpu().numpy().tobytes(), mm.MOVE_SCORE)
    del buf
    at = {int(k): j for j, k in enumerate(idx)}
    sample = rec[[at[int(k)] for k in pos]]
    assert [[int(a), int(b)] for a, b in zip(sample["method"], sample["dst"])] == want["sample"]
    ro = O.score(s, rec["method"], rec["dst"], O.LCOM_PQ | O.CBO, O.PAPER_LCOM)
    assert_fields_equal(rec, ro, MOVE_FIELDS, "medium5k SIMILAR sample")
    g.free()


def test_errors(ctx):
    s = synth.plain(20, seed=2)
    g = mm.load_system(ctx, s)
    for bad in (-1, 3):
        with pytest.raises(mm.MMError) as e:
            mm.similarity(g, bad)
        assert e.value.code == mm.MM_EINVAL
        with pytest.raises(mm.MMError) as e:
            mm.set_similarity_threshold(g, bad)
        assert e.value.code == mm.MM_EINVAL
    import ctypes
    n = ctypes.c_int64(0)
    assert mm.lib().mm_similarity_pairs(g.handle, 0, None, 0, ctypes.byref(n)) == mm.MM_OK and n.value > 1
    buf = np.zeros(1, mm.SIM_PAIR)
    assert mm.lib().mm_similarity_pairs(g.handle, 0, buf.ctypes.data, 1, ctypes.byref(n)) == mm.MM_ERANGE
    g.free()
    b = mm.load_batch(ctx, [synth.plain(10, seed=1), synth.plain(12, seed=2)])
    with pytest.raises(mm.MMError) as e:
        mm.similarity(b, mm.SIM_ABOVE_AVG)
    assert e.value.code == mm.MM_EINVAL
    with pytest.raises(mm.MMError) as e:
        mm.score_moves(b, mm.SIMILAR)
    assert e.value.code == mm.MM_EINVAL
    b.free()
    # after an edit the counts follow the edited system
    s = synth.plain(40, seed=9)
    g = mm.load_system(ctx, s)
    mm.similarity(g, mm.SIM_ABOVE_AVG)
    ed = synth.edit_batch(s, np.random.default_rng(1), k=15)
    mm.apply_edit(g, *ed)
    s2 = synth.apply_edit_arrays(s, *ed)
    m1, m2, i, u = O.similarity_pairs(s2)
    st = mm.similarity(g, mm.SIM_ABOVE_AVG)
    assert st["n_nonzero"] == len(m1) and st["n_high"] == int(O.similarity_kept(s2.n_methods, i, u, 1).sum())
    g.free()

"""Ranked suggestions (Sec. III-A) on the HIP path against the CPU oracle:
every record, in order, for each kind and threshold, on the hand fixture, small
and stress systems and the 5,000-class system."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import MOVE_FIELDS, assert_fields_equal, fixture_system, load_fixture

pytestmark = pytest.mark.gpu

KINDS = [(mm.SUGGEST_LCOM, mm.THRESH_AVERAGE), (mm.SUGGEST_CBO, mm.THRESH_AVERAGE),
         (mm.SUGGEST_LCOM, mm.THRESH_NONE), (mm.SUGGEST_CBO, mm.THRESH_NONE), (mm.SUGGEST_SIMILAR, mm.THRESH_AVERAGE)]


def say(msg):
    print(f"[gpu-suggest] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return mm.context_create(0)


def check(ctx, s, what, kinds=KINDS):
    g = mm.load_system(ctx, s)
    for kind, th in kinds:
        got = mm.suggest(g, kind, th)
        want = O.suggest(s, kind, th)
        assert len(got) == len(want), (what, kind, th)
        assert_fields_equal(got, want, MOVE_FIELDS, f"{what} kind {kind} threshold {th}")
    g.free()


def test_fixture(ctx):
    fx = load_fixture("f5_suggest.json")
    s = fixture_system(fx)
    g = mm.load_system(ctx, s)
    for kind, th, key in ((mm.SUGGEST_LCOM, mm.THRESH_AVERAGE, "suggest_lcom"),
                          (mm.SUGGEST_CBO, mm.THRESH_AVERAGE, "suggest_cbo"),
                          (mm.SUGGEST_SIMILAR, mm.THRESH_AVERAGE, "suggest_similar"),
                          (mm.SUGGEST_LCOM, mm.THRESH_NONE, "suggest_lcom_no_threshold"),
                          (mm.SUGGEST_CBO, mm.THRESH_NONE, "suggest_cbo_no_threshold")):
        r = mm.suggest(g, kind, th)
        assert [[int(a), int(b), int(c)] for a, b, c in zip(r["method"], r["src"], r["dst"])] == fx[key], key
    g.free()
    check(ctx, s, "f5")


def test_small_and_stress(ctx):
    rng = np.random.default_rng(33)
    for k in range(25):
        s = synth.tiny(rng)
        if s.n_classes >= 2 and s.n_methods >= 2:
            check(ctx, s, f"tiny {k}")
    for seed in (1, 2):
        s = synth.plain(60, seed=seed)
        say(f"plain60 seed {seed}")
        check(ctx, s, f"plain60/{seed}")
    s = synth.stress(seed=9, n_classes=150)
    say("stress")
    check(ctx, s, "stress", KINDS[:4])


def test_medium5k(ctx):
    s = synth.medium(5000)
    say("medium5k")
    check(ctx, s, "medium5k", KINDS[:4])


def test_errors(ctx):
    s = synth.plain(20, seed=3)
    g = mm.load_system(ctx, s)
    for kind, th in ((3, 1), (-1, 1), (0, 2), (0, -1)):
        with pytest.raises(mm.MMError) as e:
            mm.suggest(g, kind, th)
        assert e.value.code == mm.MM_EINVAL
    n = ctypes.c_int64(0)
    assert mm.lib().mm_suggest(g.handle, mm.SUGGEST_CBO, mm.THRESH_NONE, None, 0, ctypes.byref(n)) == mm.MM_OK
    if n.value > 0:
        buf = np.zeros(1, mm.MOVE_SCORE)
        rc = mm.lib().mm_suggest(g.handle, mm.SUGGEST_CBO, mm.THRESH_NONE, buf.ctypes.data, n.value - 1,
                                 ctypes.byref(n))
        assert rc == mm.MM_ERANGE
    g.free()
    b = mm.load_batch(ctx, [synth.plain(10, seed=1), synth.plain(12, seed=2)])
    with pytest.raises(mm.MMError) as e:
        mm.suggest(b, mm.SUGGEST_LCOM, mm.THRESH_AVERAGE)
    assert e.value.code == mm.MM_EINVAL
    r = mm.suggest(b, mm.SUGGEST_LCOM, mm.THRESH_NONE)
    assert np.all(r["keep"] == 1)
    b.free()


def test_independent_and_plan_fixture(ctx):
    fx = load_fixture("f5_suggest.json")
    s = fixture_system(fx)
    g = mm.load_system(ctx, s)
    r = mm.suggest_independent(g, mm.SUGGEST_LCOM)
    assert [[int(a), int(b), int(c)] for a, b, c in zip(r["method"], r["src"], r["dst"])] == fx["independent_lcom"]
    for kind, key in ((mm.SUGGEST_LCOM, "plan_lcom"), (mm.SUGGEST_CBO, "plan_cbo")):
        steps = mm.plan(g, kind)
        assert [[int(a), int(b), int(c)] for a, b, c in zip(steps["method"], steps["src"], steps["dst"])] == fx[key]
    g.free()


def test_independent_and_plan_match_oracle(ctx):
    for seed in (3, 5):
        s = synth.plain(80, seed=seed)
        g = mm.load_system(ctx, s)
        for kind, th in ((mm.SUGGEST_LCOM, mm.THRESH_NONE), (mm.SUGGEST_CBO, mm.THRESH_NONE),
                         (mm.SUGGEST_LCOM, mm.THRESH_AVERAGE), (mm.SUGGEST_SIMILAR, mm.THRESH_AVERAGE)):
            got = mm.suggest_independent(g, kind, th)
            want = O.independent(s, kind, th)
            assert_fields_equal(got, want, MOVE_FIELDS, f"independent seed {seed} kind {kind}")
        base = mm.compute_metrics(g)[0].copy()
        steps = mm.plan(g, mm.SUGGEST_LCOM, mm.THRESH_AVERAGE, max_moves=5)
        want, final = O.plan(s, mm.SUGGEST_LCOM, mm.THRESH_AVERAGE, max_moves=5)
        assert_fields_equal(steps, want, MOVE_FIELDS, f"plan seed {seed}")
        # restored: the metrics are those of the original system
        assert mm.compute_metrics(g)[0].tobytes() == base.tobytes()
        # kept: the metrics are those of the planned system
        mm.plan(g, mm.SUGGEST_LCOM, mm.THRESH_AVERAGE, max_moves=5, keep_applied=True)
        assert mm.compute_metrics(g)[0].tobytes() == O.metrics(final)[0].tobytes()
        g.free()


def test_independent_medium5k(ctx):
    s = synth.medium(5000)
    say("independent medium5k")
    g = mm.load_system(ctx, s)
    got = mm.suggest_independent(g, mm.SUGGEST_CBO, mm.THRESH_AVERAGE)
    want = O.independent(s, mm.SUGGEST_CBO, mm.THRESH_AVERAGE)
    assert_fields_equal(got, want, MOVE_FIELDS, "independent medium5k")
    g.free()

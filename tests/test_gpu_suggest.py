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

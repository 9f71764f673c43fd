"""The two CPU oracles against each other (they share no code).

The first oracle evaluates every metric by its definition and scores a move by
re-evaluating the changed classes; the second keeps grouped counts and derives
each delta from incremental formulas. Equal records on every move of hundreds of
tiny systems, every REFERENCED move of the 200-class and stress systems,
samples of the 5,000- and 50,000-class systems (moves touching the giant
classes included), and every rule set, pin the second oracle to the first, which
the hand fixtures and closed forms pin to the paper.
"""
import numpy as np
import pytest

from oracle import incremental as I
from oracle import oracle as O
from paper_1308_4011_amd import synth
from tests.helpers import CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal, fixture_system, load_fixture

RULE_SETS = [(O.CBO | O.LCOM_PQ, O.PARETO), (O.LCOM_PQ | O.LCOM_HS, O.PAPER_LCOM), (O.CBO, O.PAPER_CBO),
             (O.CBO | O.LCOM_PQ | O.LCOM_HS | O.RFC, O.PARETO), (O.LCOM_HS, O.PARETO), (O.CBO | O.LCOM_HS, O.PARETO),
             (O.RFC, O.PARETO), (O.LCOM_HS, O.PAPER_LCOM)]


def _same(s, cm, ct, what, rule_sets=RULE_SETS, threads=4):
    inc = I.Incremental(s)
    c1, m1 = O.metrics(s)
    c2, m2 = inc.metrics()
    assert_fields_equal(c1, c2, CLASS_FIELDS, what + " classes")
    assert_fields_equal(m1, m2, METHOD_FIELDS, what + " methods")
    for mask, rule in rule_sets:
        r1 = O.score(s, cm, ct, mask, rule)
        r2 = inc.score(cm, ct, mask, rule, threads=threads)
        assert_fields_equal(r1, r2, MOVE_FIELDS, f"{what} mask {mask} rule {rule}")
    return inc


@pytest.mark.parametrize("name", ["f1_small_two_classes.json", "f2_pareto_kept.json", "f3_caller_class.json",
                                  "f6_lcom_hs_rules.json", "f7_caller_better.json"])
def test_fixtures(name):
    s = fixture_system(load_fixture(name))
    cm, ct = O.candidates(s, O.ALL)
    _same(s, cm, ct, name)


def test_tiny_every_move():
    rng = np.random.default_rng(314)
    seen = 0
    for trial in range(300):
        s = synth.tiny(rng)
        if s.n_classes < 2:
            continue
        cm, ct = O.candidates(s, O.ALL)
        inc = _same(s, cm, ct, f"tiny{trial}")
        im, it = inc.referenced()
        rm, rt = O.candidates(s, O.REFERENCED)
        assert np.array_equal(im, rm) and np.array_equal(it, rt)
        seen += len(cm)
    assert seen > 3000


def test_plain200_every_referenced_move():
    s = synth.plain(200)
    cm, ct = O.candidates(s, O.REFERENCED)
    inc = _same(s, cm, ct, "plain200")
    im, it = inc.referenced()
    assert np.array_equal(im, cm) and np.array_equal(it, ct)


def test_stress_sample():
    """The stress system (a 700-method class, a 150-attribute class, hub methods
    called from most classes): every move of the hubs and of the wide class, and
    a uniform sample of the rest."""
    s = synth.stress()
    cm, ct = O.candidates(s, O.REFERENCED)
    fan_in = np.bincount(s.call_idx, minlength=s.n_methods)
    special = np.nonzero(np.isin(cm, np.argsort(fan_in)[-2:]) | (s.method_class[cm] == 1) | (ct == 1))[0]
    idx = np.union1d(special, np.random.default_rng(8).choice(len(cm), 1500, replace=False))
    inc = _same(s, cm[idx], ct[idx], "stress", RULE_SETS[:2])
    im, it = inc.referenced()
    assert np.array_equal(im, cm) and np.array_equal(it, ct)


def test_threads_give_identical_records():
    s = synth.plain(200, seed=9)
    inc = I.Incremental(s)
    cm, ct = inc.referenced()
    a = inc.score(cm, ct, threads=1)
    b = inc.score(cm, ct, threads=7)
    assert a.tobytes() == b.tobytes()


def test_medium5k_sample():
    s = synth.medium(5000)
    cm, ct = O.candidates(s, O.REFERENCED)
    idx = np.sort(np.random.default_rng(4).choice(len(cm), 6000, replace=False))
    _same(s, cm[idx], ct[idx], "medium5k", RULE_SETS[:4])


def test_large50k_sample_with_giants():
    s = synth.large(50000)
    inc = I.Incremental(s)
    c1, m1 = O.metrics(s)
    c2, m2 = inc.metrics()
    assert_fields_equal(c1, c2, CLASS_FIELDS, "large50k classes")
    assert_fields_equal(m1, m2, METHOD_FIELDS, "large50k methods")
    cm, ct = inc.referenced()
    rm, rt = O.candidates(s, O.REFERENCED)
    assert np.array_equal(cm, rm) and np.array_equal(ct, rt)
    n = c1["n_methods"]
    rng = np.random.default_rng(6)
    small = (n[s.method_class[cm]] < 300) & (n[ct] < 300)
    giant_src = np.nonzero(n[s.method_class[cm]] >= 500)[0]
    giant_dst = np.nonzero(n[ct] >= 500)[0]
    fan_in = np.bincount(s.call_idx, minlength=s.n_methods)
    hubs = np.nonzero(np.isin(cm, np.argsort(fan_in)[-3:]))[0]
    idx = np.unique(np.concatenate([rng.choice(np.nonzero(small)[0], 2500, replace=False),
                                    rng.choice(giant_src, 4, replace=False), rng.choice(giant_dst, 4, replace=False),
                                    hubs[:20]]))
    for mask, rule in RULE_SETS[:1]:
        r1 = O.score(s, cm[idx], ct[idx], mask, rule)
        r2 = inc.score(cm[idx], ct[idx], mask, rule)
        assert_fields_equal(r1, r2, MOVE_FIELDS, f"large50k mask {mask} rule {rule}")


def test_rejects_bad_arguments():
    s = fixture_system(load_fixture("f2_pareto_kept.json"))
    inc = I.Incremental(s)
    with pytest.raises(ValueError):
        inc.score([1], [int(s.method_class[1])])  # destination is the current owner
    with pytest.raises(ValueError):
        inc.score([1], [1 - int(s.method_class[1])], O.CBO, O.PAPER_LCOM)  # LCOM rule without an LCOM metric
    with pytest.raises(ValueError):
        inc.score([0], [99])

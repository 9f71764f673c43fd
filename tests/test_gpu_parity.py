"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every count and delta is an integer, so the bar is bit-exact equality on every
field. Sizes: hand fixtures, hundreds of tiny random systems (every move), the
stress system (multi-block MFMA operands, hash-partitioned groups, hub methods),
the 200-class system with every move, the 5,000-class system with its full
REFERENCED candidate list checked and a sample of moves scored by the oracle,
and the 50,000-class system (full metrics, sampled moves).
"""
import ctypes
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import (CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal,
                           fixture_system, load_fixture)

pytestmark = pytest.mark.gpu

RULE_SETS = [(mm.CBO | mm.LCOM_PQ, mm.PARETO), (mm.LCOM_PQ | mm.LCOM_HS, mm.PAPER_LCOM),
             (mm.CBO, mm.PAPER_CBO), (mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC, mm.PARETO)]


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = mm.context_create(0)
    yield c


def load(ctx, s):
    return mm.load_system(ctx, s)


def check_metrics(g, s, what):
    gc, gm = mm.compute_metrics(g)
    oc, om = O.metrics(s)
    assert_fields_equal(gc, oc, CLASS_FIELDS, what + " classes")
    assert_fields_equal(gm, om, METHOD_FIELDS, what + " methods")
    return oc, om


def check_scores(g, s, cm, ct, mask, rule, what):
    rg = mm.score_moves(g, mm.EXPLICIT, cm, ct, mask, rule)
    ro = O.score(s, cm, ct, mask, rule)
    assert len(rg) == len(ro)
    assert_fields_equal(rg, ro, MOVE_FIELDS, what)
    return rg


FIXTURES = [("f1_small_two_classes.json", None), ("f2_pareto_kept.json", None),
            ("f3_caller_class.json", None), ("f3_caller_class.json", "variant_b"),
            ("f6_lcom_hs_rules.json", None), ("f7_caller_better.json", None)]
RULE_NAMES = {"pareto_cbo_lcom": (mm.CBO | mm.LCOM_PQ, mm.PARETO), "paper_lcom": (mm.LCOM_PQ, mm.PAPER_LCOM),
              "paper_cbo": (mm.CBO, mm.PAPER_CBO),
              "pareto_cbo_lcom_rfc": (mm.CBO | mm.LCOM_PQ | mm.RFC, mm.PARETO),
              "paper_lcom_hs": (mm.LCOM_HS, mm.PAPER_LCOM),
              "paper_lcom_pq_hs": (mm.LCOM_PQ | mm.LCOM_HS, mm.PAPER_LCOM),
              "pareto_hs": (mm.LCOM_HS, mm.PARETO),
              "pareto_cbo_hs": (mm.CBO | mm.LCOM_HS, mm.PARETO),
              "pareto_cbo": (mm.CBO, mm.PARETO)}


@pytest.mark.parametrize("name,variant", FIXTURES)
def test_fixtures(ctx, name, variant):
    say(f"fixture {name} {variant}")
    fx = load_fixture(name)
    s = fixture_system(fx, variant)
    src = fx if variant is None else fx[variant]
    g = load(ctx, s)
    gc, gm = mm.compute_metrics(g)
    for f in CLASS_FIELDS:
        assert gc[f].tolist() == [c[f] for c in src["classes"]], f
    if "methods" in src:
        for f in METHOD_FIELDS:
            assert gm[f].tolist() == [x[f] for x in src["methods"]], f
    if variant is None:
        ref = mm.score_moves(g, mm.REFERENCED)
        assert [[int(a), int(b)] for a, b in zip(ref["method"], ref["dst"])] == fx["referenced"]
    moves = src["moves"]
    cm = [mv["method"] for mv in moves]
    ct = [mv["dst"] for mv in moves]
    for rname, expect in moves[0]["keep"].items():
        mask, rule = RULE_NAMES[rname]
        r = mm.score_moves(g, mm.EXPLICIT, cm, ct, mask, rule)
        for f in MOVE_FIELDS:
            if f == "keep":
                assert r["keep"].tolist() == [mv["keep"][rname] for mv in moves], rname
            else:
                assert r[f].tolist() == [mv[f] for mv in moves], (rname, f)
    g.free()


def test_tiny_exhaustive(ctx):
    rng = np.random.default_rng(99)
    for trial in range(150):
        s = synth.tiny(rng, max_classes=5, max_methods=6, max_attrs=4)
        say(f"tiny trial {trial} {s.summary()}")
        g = load(ctx, s)
        check_metrics(g, s, f"tiny{trial}")
        if s.n_classes > 1:
            cm, ct = O.candidates(s, O.ALL)
            for mask, rule in RULE_SETS:
                ra = mm.score_moves(g, mm.ALL, metric_mask=mask, rule=rule)
                ro = O.score(s, cm, ct, mask, rule)
                assert_fields_equal(ra, ro, MOVE_FIELDS, f"tiny{trial} ALL rule {rule} mask {mask}")
            rm, rt = O.candidates(s, O.REFERENCED)
            rr = mm.score_moves(g, mm.REFERENCED)
            assert np.array_equal(rr["method"], rm) and np.array_equal(rr["dst"], rt)
        g.free()


def test_stress_system(ctx):
    s = synth.stress()
    say(f"stress {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "stress")
    cm, ct = O.candidates(s, O.REFERENCED)
    rr = mm.score_moves(g, mm.REFERENCED)
    assert np.array_equal(rr["method"], cm) and np.array_equal(rr["dst"], ct)
    ro = O.score(s, cm, ct)
    assert_fields_equal(rr, ro, MOVE_FIELDS, "stress REFERENCED")
    # moves of the hub methods into every class (caller lists on the partitioned path)
    counts = np.bincount(s.call_idx, minlength=s.n_methods)
    hubs = np.argsort(counts)[-3:]
    hm = np.repeat(hubs, s.n_classes)
    ht = np.tile(np.arange(s.n_classes), len(hubs))
    keep = ht != s.method_class[hm]
    for mask, rule in RULE_SETS:
        check_scores(g, s, hm[keep], ht[keep], mask, rule, f"stress hubs rule {rule}")
    # every move of the attribute-rich class's methods into the giant class and back
    m1 = np.nonzero(s.method_class == 1)[0]
    m0 = np.nonzero(s.method_class == 0)[0][:40]
    check_scores(g, s, np.concatenate([m1, m0]), np.concatenate([np.zeros_like(m1), np.ones_like(m0)]),
                 mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC, mm.PARETO, "stress wide/giant")
    g.free()


def test_coaccess_wide_and_chunked_classes(ctx):
    """Co-access counts of a class larger than one LDS staging pass (9,000
    methods, 40 attributes), a class with more than 64 own attributes (several
    MFMA k-blocks) and small classes beside them; every metric against the
    oracle, and the four moves of one of the big class's methods (the oracle
    re-evaluates the 9,000-method class for each)."""
    rng = np.random.default_rng(20240611)
    s = synth.build_system([9000, 120, 3, 37, 1], [40, 150, 2, 64, 0], rng, lam_acc=2.0, lam_call=3.0)
    say(f"co-access classes {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "co-access classes")
    ms = rng.choice(9000, 1, replace=False).astype(np.int32)
    cm = np.repeat(ms, s.n_classes - 1)
    ct = np.array([t for m in ms for t in range(s.n_classes) if t != s.method_class[m]], np.int32)
    check_scores(g, s, cm, ct, mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC, mm.PARETO, "co-access classes moves")
    g.free()


def test_rows_longer_than_a_segment(ctx):
    """Methods whose calls and accesses exceed one 64-lane segment take the
    one-lane-per-method preparation and candidate fill: metrics and the full
    REFERENCED list against the oracle, under every rule set."""
    rng = np.random.default_rng(4242)
    s0 = synth.plain(150, seed=21)
    ms = np.sort(rng.choice(s0.n_methods, 5, replace=False)).astype(np.int32)
    calls = [np.sort(rng.choice(s0.n_methods, int(rng.integers(70, 200)), replace=False)) for _ in ms]
    accs = [np.sort(rng.choice(s0.n_attrs, int(rng.integers(10, 40)), replace=False)) for _ in ms]
    off = lambda rows: np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    s = synth.apply_edit_arrays(s0, ms, s0.method_class[ms], off(accs), np.concatenate(accs).astype(np.int32),
                                off(calls), np.concatenate(calls).astype(np.int32))
    row = np.diff(np.asarray(s.call_off)) + np.diff(np.asarray(s.acc_off))
    assert (row > 64).sum() >= 5
    say(f"long rows {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "long rows")
    cm, ct = O.candidates(s, O.REFERENCED)
    for mask, rule in ALL_RULE_SETS:
        rr = mm.score_moves(g, mm.REFERENCED, metric_mask=mask, rule=rule)
        assert np.array_equal(rr["method"], cm) and np.array_equal(rr["dst"], ct)
        assert_fields_equal(rr, O.score(s, cm, ct, mask, rule), MOVE_FIELDS, f"long rows mask {mask} rule {rule}")
        kept = mm.score_moves(g, mm.REFERENCED, metric_mask=mask, rule=rule, keep_only=True)
        assert kept.tobytes() == rr[rr["keep"] == 1].tobytes()
    g.free()


def test_tables_wider_than_the_lds_grouping(ctx):
    """Two methods call one method in each of 2,600 other classes: their rows
    are longer than a fill item, so they are cut into pieces of their row, and
    their classes' W tables (8,192 slots) span two partitions. Metrics and
    REFERENCED scores against the oracle."""
    rng = np.random.default_rng(977)
    s0 = synth.plain(3000, seed=23)
    mc = np.asarray(s0.method_class)
    order = np.argsort(mc, kind="stable")
    start = np.searchsorted(mc[order], np.arange(s0.n_classes + 1))
    ms = np.sort(rng.choice(s0.n_methods, 2, replace=False)).astype(np.int32)
    calls, accs = [], []
    for _ in ms:
        classes = [c for c in rng.choice(s0.n_classes, 2600, replace=False) if start[c + 1] > start[c]]
        pick = [order[start[c] + rng.integers(start[c + 1] - start[c])] for c in classes]
        calls.append(np.unique(np.asarray(pick, np.int32)))
        accs.append(np.sort(rng.choice(s0.n_attrs, 300, replace=False)))
    off = lambda rows: np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    s = synth.apply_edit_arrays(s0, ms, s0.method_class[ms], off(accs), np.concatenate(accs).astype(np.int32),
                                off(calls), np.concatenate(calls).astype(np.int32))
    assert min(len(c) for c in calls) > 2100
    say(f"wide tables {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "wide tables")
    cm, ct = O.candidates(s, O.REFERENCED)
    rr = mm.score_moves(g, mm.REFERENCED, metric_mask=mm.CBO | mm.LCOM_PQ | mm.RFC)
    assert np.array_equal(rr["method"], cm) and np.array_equal(rr["dst"], ct)
    assert_fields_equal(rr, O.score(s, cm, ct, mm.CBO | mm.LCOM_PQ | mm.RFC), MOVE_FIELDS, "wide tables")
    g.free()


def test_plain200_every_move(ctx):
    s = synth.plain(200)
    say(f"plain200 {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "plain200")
    cm, ct = O.candidates(s, O.ALL)
    ra = mm.score_moves(g, mm.ALL, metric_mask=mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC)
    ro = O.score(s, cm, ct, mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC)
    assert len(ra) == len(ro) == s.n_methods * (s.n_classes - 1)
    assert_fields_equal(ra, ro, MOVE_FIELDS, "plain200 ALL")
    g.free()


def test_medium5k(ctx):
    s = synth.medium(5000)
    say(f"medium5k {s.summary()}")
    g = load(ctx, s)
    check_metrics(g, s, "medium5k")
    cm, ct = O.candidates(s, O.REFERENCED)
    rr = mm.score_moves(g, mm.REFERENCED)
    assert np.array_equal(rr["method"], cm) and np.array_equal(rr["dst"], ct)
    idx = np.random.default_rng(1).choice(len(cm), 20000, replace=False)
    idx.sort()
    ro = O.score(s, cm[idx], ct[idx])
    assert_fields_equal(rr[idx], ro, MOVE_FIELDS, "medium5k REFERENCED sample")
    g.free()


def test_large50k(ctx):
    s = synth.large(50000)
    say(f"large50k {s.summary()}")
    g = load(ctx, s)
    oc, _ = check_metrics(g, s, "large50k")
    cm, ct = O.candidates(s, O.REFERENCED)
    n = mm.score_moves_count(g, mm.REFERENCED)
    assert n == len(cm)
    rr = mm.score_moves(g, mm.REFERENCED)
    assert np.array_equal(rr["method"], cm) and np.array_equal(rr["dst"], ct)
    rng = np.random.default_rng(2)
    # a uniform sample plus the candidates of the most-called methods
    fan_in = np.bincount(s.call_idx, minlength=s.n_methods)
    top = set(np.argsort(fan_in)[-5:].tolist())
    hub_idx = np.nonzero(np.isin(cm, list(top)))[0]
    # keep the oracle's work bounded: skip moves that touch the giant classes in the sample
    small = (oc["n_methods"][s.method_class[cm]] < 300) & (oc["n_methods"][ct] < 300)
    idx = np.union1d(rng.choice(np.nonzero(small)[0], 3000, replace=False), hub_idx[:200])
    ro = O.score(s, cm[idx], ct[idx])
    assert_fields_equal(rr[idx], ro, MOVE_FIELDS, "large50k REFERENCED sample")
    g.free()


ALL_RULE_SETS = RULE_SETS + [(mm.CBO | mm.RFC, mm.PARETO), (mm.LCOM_HS, mm.PARETO), (mm.LCOM_HS, mm.PAPER_LCOM),
                             (mm.CBO | mm.LCOM_PQ, mm.PAPER_CBO), (mm.RFC, mm.PARETO)]


def test_keep_only_is_the_filter(ctx):
    """Kept records (the pass that stops at the first settled rejection) equal the
    kept rows of the full pass, for every rule and mask, on systems with light and
    heavy caller lists."""
    systems = [("plain120", synth.plain(120, seed=5)), ("stress", synth.stress(seed=6, n_classes=180))]
    rng = np.random.default_rng(17)
    systems += [(f"tiny{k}", synth.tiny(rng)) for k in range(40)]
    say("keep_only")
    for name, s in systems:
        if s.n_classes < 2:
            continue
        g = load(ctx, s)
        modes = [mm.REFERENCED] + ([mm.ALL] if s.n_methods * (s.n_classes - 1) < 200000 else [])
        for mode in modes:
            for mask, rule in ALL_RULE_SETS:
                full = mm.score_moves(g, mode, metric_mask=mask, rule=rule)
                kept = mm.score_moves(g, mode, metric_mask=mask, rule=rule, keep_only=True)
                assert kept.tobytes() == full[full["keep"] == 1].tobytes(), (name, mode, mask, rule)
                assert mm.score_moves_count(g, mode, metric_mask=mask, rule=rule, keep_only=True) == len(kept)
        g.free()


def test_keep_only_into_device_buffer(ctx):
    """keep_only scoring straight into a device buffer gives the host pass's kept
    records in candidate order: through the short kept list (few kept), through
    the scan of the keep flags (PAPER_CBO over ALL keeps 2,209 > 2,048 moves on
    this system), and after a buffer one record too small was refused, into a
    larger one from the kept results."""
    import torch
    s = synth.plain(200)
    say("keep_only into a device buffer")
    g = load(ctx, s)
    size = mm.MOVE_SCORE.itemsize
    seen_long = seen_short = False
    for mode in (mm.REFERENCED, mm.ALL):
        for mask, rule in ALL_RULE_SETS:
            want = mm.score_moves(g, mode, metric_mask=mask, rule=rule, keep_only=True)
            n = len(want)
            seen_long |= n > 2048
            seen_short |= 0 < n <= 2048
            cap = n + 3
            buf = torch.zeros(cap * size, dtype=torch.uint8, device="cuda:0")
            got_n = mm.score_moves_device(g, buf.data_ptr(), cap, mode, metric_mask=mask, rule=rule, keep_only=True)
            torch.cuda.synchronize()
            assert got_n == n, (mode, mask, rule)
            assert buf[:n * size].cpu().numpy().tobytes() == want.tobytes(), (mode, mask, rule)
            if n > 1:
                small = torch.zeros((n - 1) * size, dtype=torch.uint8, device="cuda:0")
                with pytest.raises(mm.MMError):
                    mm.score_moves_device(g, small.data_ptr(), n - 1, mode, metric_mask=mask, rule=rule,
                                          keep_only=True)
                buf.zero_()
                got_n = mm.score_moves_device(g, buf.data_ptr(), cap, mode, metric_mask=mask, rule=rule,
                                              keep_only=True)
                torch.cuda.synchronize()
                assert got_n == n
                assert buf[:n * size].cpu().numpy().tobytes() == want.tobytes(), ("after refusal", mode, mask, rule)
    assert seen_long and seen_short
    g.free()


def test_apply_move_matches_prediction(ctx):
    s = synth.plain(150, seed=8)
    say("apply_move")
    g = load(ctx, s)
    c0, m0 = mm.compute_metrics(g)
    cm, ct = O.candidates(s, O.REFERENCED)
    rng = np.random.default_rng(4)
    cur = s.copy()
    for k in rng.choice(len(cm), 25, replace=False):
        m, T = int(cm[k]), int(ct[k])
        if cur.method_class[m] == T:
            continue
        S = int(cur.method_class[m])
        pred = mm.score_moves(g, mm.EXPLICIT, [m], [T], mm.CBO | mm.LCOM_PQ | mm.RFC)[0]
        before, _ = mm.compute_metrics(g)
        mm.apply_move(g, m, T)
        cur.method_class[m] = T
        after, am = mm.compute_metrics(g)
        oc, om = O.metrics(cur)
        assert_fields_equal(after, oc, CLASS_FIELDS, "after move")
        assert_fields_equal(am, om, METHOD_FIELDS, "after move")
        assert pred["d_cbo_src"] == after["cbo"][S] - before["cbo"][S]
        assert pred["d_cbo_dst"] == after["cbo"][T] - before["cbo"][T]
        assert pred["d_rfc_src"] == after["rfc"][S] - before["rfc"][S]
        assert pred["d_rfc_dst"] == after["rfc"][T] - before["rfc"][T]
        lc = after["lcom_p"] - after["lcom_q"]
        lb = before["lcom_p"] - before["lcom_q"]
        assert pred["d_lcom_src"] == lc[S] - lb[S] and pred["d_lcom_dst"] == lc[T] - lb[T]
        # the reverse move restores everything
        mm.apply_move(g, m, S)
        back, bm = mm.compute_metrics(g)
        assert back.tobytes() == before.tobytes()
        mm.apply_move(g, m, T)
    info = mm.system_info(g)
    assert info["version"] > 0
    g.free()


def test_apply_edit_equals_reload(ctx):
    s = synth.plain(150, seed=12)
    say("apply_edit")
    g = load(ctx, s)
    rng = np.random.default_rng(6)
    cur = s
    for step in range(4):
        ed = synth.edit_batch(cur, rng, k=int(rng.integers(1, 60)))
        mm.apply_edit(g, *ed)
        cur = synth.apply_edit_arrays(cur, *ed)
        check_metrics(g, cur, f"edit step {step}")
        fresh = load(ctx, cur)
        a = mm.score_moves(g, mm.REFERENCED, metric_mask=15)
        b = mm.score_moves(fresh, mm.REFERENCED, metric_mask=15)
        assert a.tobytes() == b.tobytes()
        cm, ct = O.candidates(cur, O.REFERENCED)
        assert_fields_equal(a, O.score(cur, cm, ct, 15), MOVE_FIELDS, f"edit step {step}")
        fresh.free()
    g.free()


def test_deterministic(ctx):
    s = synth.stress(seed=3)
    say("determinism")
    g = load(ctx, s)
    a = mm.score_moves(g, mm.REFERENCED, metric_mask=15)
    b = mm.score_moves(g, mm.REFERENCED, metric_mask=15)
    assert a.tobytes() == b.tobytes()
    c1, m1 = mm.compute_metrics(g)
    c2, m2 = mm.compute_metrics(g)
    assert c1.tobytes() == c2.tobytes() and m1.tobytes() == m2.tobytes()
    g.free()


def test_degenerate_systems(ctx):
    say("degenerate")
    # one class: no candidates at all
    s = synth.from_lists(1, [0, 0], [0], [[0], [0]], [[1], []])
    g = load(ctx, s)
    check_metrics(g, s, "one class")
    assert len(mm.score_moves(g, mm.ALL)) == 0 and len(mm.score_moves(g, mm.REFERENCED)) == 0
    g.free()
    # no attributes, no calls, empty classes
    s = synth.from_lists(4, [0, 0, 3], [], [[], [], []], [[], [], []])
    g = load(ctx, s)
    check_metrics(g, s, "bare")
    cm, ct = O.candidates(s, O.ALL)
    assert_fields_equal(mm.score_moves(g, mm.ALL, metric_mask=15), O.score(s, cm, ct, 15), MOVE_FIELDS, "bare")
    g.free()
    # no methods at all
    s = synth.from_lists(3, [], [0, 2], [], [])
    g = load(ctx, s)
    gc, gm = mm.compute_metrics(g)
    assert len(gm) == 0 and gc["n_attrs"].tolist() == [1, 0, 1]
    g.free()
    # self-calls and repeated ids
    s = synth.from_lists(2, [0, 0, 1], [0, 1], [[0, 0, 1], [0], [1, 1]], [[0, 0, 2], [1, 0], [2, 0, 0]])
    g = load(ctx, s)
    check_metrics(g, s, "self calls")
    cm, ct = O.candidates(s, O.ALL)
    for mask, rule in RULE_SETS:
        assert_fields_equal(mm.score_moves(g, mm.ALL, metric_mask=mask, rule=rule), O.score(s, cm, ct, mask, rule),
                            MOVE_FIELDS, "self calls")
    g.free()


def test_errors(ctx):
    say("errors")
    s = synth.plain(30, seed=2)
    g = load(ctx, s)
    m = 0
    S = int(s.method_class[m])
    with pytest.raises(mm.MMError) as e:
        mm.score_moves(g, mm.EXPLICIT, [m], [S])
    assert e.value.code == mm.MM_EINVAL
    for bad in ([s.n_methods], [0]), ([0], [s.n_classes]), ([-1], [0]):
        with pytest.raises(mm.MMError) as e:
            mm.score_moves(g, mm.EXPLICIT, *bad)
        assert e.value.code == mm.MM_EINVAL
    with pytest.raises(mm.MMError):
        mm.score_moves(g, mm.REFERENCED, metric_mask=16)
    with pytest.raises(mm.MMError):
        mm.score_moves(g, mm.REFERENCED, rule=3)
    with pytest.raises(mm.MMError):
        mm.score_moves(g, mm.REFERENCED, metric_mask=mm.CBO, rule=mm.PAPER_LCOM)
    with pytest.raises(mm.MMError):
        mm.apply_move(g, m, S)
    with pytest.raises(mm.MMError):
        mm.apply_move(g, s.n_methods, 0)
    # capacity too small
    import ctypes
    n = mm.score_moves_count(g, mm.REFERENCED)
    out = np.zeros(max(n - 1, 1), mm.MOVE_SCORE)
    n_out = ctypes.c_int64()
    rc = mm.lib().mm_score_moves(g.handle, mm.REFERENCED, None, None, 0, 3, 0, 0, out.ctypes.data, n - 1,
                                 ctypes.byref(n_out))
    assert rc == mm.MM_ERANGE and n_out.value == n
    g.free()
    # malformed systems
    bad = s.copy()
    bad.acc_off = bad.acc_off.copy()
    bad.acc_off[3] = bad.acc_off[2] - 1
    with pytest.raises(mm.MMError) as e:
        load(ctx, bad)
    assert e.value.code == mm.MM_EINVAL
    bad = s.copy()
    bad.call_idx = bad.call_idx.copy()
    bad.call_idx[0] = s.n_methods
    with pytest.raises(mm.MMError):
        load(ctx, bad)
    bad = s.copy()
    bad.method_class = bad.method_class.copy()
    bad.method_class[0] = s.n_classes
    with pytest.raises(mm.MMError):
        load(ctx, bad)
    # a tiny memory budget refuses the upload
    small = mm.context_create(0, mem_budget=4096)
    with pytest.raises(mm.MMError) as e:
        load(small, s)
    assert e.value.code == mm.MM_ENOMEM
    small.close()


def _part_systems():
    rng = np.random.default_rng(77)
    parts = [synth.plain(60, seed=21), synth.stress(seed=9, n_classes=120), synth.medium(300, seed=4)]
    parts += [synth.tiny(rng, max_classes=5, max_methods=6) for _ in range(4)]
    parts.append(synth.from_lists(2, [0, 1], [], [[], []], [[1], [0]]))
    return parts


def test_batch_equals_parts(ctx):
    say("batch")
    parts = _part_systems()
    b = mm.load_batch(ctx, parts)
    off = mm.system_parts(b)
    assert len(off["classes"]) == len(parts) + 1
    bc, bm = mm.compute_metrics(b)
    rec = mm.score_moves(b, mm.REFERENCED, metric_mask=15)
    per = mm.split_records(rec, off)
    for i, s in enumerate(parts):
        oc, om = O.metrics(s)
        c0, c1 = off["classes"][i], off["classes"][i + 1]
        m0, m1 = off["methods"][i], off["methods"][i + 1]
        assert_fields_equal(bc[c0:c1], oc, CLASS_FIELDS, f"batch part {i}")
        assert_fields_equal(bm[m0:m1], om, METHOD_FIELDS, f"batch part {i}")
        cm, ct = O.candidates(s, O.REFERENCED)
        assert_fields_equal(per[i], O.score(s, cm, ct, 15), MOVE_FIELDS, f"batch part {i}")
        alone = load(ctx, s)
        assert mm.score_moves(alone, mm.REFERENCED, metric_mask=15).tobytes() == per[i].tobytes()
        alone.free()
    with pytest.raises(mm.MMError) as e:
        mm.score_moves(b, mm.ALL)
    assert e.value.code == mm.MM_EINVAL
    with pytest.raises(mm.MMError):  # a move into another part's class
        mm.score_moves(b, mm.EXPLICIT, [int(off["methods"][1])], [0])
    # moves and edits that would make a reference cross parts are refused, and
    # leave the batch as it was
    m1 = int(off["methods"][1])  # first method of part 1
    for bad in (lambda: mm.apply_move(b, m1, 0),
                lambda: mm.apply_edit(b, [m1], [0], [0, 0], [], [0, 0], []),
                lambda: mm.apply_edit(b, [m1], None, [0, 1], [0], [0, 0], []),
                lambda: mm.apply_edit(b, [m1], None, [0, 0], [], [0, 1], [0])):
        with pytest.raises(mm.MMError) as e:
            bad()
        assert e.value.code == mm.MM_EINVAL
    assert mm.score_moves(b, mm.REFERENCED, metric_mask=15).tobytes() == rec.tobytes()
    b.free()


TUNINGS = [{"caller_light": 0, "heavy_chunk": 1, "delta_chunk": 0, "delta_grid": 0},
           {"caller_light": 1000, "heavy_chunk": 64, "delta_chunk": 0, "delta_grid": 0},
           {"caller_light": 4, "heavy_chunk": 256, "delta_chunk": 7, "delta_grid": 3},
           {"caller_light": 8, "heavy_chunk": 64, "delta_chunk": 1024, "delta_grid": 2048},
           {"caller_light": 32, "heavy_chunk": 256, "delta_chunk": 0, "delta_grid": 0, "fill_chunk": 64,
            "fill_group": 1},
           {"caller_light": 32, "heavy_chunk": 256, "delta_chunk": 0, "delta_grid": 0, "fill_chunk": 2048,
            "fill_group": 100}]


def test_schedules_give_identical_results(ctx):
    say("schedules")
    s = synth.stress(seed=5)
    g = load(ctx, s)
    ref = {}
    mm.context_set_tuning(ctx, None)
    metrics = mm.compute_metrics(g)
    for mode, mask, rule in [(mm.REFERENCED, 15, mm.PARETO), (mm.ALL, 3, mm.PARETO), (mm.REFERENCED, 1, mm.PAPER_CBO)]:
        mm.context_set_tuning(ctx, None)
        ref[mode, mask, rule] = mm.score_moves(g, mode, metric_mask=mask, rule=rule)
        for t in TUNINGS:
            mm.context_set_tuning(ctx, t)
            mm.compute_metrics_device(g, None, None)  # a full recompute with this schedule's fill items
            gc, gm = mm.compute_metrics(g)
            assert gc.tobytes() == metrics[0].tobytes() and gm.tobytes() == metrics[1].tobytes(), t
            got = mm.score_moves(g, mode, metric_mask=mask, rule=rule)
            assert got.tobytes() == ref[mode, mask, rule].tobytes(), t
            kept = mm.score_moves(g, mode, metric_mask=mask, rule=rule, keep_only=True)
            full = ref[mode, mask, rule]
            assert kept.tobytes() == full[full["keep"] == 1].tobytes(), t
    mm.context_set_tuning(ctx, None)
    best = mm.autotune(g, mm.REFERENCED, metric_mask=15, repeats=1)
    assert best["heavy_chunk"] >= 1 and mm.context_get_tuning(ctx) == best
    assert mm.score_moves(g, mm.REFERENCED, metric_mask=15).tobytes() == ref[mm.REFERENCED, 15, mm.PARETO].tobytes()
    mm.context_set_tuning(ctx, None)
    g.free()


def _check_affected(g, s, m, t, rec, exact, what):
    xs, d = mm.move_affected(g, int(m), int(t))
    assert len(xs) == rec["n_caller_cls"], what
    assert int((d > 0).sum()) == rec["n_caller_worse"] and int((d < 0).sum()) == rec["n_caller_better"], what
    assert np.all(np.diff(xs) > 0) and set(d.tolist()) <= {-1, 0, 1}, what
    if exact:
        ox, od = O.affected(s, int(m), int(t))
        assert xs.tolist() == ox.tolist() and d.tolist() == od.tolist(), what


def test_move_affected(ctx):
    """Per-caller-class CBO changes: equal to the oracle's re-evaluated CBO on
    fixtures, tiny systems and the stress hubs; on the 50,000-class system the
    hubs' lists agree with the oracle's caller counts and two are checked in full."""
    say("move_affected fixtures")
    fx = load_fixture("f3_caller_class.json")
    for variant in (None, "variant_b"):
        s = fixture_system(fx, variant)
        want = (fx if variant is None else fx[variant])["affected"]
        g = load(ctx, s)
        xs, d = mm.move_affected(g, want["method"], want["dst"])
        assert [[int(a), int(b)] for a, b in zip(xs, d)] == want["classes"]
        g.free()
    fx = load_fixture("f7_caller_better.json")
    g = load(ctx, fixture_system(fx))
    for want in fx["affected"]:
        xs, d = mm.move_affected(g, want["method"], want["dst"])
        assert [[int(a), int(b)] for a, b in zip(xs, d)] == want["classes"]
    g.free()
    say("move_affected tiny")
    rng = np.random.default_rng(91)
    for _ in range(60):
        s = synth.tiny(rng)
        if s.n_classes < 2 or s.n_methods == 0:
            continue
        g = load(ctx, s)
        cm, ct = O.candidates(s, O.ALL)
        pick = rng.choice(len(cm), size=min(8, len(cm)), replace=False)
        ro = O.score(s, cm[pick], ct[pick], O.CBO)
        for r in ro:
            _check_affected(g, s, r["method"], r["dst"], r, True, "tiny")
        g.free()
    say("move_affected stress hubs")
    s = synth.stress()
    g = load(ctx, s)
    counts = np.bincount(s.call_idx, minlength=s.n_methods)
    hubs = np.argsort(counts)[-3:]
    for h in hubs:
        ts = [t for t in rng.choice(s.n_classes, 4, replace=False) if t != s.method_class[h]]
        ro = O.score(s, np.full(len(ts), h), np.array(ts), O.CBO)
        for r in ro:
            _check_affected(g, s, r["method"], r["dst"], r, True, f"stress hub {h}")
    # errors: own class, out of range, capacity too small
    h = int(hubs[-1])
    with pytest.raises(mm.MMError) as e:
        mm.move_affected(g, h, int(s.method_class[h]))
    assert e.value.code == mm.MM_EINVAL
    with pytest.raises(mm.MMError) as e:
        mm.move_affected(g, s.n_methods, 0)
    assert e.value.code == mm.MM_EINVAL
    n = ctypes_count(g, h, (int(s.method_class[h]) + 1) % s.n_classes)
    assert n > 1
    buf = np.zeros(1, np.int32)
    nn = ctypes.c_int64(0)
    rc = mm.lib().mm_move_affected(g.handle, h, (int(s.method_class[h]) + 1) % s.n_classes, buf.ctypes.data,
                                   buf.ctypes.data, 1, ctypes.byref(nn))
    assert rc == mm.MM_ERANGE and nn.value == n
    g.free()
    say("move_affected large50k hubs")
    s = synth.large(50000)
    g = load(ctx, s)
    fan_in = np.bincount(s.call_idx, minlength=s.n_methods)
    top = np.argsort(fan_in)[-4:]
    cm = np.repeat(top, 3)
    ct = np.array([(int(s.method_class[m]) + 1 + 7919 * j) % s.n_classes for j, m in enumerate(cm)], np.int32)
    ct = np.where(ct == s.method_class[cm], (ct + 1) % s.n_classes, ct)
    ro = O.score(s, cm, ct, O.CBO)
    for j, r in enumerate(ro):
        _check_affected(g, s, r["method"], r["dst"], r, j < 2, f"large hub {r['method']}")
    g.free()


def ctypes_count(g, m, t):
    n = ctypes.c_int64(0)
    assert mm.lib().mm_move_affected(g.handle, m, t, None, None, 0, ctypes.byref(n)) == mm.MM_OK
    return n.value

"""Incremental recompute after moves: after every batch of moves the metrics
recomputed from the touched segments only equal, bit for bit, those of the same
system loaded afresh (full recompute) and, on small systems, the oracle's; the
scores of every REFERENCED candidate (which read the grouped counts, caller maps
and loss flags the recompute rebuilt) equal the fresh system's. Covers moves into
and out of giant classes, of hub methods with thousands of callers, into empty
classes and classes without attributes, tables and member rows that outgrow their
place, and the same sequence with the incremental path switched off."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-incr]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mm.context_create(0)
    yield c
    c.close()


def _fresh(ctx, cur):
    g = mm.load_system(ctx, cur)
    out = mm.compute_metrics(g)
    return g, out


def _compare(ctx, g, cur, what, score=True, oracle=False, mask=mm.CBO | mm.LCOM_PQ | mm.LCOM_HS | mm.RFC):
    gc, gm = mm.compute_metrics(g)
    f, (fc, fm) = _fresh(ctx, cur)
    assert_fields_equal(gc, fc, CLASS_FIELDS, what + " classes")
    assert_fields_equal(gm, fm, METHOD_FIELDS, what + " methods")
    if oracle:
        oc, om = O.metrics(cur)
        assert_fields_equal(gc, oc, CLASS_FIELDS, what + " classes vs oracle")
        assert_fields_equal(gm, om, METHOD_FIELDS, what + " methods vs oracle")
    if score:
        r = mm.score_moves(g, mm.REFERENCED, metric_mask=mask, keep_only=False)
        q = mm.score_moves(f, mm.REFERENCED, metric_mask=mask, keep_only=False)
        assert len(r) == len(q), (what, len(r), len(q))
        assert_fields_equal(r, q, MOVE_FIELDS, what + " REFERENCED records")
    f.free()


def _callers(s):
    return np.bincount(s.call_idx, minlength=s.n_methods)


def _pick_moves(s, cur, rng, k, hubs=0, into=None):
    """k random moves to a referenced class (or `into`), plus `hubs` moves of the
    most-called methods."""
    moves = []
    order = np.argsort(-_callers(s))[:hubs]
    for m in order:
        m = int(m)
        T = int((cur.method_class[m] + 1 + rng.integers(0, s.n_classes - 1)) % s.n_classes)
        moves.append((m, T))
    for _ in range(k):
        m = int(rng.integers(0, s.n_methods))
        if into is not None:
            T = into
        else:
            row = s.call_idx[s.call_off[m]:s.call_off[m + 1]]
            refs = cur.method_class[row] if len(row) else np.array([], np.int32)
            T = int(refs[rng.integers(0, len(refs))]) if len(refs) else int(rng.integers(0, s.n_classes))
        if T == cur.method_class[m]:
            continue
        moves.append((m, T))
    return moves


def _apply(g, cur, moves):
    for m, T in moves:
        if cur.method_class[m] == T:
            continue
        mm.apply_move(g, m, T)
        cur.method_class[m] = T


@pytest.mark.parametrize("name", ["stress", "plain200"])
def test_small_systems_every_batch(ctx, name):
    s = synth.stress() if name == "stress" else synth.plain(200)
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(17)
    for step in range(12):
        moves = _pick_moves(s, cur, rng, k=int(rng.integers(1, 6)), hubs=1 if step % 4 == 0 else 0)
        _apply(g, cur, moves)
        _compare(ctx, g, cur, f"{name} step {step}", oracle=True)
    g.free()


def test_growth_and_empty_classes(ctx):
    """Sixty methods moved one by one into a class of two (its member row and its
    W and CNT tables outgrow their place several times), a class emptied, and
    moves into an empty class and into a class without attributes."""
    s = synth.plain(120, seed=23)
    mc = np.asarray(s.method_class)
    sizes = np.bincount(mc, minlength=s.n_classes)
    target = int(np.nonzero(sizes == 2)[0][0]) if (sizes == 2).any() else int(np.argmin(np.where(sizes > 0, sizes, 99)))
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(5)
    movers = [int(x) for x in rng.choice(np.nonzero(mc != target)[0], 60, replace=False)]
    for i, m in enumerate(movers):
        _apply(g, cur, [(m, target)])
        if i % 15 == 14:
            _compare(ctx, g, cur, f"growth {i + 1}", oracle=True)
    # empty a class, then move one method into it, and one into a class without attributes
    victim = int(np.argmax(np.bincount(cur.method_class, minlength=s.n_classes) * (np.arange(s.n_classes) != target)))
    members = np.nonzero(cur.method_class == victim)[0]
    _apply(g, cur, [(int(x), target) for x in members])
    _compare(ctx, g, cur, "emptied class", oracle=True)
    _apply(g, cur, [(movers[0], victim)])
    no_attr = np.nonzero(np.bincount(s.attr_class, minlength=s.n_classes) == 0)[0]
    if len(no_attr):
        _apply(g, cur, [(movers[1], int(no_attr[0]))])
    _compare(ctx, g, cur, "into empty / attribute-less classes", oracle=True)
    g.free()


def test_medium5k_batches(ctx):
    s = synth.medium(5000)
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(29)
    for step, k in enumerate((1, 8, 40)):
        _apply(g, cur, _pick_moves(s, cur, rng, k=k, hubs=1))
        _compare(ctx, g, cur, f"medium5k batch {step} ({k} moves + a hub)")
    # moved methods' entry classes: a few moves without a hub are patched in
    # place; more than 256 pending moves are gathered again in full
    for step, k in enumerate((3, 300)):
        _apply(g, cur, _pick_moves(s, cur, rng, k=k))
        _compare(ctx, g, cur, f"medium5k batch {3 + step} ({k} moves)")
    g.free()


def test_large50k_giants_and_hubs(ctx):
    """The 50,000-class system: moves of the most-called methods (thousands of
    caller classes), moves into and out of the classes of 500-2,000 methods, and
    random moves; metrics and the kept records of the benchmark's rule set
    against a fresh load after each batch, and the incremental recompute's device
    time against the full one."""
    s = synth.large(50000)
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(31)
    sizes = np.bincount(s.method_class, minlength=s.n_classes)
    giants = np.argsort(-sizes)[:4]
    batches = [
        _pick_moves(s, cur, rng, k=1),
        _pick_moves(s, cur, rng, k=0, hubs=2),
        [(int(m), int(giants[0])) for m in rng.integers(0, s.n_methods, 20)],
        [(int(m), int(giants[2])) for m in np.nonzero(s.method_class == giants[1])[0][:30]],
        _pick_moves(s, cur, rng, k=200),
    ]
    for i, moves in enumerate(batches):
        _apply(g, cur, moves)
        gc, gm = mm.compute_metrics(g)
        f, (fc, fm) = _fresh(ctx, cur)
        assert_fields_equal(gc, fc, CLASS_FIELDS, f"large50k batch {i}")
        assert_fields_equal(gm, fm, METHOD_FIELDS, f"large50k batch {i}")
        r = mm.score_moves(g, mm.REFERENCED, metric_mask=mm.CBO | mm.LCOM_PQ, keep_only=True)
        q = mm.score_moves(f, mm.REFERENCED, metric_mask=mm.CBO | mm.LCOM_PQ, keep_only=True)
        assert_fields_equal(r, q, MOVE_FIELDS, f"large50k batch {i} kept records")
        # every REFERENCED record under every metric (caller counts read the loss flags)
        r = mm.score_moves(g, mm.REFERENCED, metric_mask=15, keep_only=False)
        q = mm.score_moves(f, mm.REFERENCED, metric_mask=15, keep_only=False)
        assert len(r) == len(q)
        if r.tobytes() != q.tobytes():
            assert_fields_equal(r, q, MOVE_FIELDS, f"large50k batch {i} every record")
        del r, q
        f.free()
        say(f"large50k batch {i}: {len(moves)} moves equal a fresh load")
    # device time: one move's recompute against the full recompute
    import torch
    mm.context_set_timing(ctx, "*")
    m = int(rng.integers(0, s.n_methods))
    for _ in range(3):
        T = int((cur.method_class[m] + 1) % s.n_classes)
        _apply(g, cur, [(m, T)])
        mm.compute_metrics(g)
    torch.cuda.synchronize()
    inc = sum(v[1] for v in mm.context_timing(ctx, reset=True).values()) / 3
    mm.set_incremental(g, False)
    T = int((cur.method_class[m] + 1) % s.n_classes)
    _apply(g, cur, [(m, T)])
    t0 = time.perf_counter()
    mm.compute_metrics(g)
    host_full = time.perf_counter() - t0
    torch.cuda.synchronize()
    full = sum(v[1] for v in mm.context_timing(ctx, reset=True).values())
    mm.context_set_timing(ctx, None)
    say(f"large50k one move: incremental recompute {inc * 1000:.1f} us of kernels, "
        f"full recompute {full * 1000:.1f} us (+ host layout, call {host_full * 1000:.1f} ms)")
    _compare(ctx, g, cur, "large50k after the full path", score=False)
    g.free()


def test_same_sequence_with_incremental_off(ctx):
    s = synth.stress(seed=44)
    a = mm.load_system(ctx, s)
    b = mm.load_system(ctx, s)
    mm.set_incremental(b, False)
    cur = s.copy()
    rng = np.random.default_rng(2)
    for step in range(6):
        moves = _pick_moves(s, cur, rng, k=5, hubs=1)
        for m, T in moves:
            if cur.method_class[m] == T:
                continue
            mm.apply_move(a, m, T)
            mm.apply_move(b, m, T)
            cur.method_class[m] = T
        ac, am = mm.compute_metrics(a)
        bc, bm = mm.compute_metrics(b)
        assert ac.tobytes() == bc.tobytes() and am.tobytes() == bm.tobytes(), step
        ra = mm.score_moves(a, mm.REFERENCED, metric_mask=15, keep_only=False)
        rb = mm.score_moves(b, mm.REFERENCED, metric_mask=15, keep_only=False)
        assert ra.tobytes() == rb.tobytes(), step
    with pytest.raises(mm.MMError):
        mm._check(mm.lib().mm_system_set_incremental(a.handle, 2))
    a.free()
    b.free()


def _edit(g, cur, ed):
    mm.apply_edit(g, *ed)
    return synth.apply_edit_arrays(cur, *ed)


@pytest.mark.parametrize("name", ["stress", "plain200"])
def test_edits_small_systems(ctx, name):
    """Edits of 1-40 methods (rows replaced, a quarter of them changing owner),
    mixed with moves, each against a fresh load and the oracle."""
    s = synth.stress(seed=12) if name == "stress" else synth.plain(200, seed=13)
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(77)
    for step in range(10):
        cur = _edit(g, cur, synth.edit_batch(cur, rng, k=int(rng.integers(1, 41))))
        if step % 3 == 2:
            _apply(g, cur, _pick_moves(s, cur, rng, k=3, hubs=1))
        _compare(ctx, g, cur, f"{name} edit {step}", oracle=True)
    g.free()


def test_edits_that_reach_hubs_and_grow_rows(ctx):
    """Edits that add calls to the most-called method and to methods without
    callers (caller maps change kind or outgrow their region), rows that change
    length group, and an edit that empties a method's rows."""
    s = synth.plain(150, seed=19)
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    hub = int(np.argmax(np.bincount(s.call_idx, minlength=s.n_methods)))
    lonely = np.nonzero(np.bincount(s.call_idx, minlength=s.n_methods) == 0)[0]
    rng = np.random.default_rng(3)
    for step in range(4):
        k = 40
        methods = np.sort(rng.choice(s.n_methods, k, replace=False)).astype(np.int32)
        acc_rows, call_rows = [], []
        for i, m in enumerate(methods):
            extra = [hub] + ([int(lonely[(step * k + i) % len(lonely)])] if len(lonely) else [])
            n_more = int(rng.integers(0, 70)) if i % 5 == 0 else 0  # some rows jump length group
            call_rows.append(np.array(extra + list(rng.integers(0, s.n_methods, n_more)), np.int32))
            acc_rows.append(np.array([], np.int32) if i % 7 == 0 else
                            rng.integers(0, s.n_attrs, int(rng.integers(0, 6))).astype(np.int32))
        if step == 3:
            call_rows[0] = np.array([], np.int32)
            acc_rows[0] = np.array([], np.int32)
        owners = cur.method_class[methods].copy()
        owners[::4] = rng.integers(0, s.n_classes, len(owners[::4]))
        ao = synth._offsets(np.array([len(r) for r in acc_rows], np.int64))
        co = synth._offsets(np.array([len(r) for r in call_rows], np.int64))
        ed = (methods, owners.astype(np.int32), ao, np.concatenate(acc_rows).astype(np.int32), co,
              np.concatenate(call_rows).astype(np.int32))
        cur = _edit(g, cur, ed)
        _compare(ctx, g, cur, f"hub edit {step}", oracle=True)
    g.free()


@pytest.mark.parametrize("name,k", [("medium5k", 200), ("large50k", 500)])
def test_edits_full_size(ctx, name, k):
    """Edits of k methods on the 5,000- and 50,000-class systems against a fresh
    load: every metric, the kept records of the benchmark's rule set and every
    REFERENCED record; the device time of the recompute after the edit."""
    import torch
    s = synth.WORKLOADS[name]()
    g = mm.load_system(ctx, s)
    mm.compute_metrics(g)
    cur = s.copy()
    rng = np.random.default_rng(101)
    for step in range(2):
        ed = synth.edit_batch(cur, rng, k=k)
        t0 = time.perf_counter()
        mm.apply_edit(g, *ed)
        host_edit = time.perf_counter() - t0
        cur = synth.apply_edit_arrays(cur, *ed)
        mm.context_set_timing(ctx, "*")
        t0 = time.perf_counter()
        gc, gm = mm.compute_metrics(g)
        host_rec = time.perf_counter() - t0
        torch.cuda.synchronize()
        kern = sum(v[1] for v in mm.context_timing(ctx, reset=True).values())
        mm.context_set_timing(ctx, None)
        say(f"{name} edit of {k} methods: apply {host_edit * 1000:.2f} ms, recompute call "
            f"{host_rec * 1000:.2f} ms, {kern * 1000:.1f} us of kernels")
        f, (fc, fm) = _fresh(ctx, cur)
        assert_fields_equal(gc, fc, CLASS_FIELDS, f"{name} edit {step}")
        assert_fields_equal(gm, fm, METHOD_FIELDS, f"{name} edit {step}")
        r = mm.score_moves(g, mm.REFERENCED, metric_mask=15, keep_only=False)
        q = mm.score_moves(f, mm.REFERENCED, metric_mask=15, keep_only=False)
        assert len(r) == len(q)
        if r.tobytes() != q.tobytes():
            assert_fields_equal(r, q, MOVE_FIELDS, f"{name} edit {step} every record")
        del r, q
        f.free()
    g.free()


def test_edit_sequence_with_incremental_off(ctx):
    s = synth.stress(seed=45)
    a = mm.load_system(ctx, s)
    b = mm.load_system(ctx, s)
    mm.compute_metrics(a)
    mm.set_incremental(b, False)
    cur = s.copy()
    rng = np.random.default_rng(8)
    for step in range(5):
        ed = synth.edit_batch(cur, rng, k=int(rng.integers(5, 60)))
        mm.apply_edit(a, *ed)
        mm.apply_edit(b, *ed)
        cur = synth.apply_edit_arrays(cur, *ed)
        ac, am = mm.compute_metrics(a)
        bc, bm = mm.compute_metrics(b)
        assert ac.tobytes() == bc.tobytes() and am.tobytes() == bm.tobytes(), step
        ra = mm.score_moves(a, mm.REFERENCED, metric_mask=15, keep_only=False)
        rb = mm.score_moves(b, mm.REFERENCED, metric_mask=15, keep_only=False)
        assert ra.tobytes() == rb.tobytes(), step
    a.free()
    b.free()

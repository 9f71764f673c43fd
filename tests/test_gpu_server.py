"""The request server: every result is the same alone and in the mix, equals the
oracle on the edited system, and admission by memory and queue capacity work."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import MOVE_FIELDS, assert_fields_equal

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-server] {msg}", flush=True)
    sys.stdout.flush()


def _scenario(extra=()):
    """Per system: its initial arrays and a list of requests ("edit", edit) / ("score", None)."""
    systems = [synth.plain(60, seed=31), synth.plain(90, seed=32), synth.stress(seed=33, n_classes=140),
               synth.medium(400, seed=34), synth.plain(40, seed=35), *extra]
    rng = np.random.default_rng(8)
    plans = []
    for s in systems:
        cur, reqs = s, []
        for step in range(4):
            ed = synth.edit_batch(cur, rng, k=int(rng.integers(1, 25)))
            reqs.append(("edit", ed))
            cur = synth.apply_edit_arrays(cur, *ed)
            if step % 2 == 1:
                reqs.append(("score", None))
        plans.append((s, reqs, cur))
    return plans


def _run(server, plans, order):
    """Submit LOAD then the requests of the systems listed in `order` (interleaved
    round-robin), return {(system, index): records}."""
    tickets = {}
    for i in order:
        tickets[(i, -1)] = server.load(i, plans[i][0])
    longest = max(len(plans[i][1]) for i in order)
    for j in range(longest):
        for i in order:
            reqs = plans[i][1]
            if j >= len(reqs):
                continue
            kind, ed = reqs[j]
            if kind == "edit":
                tickets[(i, j)] = server.edit(i, *ed, metric_mask=15, keep_only=False)
            else:
                tickets[(i, j)] = server.score(i, mm.REFERENCED, metric_mask=15, keep_only=False)
    out = {}
    for key, t in tickets.items():
        r = server.wait(t)
        assert r["status"] == mm.MM_OK, (key, r["error"])
        out[key] = r["records"]
    return out


def test_alone_equals_mix():
    plans = _scenario()
    say("mix: all systems on 4 slots")
    srv = mm.Server(n_slots=4)
    mix = _run(srv, plans, list(range(len(plans))))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(mix) and st["failed"] == 0
    for i in range(len(plans)):
        say(f"alone: system {i}")
        srv = mm.Server(n_slots=1)
        alone = _run(srv, plans, [i])
        srv.close()
        for key, rec in alone.items():
            assert rec.tobytes() == mix[key].tobytes(), key
    # the final full score of every system equals the oracle on the edited arrays
    for i, (s0, reqs, final) in enumerate(plans):
        last = max(j for j, (k, _) in enumerate(reqs) if k == "score")
        cm, ct = O.candidates(final, O.REFERENCED)
        if last == len(reqs) - 1:
            assert_fields_equal(mix[(i, last)], O.score(final, cm, ct, 15), MOVE_FIELDS, f"system {i} final")


def test_edit_result_is_the_edited_methods_candidates():
    s = synth.plain(70, seed=41)
    rng = np.random.default_rng(3)
    ed = synth.edit_batch(s, rng, k=12)
    after = synth.apply_edit_arrays(s, *ed)
    srv = mm.Server(n_slots=2)
    srv.wait(srv.load(7, s))
    r = srv.wait(srv.edit(7, *ed, metric_mask=15, keep_only=False))
    srv.close()
    cm, ct = O.candidates(after, O.REFERENCED)
    sel = np.isin(cm, ed[0])
    assert_fields_equal(r["records"], O.score(after, cm[sel], ct[sel], 15), MOVE_FIELDS, "edit result")


def test_admission_and_refusal():
    small = [synth.plain(50, seed=50 + i) for i in range(6)]
    # a budget that holds a few of these systems: later loads evict idle ones
    srv = mm.Server(n_slots=1)
    srv.wait(srv.load(0, small[0]))
    one = srv.stats()["device_bytes"]
    srv.close()
    srv = mm.Server(n_slots=2, mem_budget=int(4 * one))
    for i, s in enumerate(small):
        r = srv.wait(srv.load(i, s))
        assert r["status"] == mm.MM_OK, r["error"]
    st = srv.stats()
    assert st["evicted"] >= 2 and st["resident"] <= 4
    # an unknown system
    r = srv.wait(srv.score(99))
    assert r["status"] == mm.MM_ENOTFOUND
    # a system that can never fit
    r = srv.wait(srv.load(100, synth.medium(3000, seed=1)))
    assert r["status"] == mm.MM_ENOMEM
    srv.close()
    # a full queue refuses
    srv = mm.Server(n_slots=1, queue_capacity=2)
    refused = 0
    tickets = []
    for i in range(12):
        try:
            tickets.append(srv.load(i, small[i % 4]))
        except mm.MMError as e:
            assert e.code == mm.MM_EBUSY
            refused += 1
    for t in tickets:
        srv.wait(t)
    assert refused >= 1 and srv.stats()["refused"] == refused
    srv.close()


def test_reload_replaces_and_keeps_order():
    """A load of a resident id replaces it; requests after it see the new system,
    requests before it the old one; repeated loads of one id all finish."""
    a, b = synth.plain(60, seed=61), synth.plain(80, seed=62)
    srv = mm.Server(n_slots=3)
    t = [srv.load(5, a), srv.score(5, mm.REFERENCED, metric_mask=15, keep_only=False),
         srv.load(5, b), srv.score(5, mm.REFERENCED, metric_mask=15, keep_only=False),
         srv.load(5, b), srv.load(5, a), srv.load(5, b),
         srv.score(5, mm.REFERENCED, metric_mask=15, keep_only=False)]
    res = [srv.wait(x) for x in t]
    srv.drain()
    st = srv.stats()
    srv.close()
    assert all(r["status"] == mm.MM_OK for r in res), [r["error"] for r in res]
    assert st["resident"] == 1 and st["queued"] == 0
    for i, sysd in ((1, a), (3, b), (7, b)):
        cm, ct = O.candidates(sysd, O.REFERENCED)
        assert_fields_equal(res[i]["records"], O.score(sysd, cm, ct, 15), MOVE_FIELDS, f"score {i}")


def test_edits_under_memory_pressure():
    """With a budget barely above the resident structure, edits reclaim idle
    scratch and evict idle systems instead of failing; the results are those of
    an unconstrained server."""
    systems = [synth.plain(80, seed=70 + i) for i in range(5)]
    rng = np.random.default_rng(12)
    stream, cur = [], list(systems)
    for _ in range(30):
        j = int(rng.integers(0, len(systems)))
        ed = synth.edit_batch(cur[j], rng, k=int(rng.integers(1, 30)))
        cur[j] = synth.apply_edit_arrays(cur[j], *ed)
        stream.append((j, ed))

    def run(budget):
        srv = mm.Server(n_slots=2, mem_budget=budget)
        for j, s in enumerate(systems):
            assert srv.wait(srv.load(j, s))["status"] == mm.MM_OK
        resident = srv.stats(reset=True)["device_bytes"]  # the peak counts from here
        out = []
        for j, ed in stream:
            # an evicted system is reloaded by the server from its kept state
            r = srv.wait(srv.edit(j, *ed, metric_mask=15, keep_only=False))
            assert r["status"] == mm.MM_OK, r["error"]
            out.append(r["records"])
        st = srv.stats()
        srv.close()
        return out, resident, st

    free, resident, st0 = run(0)
    # room for every system plus part of one request's work memory: each edit
    # needs an idle system evicted first
    tight, _, st = run(int(resident + 0.5 * (st0["peak_bytes"] - resident)))
    say(f"pressure: evicted {st['evicted']}, reloaded {st['reloaded']}")
    assert st["evicted"] >= 1 and st["reloaded"] >= 1
    for i, (x, y) in enumerate(zip(free, tight)):
        assert x.tobytes() == y.tobytes(), i


def test_alone_equals_mix_under_budget():
    """Every request of every system submitted at once to four slots under a
    memory budget that holds only some of the systems: idle systems are evicted
    and reloaded from their kept state (edits included), and every result equals
    the same system's requests run alone on an unconstrained server."""
    # three systems of medium size, so that their structures alone outgrow a
    # budget that any one of them fits with its heaviest request
    plans = _scenario(extra=(synth.medium(350, seed=36), synth.medium(380, seed=37)))
    # the most memory any one system needs alone: its structure plus the scratch
    # of its heaviest request (every record of a full scoring)
    need = 0
    for i in range(len(plans)):
        srv = mm.Server(n_slots=1)
        _run(srv, plans, [i])
        need = max(need, srv.stats()["peak_bytes"])
        srv.close()
    srv = mm.Server(n_slots=1)
    for i in range(len(plans)):
        assert srv.wait(srv.load(i, plans[i][0]))["status"] == mm.MM_OK
    resident = srv.stats()["device_bytes"]
    srv.close()
    budget = int(need * 1.15)
    say(f"mix under a budget of {budget} bytes (one system alone needs at most {need}, all resident {resident})")
    assert resident > budget, "the scenario must not fit the budget all at once"
    srv = mm.Server(n_slots=4, mem_budget=budget)
    mix = _run(srv, plans, list(range(len(plans))))
    st = srv.stats()
    srv.close()
    say(f"  evicted {st['evicted']}, reloaded {st['reloaded']}, failed {st['failed']}")
    assert st["failed"] == 0 and st["evicted"] >= 1 and st["reloaded"] >= 1
    for i in range(len(plans)):
        srv = mm.Server(n_slots=1)
        alone = _run(srv, plans, [i])
        srv.close()
        for key, rec in alone.items():
            assert rec.tobytes() == mix[key].tobytes(), key


def test_free_of_an_evicted_system():
    """FREE of a system the server evicted drops its kept state; a later request
    on that id is refused as unknown."""
    small = [synth.plain(50, seed=80 + i) for i in range(12)]
    # the budget holds one system with the scratch of a full scoring, and a few
    # systems' structure, not all twelve
    srv = mm.Server(n_slots=1)
    srv.wait(srv.load(0, small[1]))
    one = srv.stats()["device_bytes"]
    srv.wait(srv.score(0, mm.REFERENCED, metric_mask=15, keep_only=False))
    peak = srv.stats()["peak_bytes"]
    srv.close()
    srv = mm.Server(n_slots=1, mem_budget=int(max(2.5 * one, 1.25 * peak)))
    for i, s in enumerate(small):
        assert srv.wait(srv.load(i, s))["status"] == mm.MM_OK
    st = srv.stats()
    say(f"free of an evicted system: one system {one} bytes, scoring peak {peak}, evicted {st['evicted']}")
    assert st["evicted"] >= 2  # systems 0 and 1 (least recently used) at least
    assert srv.wait(srv.free(0))["status"] == mm.MM_OK  # system 0 was evicted first (least recently used)
    assert srv.wait(srv.score(0))["status"] == mm.MM_ENOTFOUND
    r = srv.wait(srv.score(1, mm.REFERENCED, metric_mask=15, keep_only=False))  # evicted too: reloaded
    assert r["status"] == mm.MM_OK
    cm, ct = O.candidates(small[1], O.REFERENCED)
    assert_fields_equal(r["records"], O.score(small[1], cm, ct, 15), MOVE_FIELDS, "reloaded system")
    srv.close()

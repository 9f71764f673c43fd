"""The served workload at full size: 64 resident systems of 1,000-50,000
classes (848,521 classes in all) and a stream of edit requests (1-500 changed
methods, log-uniform) submitted at once to a server of four slots, as the
saturated level of the benchmark does.

Each request's result is the kept moves among its edited methods' REFERENCED
candidates after the edit. It is checked
* against the same edit applied alone: a copy of every system is loaded outside
  the server, the edits are applied to it in submission order, and the kept
  records of the edited methods are taken from a REFERENCED pass over it;
* against the oracle for every request on a system of at most 3,000 classes.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import MOVE_FIELDS, assert_fields_equal

pytestmark = pytest.mark.gpu

N_REQUESTS = 96
ORACLE_MAX_CLASSES = 3000


def say(msg):
    print(f"[gpu-served-full] {msg}", flush=True)
    sys.stdout.flush()


def test_served_results_equal_alone_and_oracle():
    counts = synth.served_class_counts(64)
    systems = [synth.served_system(int(k), synth.BASE_SEED + 5000 + j) for j, k in enumerate(counts)]
    say(f"{len(systems)} systems, {sum(s.n_classes for s in systems)} classes")
    rng = np.random.default_rng(synth.BASE_SEED + 6001)
    reqs = []
    for _ in range(N_REQUESTS):
        j = int(rng.integers(0, len(systems)))
        k = int(round(math.exp(rng.uniform(0, math.log(500)))))
        reqs.append((j, synth.edit_batch(systems[j], rng, k=k)))

    srv = mm.Server(n_slots=4)
    for t in [srv.load(j, s) for j, s in enumerate(systems)]:
        r = srv.wait(t, timeout_ms=120_000)
        assert r["status"] == mm.MM_OK, r["error"]
    tickets = [srv.edit(j, *ed) for j, ed in reqs]
    results = [srv.wait(t, timeout_ms=120_000) for t in tickets]
    srv.close()
    assert all(r["status"] == mm.MM_OK for r in results), [r["error"] for r in results if r["status"]]
    say(f"{len(results)} requests served, {sum(len(r['records']) for r in results)} kept records")

    ctx = mm.context_create(0)
    alone = {}
    state = list(systems)
    n_oracle = 0
    try:
        for i, ((j, ed), res) in enumerate(zip(reqs, results)):
            if j not in alone:
                alone[j] = mm.load_system(ctx, systems[j])
            g = alone[j]
            mm.apply_edit(g, *ed)
            kept = mm.score_moves(g, mm.REFERENCED, keep_only=True)
            mine = kept[np.isin(kept["method"], ed[0])]
            assert mine.tobytes() == res["records"].tobytes(), f"request {i} on system {j}"
            if state[j].n_classes <= ORACLE_MAX_CLASSES:
                state[j] = synth.apply_edit_arrays(state[j], *ed)
                cm, ct = O.candidates(state[j], O.REFERENCED)
                sel = np.isin(cm, ed[0])
                ro = O.score(state[j], cm[sel], ct[sel])
                assert_fields_equal(res["records"], ro[ro["keep"] == 1], MOVE_FIELDS, f"request {i} oracle")
                n_oracle += 1
    finally:
        for g in alone.values():
            g.free()
        mm.context_destroy(ctx)
    say(f"every result equals the edit applied alone; {n_oracle} checked against the oracle")
    assert n_oracle >= 10

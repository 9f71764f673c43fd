"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* hand-derived fixtures (tests/golden/f*.json, each with its citation and its
  derivation);
* the #values column of Table I against the count of Sec. III-B;
* closed forms and special systems whose metric values follow directly from the
  definitions of Sec. II;
* the same metrics through a different route: boolean incidence matrices and
  numpy integer matrix products (the co-access matrix G_C = B_C B_C^T, the
  class-to-class use matrix, the response set);
* relabelling invariance (catches swapped or misindexed ids);
* brute force: every move on many tiny systems, scored against a full
  re-evaluation of every class of the moved system.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import synth
from tests.helpers import (CLASS_FIELDS, METHOD_FIELDS, MOVE_FIELDS, assert_fields_equal,
                           fixture_system, load_fixture)

FIXTURES = ["f1_small_two_classes.json", "f2_pareto_kept.json", "f3_caller_class.json",
            "f6_lcom_hs_rules.json", "f7_caller_better.json"]
# rule sets named in the fixtures' "keep" maps: (metric mask, rule)
RULES = {"pareto_cbo_lcom": (O.CBO | O.LCOM_PQ, O.PARETO),
         "paper_lcom": (O.LCOM_PQ, O.PAPER_LCOM),
         "paper_cbo": (O.CBO, O.PAPER_CBO),
         "pareto_cbo_lcom_rfc": (O.CBO | O.LCOM_PQ | O.RFC, O.PARETO),
         "paper_lcom_hs": (O.LCOM_HS, O.PAPER_LCOM),
         "paper_lcom_pq_hs": (O.LCOM_PQ | O.LCOM_HS, O.PAPER_LCOM),
         "pareto_hs": (O.LCOM_HS, O.PARETO),
         "pareto_cbo_hs": (O.CBO | O.LCOM_HS, O.PARETO),
         "pareto_cbo": (O.CBO, O.PARETO)}


def _expect(records, fields):
    return {f: np.array([r[f] for r in records]) for f in fields}


@pytest.mark.parametrize("name,variant", [(n, None) for n in FIXTURES] + [("f3_caller_class.json", "variant_b")])
def test_fixture_metrics(name, variant):
    fx = load_fixture(name)
    sys_ = fixture_system(fx, variant)
    src = fx if variant is None else fx[variant]
    cls, meth = O.metrics(sys_)
    assert_fields_equal(cls, _expect(src["classes"], CLASS_FIELDS), CLASS_FIELDS, name)
    if "methods" in src:
        assert_fields_equal(meth, _expect(src["methods"], METHOD_FIELDS), METHOD_FIELDS, name)


@pytest.mark.parametrize("name", FIXTURES)
def test_fixture_referenced_candidates(name):
    fx = load_fixture(name)
    cm, ct = O.candidates(fixture_system(fx), O.REFERENCED)
    assert [[int(a), int(b)] for a, b in zip(cm, ct)] == fx["referenced"]


@pytest.mark.parametrize("name,variant", [(n, None) for n in FIXTURES] + [("f3_caller_class.json", "variant_b")])
def test_fixture_moves(name, variant):
    fx = load_fixture(name)
    sys_ = fixture_system(fx, variant)
    moves = (fx if variant is None else fx[variant])["moves"]
    cm = [mv["method"] for mv in moves]
    ct = [mv["dst"] for mv in moves]
    fields = [f for f in MOVE_FIELDS if f != "keep"]
    for rule_name in moves[0]["keep"]:
        mask, rule = RULES[rule_name]
        out = O.score(sys_, cm, ct, mask, rule)
        assert_fields_equal(out, _expect(moves, fields), fields, f"{name} {rule_name}")
        assert out["keep"].tolist() == [mv["keep"][rule_name] for mv in moves], rule_name


def test_table1_value_counts():
    fx = load_fixture("table1_value_counts.json")
    for row in fx["rows"]:
        v = O.value_count(row["classes"], row["methods"]) / 1e6
        # printed with one decimal; JUnit is printed truncated (1.28 -> 1.2)
        assert abs(v - row["values_millions"]) < 0.1, row


def _rows(off, idx, i):
    return idx[off[i]:off[i + 1]]


def _incidence(s):
    """Boolean incidence matrices of a system (rows read as sets)."""
    nm, na, c = s.n_methods, s.n_attrs, s.n_classes
    Bacc = np.zeros((nm, na), np.int64)
    Bcall = np.zeros((nm, nm), np.int64)
    r = np.repeat(np.arange(nm), np.diff(s.acc_off))
    Bacc[r, s.acc_idx] = 1
    r = np.repeat(np.arange(nm), np.diff(s.call_off))
    Bcall[r, s.call_idx] = 1
    Own = np.zeros((nm, c), np.int64)
    Own[np.arange(nm), s.method_class] = 1
    Acls = np.zeros((na, c), np.int64)
    Acls[np.arange(na), s.attr_class] = 1
    return Bacc, Bcall, Own, Acls


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_matrix_product_route(seed):
    s = synth.plain(40, seed=seed)
    cls, meth = O.metrics(s)
    Bacc, Bcall, Own, Acls = _incidence(s)
    nm, c = s.n_methods, s.n_classes
    # fan-in / fan-out are column / row sums of the call matrix
    assert np.array_equal(meth["fan_out"], Bcall.sum(1))
    assert np.array_equal(meth["fan_in"], Bcall.sum(0))
    # class-to-class use counts: W = Own^T (Bcall Own + Bacc Acls)
    W = Own.T @ (Bcall @ Own + Bacc @ Acls)
    np.fill_diagonal(W, 0)
    assert np.array_equal(cls["cbo"], (W > 0).sum(1))
    # response set: Own^T (I + Bcall)
    R = Own.T @ (np.eye(nm, dtype=np.int64) + Bcall)
    assert np.array_equal(cls["rfc"], (R > 0).sum(1))
    rnz = np.zeros(nm, np.int64)
    for C in range(c):
        M = np.nonzero(s.method_class == C)[0]
        A = np.nonzero(s.attr_class == C)[0]
        B = Bacc[np.ix_(M, A)]
        G = B @ B.T  # co-access counts over C's attributes
        n = len(M)
        iu = np.triu_indices(n, 1)
        Q = int((G[iu] > 0).sum())
        assert cls["lcom_q"][C] == Q
        assert cls["lcom_p"][C] == n * (n - 1) // 2 - Q
        off = (G > 0).astype(np.int64)
        np.fill_diagonal(off, 0)
        rnz[M] = off.sum(1)
        U = int(B.sum())
        assert np.array_equal(meth["own_attr_uses"][M], B.sum(1))
        if n * len(A) == 0:
            assert (cls["hs_num"][C], cls["hs_den"][C]) == (0, 1)
        else:
            assert (cls["hs_num"][C], cls["hs_den"][C]) == (n * len(A) - U, n * len(A))
    assert np.array_equal(meth["own_coaccess_partners"], rnz)


def test_closed_forms_random():
    s = synth.plain(80, seed=7)
    cls, meth = O.metrics(s)
    n = cls["n_methods"].astype(np.int64)
    assert np.array_equal(cls["lcom_p"] + cls["lcom_q"], n * (n - 1) // 2)
    pairs = np.unique(np.stack([np.repeat(np.arange(s.n_methods), np.diff(s.call_off)), s.call_idx]), axis=1)
    assert meth["fan_in"].sum() == meth["fan_out"].sum() == pairs.shape[1]
    fo = np.bincount(s.method_class, weights=meth["fan_out"], minlength=s.n_classes)
    assert np.all(cls["rfc"] >= n) and np.all(cls["rfc"] <= n + fo)
    refs = np.bincount(s.method_class, weights=np.diff(s.call_off) + np.diff(s.acc_off), minlength=s.n_classes)
    assert np.all(cls["cbo"] <= np.minimum(s.n_classes - 1, refs))
    assert np.array_equal(cls["n_methods"], np.bincount(s.method_class, minlength=s.n_classes))
    assert np.array_equal(cls["n_attrs"], np.bincount(s.attr_class, minlength=s.n_classes))


@pytest.mark.parametrize("n", [1, 2, 5, 17])
def test_special_one_shared_attribute(n):
    # every method of class 0 uses the same attribute (twice, to exercise set reading)
    s = synth.from_lists(2, [0] * n + [1], [0, 1], [[0, 0]] * n + [[1]], [[]] * (n + 1))
    cls, meth = O.metrics(s)
    assert cls["lcom_q"][0] == n * (n - 1) // 2 and cls["lcom_p"][0] == 0
    assert cls["hs_num"][0] == 0 and cls["hs_den"][0] == n
    assert np.all(meth["own_coaccess_partners"][:n] == n - 1)


@pytest.mark.parametrize("n", [1, 3, 9])
def test_special_distinct_attributes(n):
    s = synth.from_lists(1, [0] * n, [0] * n, [[i] for i in range(n)], [[]] * n)
    cls, meth = O.metrics(s)
    assert cls["lcom_q"][0] == 0 and cls["lcom_p"][0] == n * (n - 1) // 2
    assert (cls["hs_num"][0], cls["hs_den"][0]) == (n * n - n, n * n)
    assert np.all(meth["own_coaccess_partners"] == 0)


def test_special_every_attribute_used():
    a = 4
    s = synth.from_lists(1, [0] * 3, [0] * a, [list(range(a))] * 3, [[]] * 3)
    cls, _ = O.metrics(s)
    assert cls["hs_num"][0] == 0 and cls["hs_den"][0] == 3 * a


def test_special_empty_and_attributeless_classes():
    # class 1 has no methods, class 2 has methods but no attributes
    s = synth.from_lists(3, [0, 2, 2], [0], [[0], [0], []], [[1], [0], []])
    cls, _ = O.metrics(s)
    assert cls["n_methods"].tolist() == [1, 0, 2]
    assert (cls["hs_num"][1], cls["hs_den"][1]) == (0, 1)
    assert (cls["hs_num"][2], cls["hs_den"][2]) == (0, 1)
    assert cls["lcom_p"][1] == cls["lcom_q"][1] == 0
    # class 2 uses class 0 (through the access and the call), class 0 uses class 2
    assert cls["cbo"].tolist() == [1, 0, 1]


def test_relabelling_invariance():
    s = synth.plain(30, seed=11)
    rng = np.random.default_rng(5)
    pc = rng.permutation(s.n_classes)  # old class -> new class
    pm = rng.permutation(s.n_methods)  # old method -> new method
    pa = rng.permutation(s.n_attrs)
    inv_m = np.argsort(pm)
    acc_rows = [pa[s.acc_idx[s.acc_off[o]:s.acc_off[o + 1]]] for o in inv_m]
    call_rows = [pm[s.call_idx[s.call_off[o]:s.call_off[o + 1]]] for o in inv_m]
    mc = np.empty(s.n_methods, np.int32)
    mc[pm] = pc[s.method_class]
    ac = np.empty(s.n_attrs, np.int32)
    ac[pa] = pc[s.attr_class]
    s2 = synth.from_lists(s.n_classes, mc, ac, acc_rows, call_rows)
    c1, m1 = O.metrics(s)
    c2, m2 = O.metrics(s2)
    for f in CLASS_FIELDS:
        assert np.array_equal(c2[f][pc], c1[f]), f
    for f in METHOD_FIELDS:
        assert np.array_equal(m2[f][pm], m1[f]), f
    cm, ct = O.candidates(s, O.REFERENCED)
    sel = np.arange(0, len(cm), 7)
    r1 = O.score(s, cm[sel], ct[sel])
    r2 = O.score(s2, pm[cm[sel]], pc[ct[sel]])
    for f in MOVE_FIELDS[3:]:
        assert np.array_equal(r1[f], r2[f]), f


def _lcom(c):
    return c["lcom_p"].astype(np.int64) - c["lcom_q"].astype(np.int64)


def test_bruteforce_tiny_all_moves():
    """Every move of many tiny systems against a full re-evaluation of every class."""
    rng = np.random.default_rng(2024)
    checked = 0
    for trial in range(300):
        s = synth.tiny(rng)
        if s.n_classes < 2:
            continue
        before, mb = O.metrics(s)
        cm, ct = O.candidates(s, O.ALL)
        assert len(cm) == s.n_methods * (s.n_classes - 1)
        recs = O.score(s, cm, ct, O.CBO | O.LCOM_PQ, O.PARETO)
        for r in recs:
            m, S, T = int(r["method"]), int(r["src"]), int(r["dst"])
            after, ma = O.metrics(O.moved(s, m, T))
            # fan-in and fan-out never change
            assert np.array_equal(ma["fan_in"], mb["fan_in"]) and np.array_equal(ma["fan_out"], mb["fan_out"])
            assert r["d_cbo_src"] == after["cbo"][S] - before["cbo"][S]
            assert r["d_cbo_dst"] == after["cbo"][T] - before["cbo"][T]
            assert r["d_rfc_src"] == after["rfc"][S] - before["rfc"][S]
            assert r["d_rfc_dst"] == after["rfc"][T] - before["rfc"][T]
            assert r["d_lcom_src"] == _lcom(after)[S] - _lcom(before)[S]
            assert r["d_lcom_dst"] == _lcom(after)[T] - _lcom(before)[T]
            assert (r["hs_num_src"], r["hs_den_src"]) == (after["hs_num"][S], after["hs_den"][S])
            assert (r["hs_num_dst"], r["hs_den_dst"]) == (after["hs_num"][T], after["hs_den"][T])
            callers = {int(s.method_class[y]) for y in range(s.n_methods)
                       if y != m and m in set(s.call_idx[s.call_off[y]:s.call_off[y + 1]].tolist())}
            callers -= {S, T}
            worse = better = 0
            for X in range(s.n_classes):
                if X in (S, T):
                    continue
                for f in CLASS_FIELDS:
                    if f == "cbo":
                        continue
                    assert after[f][X] == before[f][X], (f, X)
                d = int(after["cbo"][X]) - int(before["cbo"][X])
                if X not in callers:
                    assert d == 0
                worse += d > 0
                better += d < 0
            assert r["n_caller_cls"] == len(callers)
            assert (r["n_caller_worse"], r["n_caller_better"]) == (worse, better)
            checked += 1
    assert checked > 1000


def test_move_then_reverse_negates():
    s = synth.plain(40, seed=3)
    cm, ct = O.candidates(s, O.REFERENCED)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(cm), 40, replace=False):
        m, T = int(cm[k]), int(ct[k])
        S = int(s.method_class[m])
        fwd = O.score(s, [m], [T])[0]
        s2 = O.moved(s, m, T)
        back = O.score(s2, [m], [S])[0]
        assert back["d_cbo_src"] == -fwd["d_cbo_dst"] and back["d_cbo_dst"] == -fwd["d_cbo_src"]
        assert back["d_rfc_src"] == -fwd["d_rfc_dst"] and back["d_rfc_dst"] == -fwd["d_rfc_src"]
        assert back["d_lcom_src"] == -fwd["d_lcom_dst"] and back["d_lcom_dst"] == -fwd["d_lcom_src"]
        c0, _ = O.metrics(s)
        assert (back["hs_num_dst"], back["hs_den_dst"]) == (c0["hs_num"][S], c0["hs_den"][S])
        assert (back["hs_num_src"], back["hs_den_src"]) == (c0["hs_num"][T], c0["hs_den"][T])
        # moving back restores every metric
        c3, m3 = O.metrics(O.moved(s2, m, S))
        for f in CLASS_FIELDS:
            assert np.array_equal(c3[f], c0[f])


def test_rules_reject_bad_arguments():
    fx = load_fixture("f2_pareto_kept.json")
    s = fixture_system(fx)
    with pytest.raises(ValueError):
        O.score(s, [1], [0])  # destination is the current owner
    with pytest.raises(ValueError):
        O.score(s, [1], [1], O.CBO, O.PAPER_LCOM)  # LCOM rule without an LCOM metric
    with pytest.raises(ValueError):
        O.score(s, [1], [1], O.CBO, 7)


@pytest.mark.parametrize("variant", [None, "variant_b"])
def test_fixture_affected_caller_classes(variant):
    """Per-caller-class CBO change of the hand-derived caller-class fixture."""
    fx = load_fixture("f3_caller_class.json")
    s = fixture_system(fx, variant)
    want = (fx if variant is None else fx[variant])["affected"]
    xs, d = O.affected(s, want["method"], want["dst"])
    assert [[int(a), int(b)] for a, b in zip(xs, d)] == want["classes"]


def test_fixture_affected_caller_better_and_worse():
    """A caller class whose CBO falls and one whose CBO rises (hand fixture f7)."""
    fx = load_fixture("f7_caller_better.json")
    s = fixture_system(fx)
    for want in fx["affected"]:
        xs, d = O.affected(s, want["method"], want["dst"])
        assert [[int(a), int(b)] for a, b in zip(xs, d)] == want["classes"]


def test_keep_rules_cover_every_branch():
    """The hand fixtures hold, for every rule branch, a move whose keep bit that
    branch alone decides: an LCOM_HS fraction that falls in both classes (kept
    by the LCOM rule and by PARETO on LCOM_HS), one that rises in the
    destination while P - Q falls in both (rejected only through LCOM_HS), a
    move kept only because a caller class's CBO falls, and one rejected only
    because a caller class's CBO rises. Guards the fixture set itself."""
    f6 = load_fixture("f6_lcom_hs_rules.json")["moves"]
    f7 = load_fixture("f7_caller_better.json")["moves"]
    assert f6[0]["keep"]["paper_lcom_hs"] == 1 and f6[0]["keep"]["pareto_hs"] == 1
    assert f6[1]["keep"]["paper_lcom"] == 1 and f6[1]["keep"]["paper_lcom_pq_hs"] == 0
    assert f6[1]["keep"]["pareto_cbo_hs"] == 0 and f6[1]["d_cbo_src"] < 0
    assert f7[0]["d_cbo_src"] == f7[0]["d_cbo_dst"] == 0 and f7[0]["n_caller_better"] == 1
    assert f7[0]["keep"]["pareto_cbo"] == 1
    assert f7[1]["d_cbo_src"] < 0 and f7[1]["n_caller_worse"] == 1
    assert f7[1]["keep"]["pareto_cbo"] == 0 and f7[1]["keep"]["paper_cbo"] == 0


def test_affected_agrees_with_caller_summary():
    """The per-class list matches the summary counts of the scored record (two
    independent routes: re-evaluated CBO against the delta formulas)."""
    rng = np.random.default_rng(77)
    seen = 0
    for _ in range(120):
        s = synth.tiny(rng)
        if s.n_classes < 2 or s.n_methods == 0:
            continue
        cm, ct = O.candidates(s, O.ALL)
        pick = rng.choice(len(cm), size=min(6, len(cm)), replace=False)
        recs = O.score(s, cm[pick], ct[pick], O.CBO, O.PARETO)
        for r in recs:
            xs, d = O.affected(s, int(r["method"]), int(r["dst"]))
            assert np.all(np.diff(xs) > 0) and not np.isin([r["src"], r["dst"]], xs).any()
            assert set(d.tolist()) <= {-1, 0, 1}
            assert r["n_caller_cls"] == len(xs)
            assert r["n_caller_worse"] == int((d > 0).sum()) and r["n_caller_better"] == int((d < 0).sum())
            seen += len(xs)
    assert seen > 50


# ---- similarity (Sec. II-A) and similarity-driven candidates (Sec. III-A)

def test_fixture_similarity():
    fx = load_fixture("f4_similarity.json")
    s = fixture_system(fx)
    m1, m2, i, u = O.similarity_pairs(s)
    assert [list(map(int, r)) for r in zip(m1, m2, i, u)] == fx["pairs"]
    avg = O.similarity_average(s.n_methods, i, u, O.SIM_ABOVE_AVG)
    assert (avg.numerator, avg.denominator) == tuple(fx["average_all"])
    avg = O.similarity_average(s.n_methods, i, u, O.SIM_ABOVE_AVG_NZ)
    assert (avg.numerator, avg.denominator) == tuple(fx["average_nonzero"])
    assert O.similarity_kept(s.n_methods, i, u, O.SIM_ABOVE_AVG).astype(int).tolist() == fx["kept_all"]
    assert O.similarity_kept(s.n_methods, i, u, O.SIM_ABOVE_AVG_NZ).astype(int).tolist() == fx["kept_nonzero"]
    for mode, key in ((O.SIM_ABOVE_AVG, "candidates_all"), (O.SIM_ABOVE_AVG_NZ, "candidates_nonzero")):
        cm, ct = O.similar_candidates(s, mode)
        assert [[int(a), int(b)] for a, b in zip(cm, ct)] == fx[key]


def _property_matrix(s):
    B = np.zeros((s.n_methods, s.n_methods + s.n_attrs), bool)
    for y in range(s.n_methods):
        B[y, s.call_idx[s.call_off[y]:s.call_off[y + 1]]] = True
        B[y, s.n_methods + s.acc_idx[s.acc_off[y]:s.acc_off[y + 1]]] = True
    return B


def test_similarity_matches_scipy_jaccard():
    """Jaccard similarity of every pair equals 1 - scipy's Jaccard distance on the
    boolean property matrix (pairs with an empty union excluded: J = 0 there)."""
    from scipy.spatial.distance import pdist, squareform
    rng = np.random.default_rng(5)
    for trial in range(40):
        s = synth.tiny(rng)
        if s.n_methods < 2:
            continue
        B = _property_matrix(s)
        J = 1.0 - squareform(pdist(B, "jaccard"))
        inter_ref = B.astype(np.int64) @ B.T.astype(np.int64)
        deg = B.sum(1)
        m1, m2, i, u = O.similarity_pairs(s)
        want = [(a, b) for a in range(s.n_methods) for b in range(a + 1, s.n_methods) if inter_ref[a, b] > 0]
        assert list(zip(m1.tolist(), m2.tolist())) == want
        assert np.array_equal(i, inter_ref[m1, m2]) and np.array_equal(u, deg[m1] + deg[m2] - i)
        assert np.allclose(i / u, J[m1, m2], rtol=0, atol=1e-12)


def test_similarity_rows_partition_and_relabel():
    """Row ranges partition the pair list; permuting method ids permutes pairs."""
    s = synth.plain(30, seed=8)
    full = O.similarity_pairs(s)
    parts = [O.similarity_pairs(s, lo, hi) for lo, hi in ((0, 50), (50, 120), (120, s.n_methods))]
    for k in range(4):
        assert np.array_equal(full[k], np.concatenate([p[k] for p in parts]))
    perm = np.random.default_rng(1).permutation(s.n_methods)
    inv = np.argsort(perm)
    # method y of the permuted system is method perm[y] of the original
    rows_acc = [s.acc_idx[s.acc_off[perm[y]]:s.acc_off[perm[y] + 1]] for y in range(s.n_methods)]
    rows_call = [inv[s.call_idx[s.call_off[perm[y]]:s.call_off[perm[y] + 1]]] for y in range(s.n_methods)]
    sp = synth.from_lists(s.n_classes, s.method_class[perm], s.attr_class, rows_acc, rows_call)
    pm = O.similarity_pairs(sp)
    got = {(min(perm[a], perm[b]), max(perm[a], perm[b])): (i, u) for a, b, i, u in zip(*(x.tolist() for x in pm))}
    want = {(a, b): (i, u) for a, b, i, u in zip(*(x.tolist() for x in full))}
    assert got == want


def test_similar_candidates_are_referenced_or_partner_classes():
    """Every similarity-driven candidate moves a method of a high cross-class pair
    to its partner's class or to a class it references by a call."""
    s = synth.plain(25, seed=4)
    m1, m2, i, u = O.similarity_pairs(s)
    for mode in (O.SIM_ABOVE_AVG, O.SIM_ABOVE_AVG_NZ, O.SIM_NONZERO):
        keep = O.similarity_kept(s.n_methods, i, u, mode)
        cm, ct = O.similar_candidates(s, mode)
        order = np.lexsort((ct, cm))
        assert np.array_equal(order, np.arange(len(cm)))
        assert len(set(zip(cm.tolist(), ct.tolist()))) == len(cm)
        partner = {}
        for a, b in zip(m1[keep].tolist(), m2[keep].tolist()):
            partner.setdefault(a, set()).add(int(s.method_class[b]))
            partner.setdefault(b, set()).add(int(s.method_class[a]))
        for m, t in zip(cm.tolist(), ct.tolist()):
            called = {int(s.method_class[x]) for x in s.call_idx[s.call_off[m]:s.call_off[m + 1]]}
            assert t != s.method_class[m] and (t in partner[m] or t in called)
        if mode == O.SIM_ABOVE_AVG_NZ:
            assert keep.sum() < len(keep)  # the nonzero average is a real cut on this system


# ---- ranked suggestions (Sec. III-A)

def test_fixture_suggestions():
    fx = load_fixture("f5_suggest.json")
    s = fixture_system(fx)
    cls, meth = O.metrics(s)
    assert_fields_equal(cls, _expect(fx["classes"], CLASS_FIELDS), CLASS_FIELDS, "f5")
    assert_fields_equal(meth, _expect(fx["methods"], METHOD_FIELDS), METHOD_FIELDS, "f5")
    cm, ct = O.candidates(s, O.REFERENCED)
    assert [[int(a), int(b)] for a, b in zip(cm, ct)] == fx["referenced"]
    for kind, th, key in ((O.SUGGEST_LCOM, O.THRESH_AVERAGE, "suggest_lcom"), (O.SUGGEST_CBO, O.THRESH_AVERAGE, "suggest_cbo"),
                          (O.SUGGEST_SIMILAR, O.THRESH_AVERAGE, "suggest_similar"),
                          (O.SUGGEST_LCOM, O.THRESH_NONE, "suggest_lcom_no_threshold"),
                          (O.SUGGEST_CBO, O.THRESH_NONE, "suggest_cbo_no_threshold")):
        r = O.suggest(s, kind, th)
        assert [[int(a), int(b), int(c)] for a, b, c in zip(r["method"], r["src"], r["dst"])] == fx[key], key


def test_suggestions_are_ranked_kept_moves():
    """Suggestions are kept moves out of above-average classes, keys never rise
    along the list, and equal keys stay in candidate order."""
    s = synth.plain(50, seed=12)
    cls, meth = O.metrics(s)
    for kind in (O.SUGGEST_LCOM, O.SUGGEST_CBO):
        r = O.suggest(s, kind)
        allr = O.suggest(s, kind, O.THRESH_NONE)
        assert set(zip(r["method"].tolist(), r["dst"].tolist())) <= set(zip(allr["method"].tolist(), allr["dst"].tolist()))
        value = (cls["lcom_p"] - cls["lcom_q"]) if kind == O.SUGGEST_LCOM else cls["cbo"]
        avg = value.sum() / s.n_classes
        assert all(value[S] > avg for S in r["src"].tolist())
        key = meth["fan_out"][r["method"]] if kind == O.SUGGEST_LCOM else \
            meth["fan_in"][r["method"]] + meth["fan_out"][r["method"]]
        assert np.all(np.diff(key) <= 0)
        for k in np.unique(key):
            sel = np.nonzero(key == k)[0]
            pairs = list(zip(r["method"][sel].tolist(), r["dst"][sel].tolist()))
            assert pairs == sorted(pairs)
        assert np.all(r["keep"] == 1)


# ---- multi-move planning

def test_fixture_independent_and_plan():
    fx = load_fixture("f5_suggest.json")
    s = fixture_system(fx)
    r = O.independent(s, O.SUGGEST_LCOM)
    assert [[int(a), int(b), int(c)] for a, b, c in zip(r["method"], r["src"], r["dst"])] == fx["independent_lcom"]
    for kind, key in ((O.SUGGEST_LCOM, "plan_lcom"), (O.SUGGEST_CBO, "plan_cbo")):
        steps, _ = O.plan(s, kind)
        assert [[int(a), int(b), int(c)] for a, b, c in zip(steps["method"], steps["src"], steps["dst"])] == fx[key]


def _lcom(c):
    return c["lcom_p"] - c["lcom_q"]


def test_independent_moves_apply_together_exactly():
    """Applying a whole independent set at once changes each class by exactly the
    delta predicted for the one move that touches it (metrics re-evaluated)."""
    checked = 0
    for seed in (3, 4, 5):
        s = synth.plain(80, seed=seed)
        for kind in (O.SUGGEST_LCOM, O.SUGGEST_CBO):
            r = O.independent(s, kind, O.THRESH_NONE)
            if len(r) < 2:
                continue
            before, _ = O.metrics(s)
            after_sys = s.copy()
            for rec in r:
                after_sys.method_class[int(rec["method"])] = int(rec["dst"])
            after, _ = O.metrics(after_sys)
            touched = {}
            for rec in r:
                m, S, T = int(rec["method"]), int(rec["src"]), int(rec["dst"])
                for X in O.affected_classes(s, m, T):
                    assert X not in touched
                    touched[X] = rec
                assert _lcom(after)[S] - _lcom(before)[S] == rec["d_lcom_src"]
                assert _lcom(after)[T] - _lcom(before)[T] == rec["d_lcom_dst"]
                assert after["cbo"][S] - before["cbo"][S] == rec["d_cbo_src"]
                assert after["cbo"][T] - before["cbo"][T] == rec["d_cbo_dst"]
                assert after["rfc"][S] - before["rfc"][S] == rec["d_rfc_src"]
                assert after["rfc"][T] - before["rfc"][T] == rec["d_rfc_dst"]
            for X in range(s.n_classes):
                if X not in touched:
                    assert after[X] == before[X], X
            checked += len(r)
    assert checked > 40


def test_plan_steps_match_reevaluation():
    s = synth.plain(60, seed=21)
    steps, final = O.plan(s, O.SUGGEST_LCOM, O.THRESH_AVERAGE, max_moves=6)
    cur = s.copy()
    for rec in steps:
        m, S, T = int(rec["method"]), int(rec["src"]), int(rec["dst"])
        before, _ = O.metrics(cur)
        nxt = O.moved(cur, m, T)
        after, _ = O.metrics(nxt)
        assert _lcom(after)[S] - _lcom(before)[S] == rec["d_lcom_src"] < 0
        assert _lcom(after)[T] - _lcom(before)[T] == rec["d_lcom_dst"] < 0
        cur = nxt
    assert np.array_equal(cur.method_class, final.method_class)

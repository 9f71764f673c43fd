"""Pins of the oracle's WMC, NOC and DIT (the rest of the CK suite named in
Sec. II-B) against values that do not come from the oracle: the hand-derived
fixture f8, closed forms of chains and stars, DIT as a breadth-first distance in
the hierarchy graph (scipy), NOC and WMC as weighted counts (numpy), relabelling,
and the effect of a move."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

from oracle import oracle as O
from paper_1308_4011_amd import synth
from tests.helpers import load_fixture, fixture_system


def test_fixture_f8_by_hand():
    fx = load_fixture("f8_ck_hierarchy.json")
    s = fixture_system(fx)
    r = O.ck(s, fx["parent"], fx["weight"])
    assert r["wmc"].tolist() == fx["wmc"]
    assert r["noc"].tolist() == fx["noc"]
    assert r["dit"].tolist() == fx["dit"]
    u = O.ck(s, fx["parent"])
    assert u["wmc"].tolist() == fx["wmc_unit"]
    moved = s.copy()
    moved.method_class[fx["move"]["method"]] = fx["move"]["dst"]
    mv = O.ck(moved, fx["parent"], fx["weight"])
    assert mv["wmc"].tolist() == fx["move"]["wmc"]
    assert mv["noc"].tolist() == fx["noc"] and mv["dit"].tolist() == fx["dit"]
    with pytest.raises(O.CycleError):
        O.ck(s, fx["cycle_parent"], fx["weight"])
    with pytest.raises(ValueError):
        O.ck(s, fx["bad_parent"], fx["weight"])


def _bfs_dit(parent):
    """DIT as the breadth-first distance from a virtual root joined to every class
    without a parent, minus one (scipy on the hierarchy graph, parent -> child)."""
    c = len(parent)
    src = np.where(parent < 0, c, parent)
    g = csr_matrix((np.ones(c), (src, np.arange(c))), shape=(c + 1, c + 1))
    d = shortest_path(g, directed=True, unweighted=True, indices=c)
    return (d[:c] - 1).astype(np.int64)


@pytest.mark.parametrize("maker,seed", [(lambda: synth.plain(200), 5), (lambda: synth.medium(3000), 6)])
def test_generated_hierarchies_against_graph_routines(maker, seed):
    s = maker()
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, seed)
    r = O.ck(s, parent, weight)
    assert np.array_equal(r["dit"], _bfs_dit(parent))
    has = parent >= 0
    assert np.array_equal(r["noc"], np.bincount(parent[has], minlength=s.n_classes))
    wmc = np.bincount(s.method_class, weights=weight.astype(np.float64), minlength=s.n_classes)
    assert np.array_equal(r["wmc"], wmc.astype(np.int64))
    assert r["noc"].sum() == has.sum()
    assert r["wmc"].sum() == weight.sum()
    assert r["dit"].max() >= 3  # the generator makes hierarchies several levels deep


def test_chain_and_star_closed_forms():
    c = 300
    s = synth.from_lists(c, list(range(c)), [], [[] for _ in range(c)], [[] for _ in range(c)])
    perm = np.random.default_rng(3).permutation(c)  # class perm[i] sits at depth i
    parent = np.full(c, -1, np.int64)
    parent[perm[1:]] = perm[:-1]
    r = O.ck(s, parent)
    assert np.array_equal(r["dit"][perm], np.arange(c))
    assert np.array_equal(r["noc"][perm], np.r_[np.ones(c - 1, int), 0])
    assert np.array_equal(r["wmc"], np.ones(c))
    star = np.zeros(c, np.int64)
    star[0] = -1
    r = O.ck(s, star)
    assert r["noc"][0] == c - 1 and (r["noc"][1:] == 0).all()
    assert r["dit"][0] == 0 and (r["dit"][1:] == 1).all()
    selfish = np.full(c, -1)
    selfish[17] = 17  # a class that extends itself is a cycle of length one
    with pytest.raises(O.CycleError):
        O.ck(s, selfish)


def test_relabelling_permutes_the_results():
    s = synth.plain(120, seed=41)
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, 41)
    r = O.ck(s, parent, weight)
    rng = np.random.default_rng(9)
    pc = rng.permutation(s.n_classes)  # class C gets id pc[C]
    pm = rng.permutation(s.n_methods)
    t = s.copy()
    t.method_class = np.empty_like(s.method_class)
    t.method_class[pm] = pc[s.method_class]
    w2 = np.empty_like(weight)
    w2[pm] = weight
    p2 = np.full(s.n_classes, -1, np.int32)
    p2[pc] = np.where(parent >= 0, pc[np.maximum(parent, 0)], -1)
    r2 = O.ck(t, p2, w2)
    assert np.array_equal(r2[pc], r)


def test_moves_change_wmc_only():
    s = synth.plain(80, seed=42)
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, 42)
    r0 = O.ck(s, parent, weight)
    rng = np.random.default_rng(1)
    for _ in range(20):
        m = int(rng.integers(0, s.n_methods))
        S = int(s.method_class[m])
        T = int((S + 1 + rng.integers(0, s.n_classes - 1)) % s.n_classes)
        t = s.copy()
        t.method_class[m] = T
        r1 = O.ck(t, parent, weight)
        d = r1["wmc"] - r0["wmc"]
        want = np.zeros(s.n_classes, np.int64)
        want[S] -= weight[m]
        want[T] += weight[m]
        assert np.array_equal(d, want)
        assert np.array_equal(r1["noc"], r0["noc"]) and np.array_equal(r1["dit"], r0["dit"])

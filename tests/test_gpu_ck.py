"""WMC, NOC and DIT on the GPU against the oracle, field by field: the hand
fixture, generated hierarchies at every single-system size (the 50,000-class
system included), after moves and edits, a chain deeper than one pointer-jumping
round, a cycle, a batch, and the device-output call."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_4011_amd import mm, synth
from tests.helpers import fixture_system, load_fixture

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-ck]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mm.context_create(0)
    yield c
    c.close()


def _same(a, b, what):
    for f in ("wmc", "noc", "dit"):
        x, y = np.asarray(a[f]), np.asarray(b[f])
        if not np.array_equal(x, y):
            bad = np.nonzero(x != y)[0][:8]
            raise AssertionError(f"{what}: {f} differs at {bad.tolist()}: {x[bad].tolist()} vs {y[bad].tolist()}")


def test_fixture_f8(ctx):
    fx = load_fixture("f8_ck_hierarchy.json")
    s = fixture_system(fx)
    g = mm.load_system(ctx, s)
    r = mm.compute_ck(g)  # no hierarchy yet: every class a root, unit weights
    assert r["wmc"].tolist() == fx["wmc_unit"] and not r["noc"].any() and not r["dit"].any()
    mm.set_hierarchy(g, fx["parent"], fx["weight"])
    r = mm.compute_ck(g)
    assert r["wmc"].tolist() == fx["wmc"] and r["noc"].tolist() == fx["noc"] and r["dit"].tolist() == fx["dit"]
    mm.apply_move(g, fx["move"]["method"], fx["move"]["dst"])
    r = mm.compute_ck(g)
    assert r["wmc"].tolist() == fx["move"]["wmc"] and r["dit"].tolist() == fx["dit"]
    for bad in ("cycle_parent", "bad_parent"):
        with pytest.raises(mm.MMError) as e:
            mm.set_hierarchy(g, fx[bad], fx["weight"])
        assert e.value.code == mm.MM_EINVAL
    r = mm.compute_ck(g)  # a refused hierarchy leaves none set
    assert not r["noc"].any() and not r["dit"].any()
    g.free()


@pytest.mark.parametrize("name", ["plain200", "medium5k", "large50k"])
def test_generated(ctx, name):
    s = synth.WORKLOADS[name]()
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, 77)
    g = mm.load_system(ctx, s)
    mm.set_hierarchy(g, parent, weight)
    got = mm.compute_ck(g)
    want = O.ck(s, parent, weight)
    say(f"{name}: {s.n_classes} classes, max DIT {want['dit'].max()}, max NOC {want['noc'].max()}")
    _same(got, want, name)
    import torch
    d = torch.zeros(s.n_classes * mm.CLASS_CK.itemsize, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    mm.compute_ck_device(g, d.data_ptr())
    torch.cuda.synchronize()
    _same(np.frombuffer(d.cpu().numpy().tobytes(), mm.CLASS_CK), want, name + " device output")
    mm.set_hierarchy(g, parent)  # unit weights
    _same(mm.compute_ck(g), O.ck(s, parent), name + " unit weights")
    g.free()


def test_after_moves_and_edits(ctx):
    s = synth.medium(1500, seed=61)
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, 61)
    g = mm.load_system(ctx, s)
    mm.set_hierarchy(g, parent, weight)
    rng = np.random.default_rng(4)
    cur = s.copy()
    for _ in range(10):
        m = int(rng.integers(0, s.n_methods))
        T = int((cur.method_class[m] + 1 + rng.integers(0, s.n_classes - 1)) % s.n_classes)
        mm.apply_move(g, m, T)
        cur.method_class[m] = T
    _same(mm.compute_ck(g), O.ck(cur, parent, weight), "after moves")
    ed = synth.edit_batch(cur, rng, k=200)
    mm.apply_edit(g, *ed)
    cur = synth.apply_edit_arrays(cur, *ed)
    _same(mm.compute_ck(g), O.ck(cur, parent, weight), "after an edit")
    g.free()


def test_deep_chain(ctx):
    """A single chain of 200,000 classes (18 pointer-jumping rounds) in random id
    order: DIT is the position in the chain (closed form; the oracle's walk is
    quadratic here), and a 3,000-class chain against the oracle."""
    for c, check_oracle in ((200_000, False), (3000, True)):
        s = synth.from_lists(c, [0, c - 1], [], [[], []], [[1], []])
        perm = np.random.default_rng(c).permutation(c)
        parent = np.full(c, -1, np.int32)
        parent[perm[1:]] = perm[:-1]
        g = mm.load_system(ctx, s)
        mm.set_hierarchy(g, parent)
        r = mm.compute_ck(g)
        assert np.array_equal(r["dit"][perm], np.arange(c)), c
        assert np.array_equal(r["noc"][perm], np.r_[np.ones(c - 1, np.int32), 0]), c
        if check_oracle:
            _same(r, O.ck(s, parent), f"chain of {c}")
        cyc = parent.copy()
        cyc[perm[0]] = perm[c // 2]  # the root now extends a class below it
        with pytest.raises(mm.MMError) as e:
            mm.set_hierarchy(g, cyc)
        assert e.value.code == mm.MM_EINVAL and "cycle" in str(e.value)
        g.free()


def test_batch(ctx):
    systems = [synth.plain(50, seed=90 + i) for i in range(3)]
    hs = [synth.hierarchy(x.n_classes, x.n_methods, 90 + i) for i, x in enumerate(systems)]
    b = mm.load_batch(ctx, systems)
    off_c = np.cumsum([0] + [x.n_classes for x in systems])
    parent = np.concatenate([np.where(p >= 0, p + o, -1) for (p, _), o in zip(hs, off_c)]).astype(np.int32)
    weight = np.concatenate([w for _, w in hs])
    bad = parent.copy()
    bad[off_c[1]] = 0  # a class of the second part extends one of the first
    with pytest.raises(mm.MMError):
        mm.set_hierarchy(b, bad, weight)
    mm.set_hierarchy(b, parent, weight)
    r = mm.compute_ck(b)
    for i, (x, (p, w)) in enumerate(zip(systems, hs)):
        _same(r[off_c[i]:off_c[i + 1]], O.ck(x, p, w), f"part {i}")
    b.free()

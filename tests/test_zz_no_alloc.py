"""The allocation-free variant of the per-caller-class detail
(mm_move_affected_noalloc) against mm_move_affected, through the C ABI: two
calls in a row on the library's shared scratch array, the second on a smaller
system, each output compared element by element; the context's device memory
does not change across the calls; sizes beyond the array's limit and stale
metrics are refused."""
import ctypes

import numpy as np
import pytest

from paper_1308_4011_amd import mm, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[no-alloc]", *a, flush=True)


def _busiest_move(s):
    """The method with the most distinct caller classes and a destination that is
    neither its class nor one of them when possible (so every caller class is
    listed)."""
    owner = np.asarray(s.method_class)
    callers = np.repeat(np.arange(s.n_methods), np.diff(s.call_off))
    callee = np.asarray(s.call_idx)
    pairs = np.unique(callee.astype(np.int64) * s.n_classes + owner[callers])
    per = np.bincount((pairs // s.n_classes).astype(np.int64), minlength=s.n_methods)
    m = int(np.argmax(per))
    taken = set((pairs[pairs // s.n_classes == m] % s.n_classes).tolist()) | {int(owner[m])}
    T = next(t for t in range(s.n_classes) if t not in taken)
    return m, T


def _noalloc(torch, g, m, T, cap):
    dev = torch.device("cuda:0")
    d_cls = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)
    d_cbo = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)
    d_n = torch.full((1,), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    mm.move_affected_noalloc(g, m, T, d_cls.data_ptr(), d_cbo.data_ptr(), cap, d_n.data_ptr())
    return d_cls, d_cbo, d_n


def test_noalloc_equals_move_affected_two_calls():
    import torch
    torch.cuda.set_device(0)
    big = synth.medium(2000, seed=909)
    small = synth.plain(60, seed=910)
    ctx = mm.context_create(0)  # its own stream: both calls are ordered on it
    try:
        gb = mm.load_system(ctx, big)
        gs = mm.load_system(ctx, small)
        mm.compute_metrics(gb)
        mm.compute_metrics(gs)
        cases = [(gb, big, "2,000 classes"), (gs, small, "60 classes")]
        want, moves = [], []
        for g, s, name in cases:
            m, T = _busiest_move(s)
            cls, dcbo = mm.move_affected(g, m, T)
            say(f"{name}: method {m} -> class {T}: {len(cls)} caller classes")
            assert len(cls) >= 2
            want.append((cls, dcbo))
            moves.append((m, T))
        used0 = ctx.memory()
        # the second call runs on the smaller system right after the first, on the
        # same stream, with no wait between them
        outs = [_noalloc(torch, g, m, T, len(w[0])) for (g, _, _), (m, T), w in zip(cases, moves, want)]
        torch.cuda.synchronize()
        assert ctx.memory() == used0, "the allocation-free call changed the context's device memory"
        for (d_cls, d_cbo, d_n), (cls, dcbo), (_, _, name) in zip(outs, want, cases):
            n = int(d_n.cpu()[0])
            assert n == len(cls), (name, n, len(cls))
            assert np.array_equal(d_cls.cpu().numpy()[:n], cls), name
            assert np.array_equal(d_cbo.cpu().numpy()[:n], dcbo), name
        # a capacity below the count writes only the first entries and still reports the count
        (g, _, _), (m, T), (cls, dcbo) = cases[0], moves[0], want[0]
        d_cls, d_cbo, d_n = _noalloc(torch, g, m, T, 3)
        torch.cuda.synchronize()
        assert int(d_n.cpu()[0]) == len(cls)
        assert np.array_equal(d_cls.cpu().numpy()[:3], cls[:3])
        assert np.array_equal(d_cbo.cpu().numpy()[:3], dcbo[:3])
        # the count alone (capacity 0, no arrays)
        d_n = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
        mm.move_affected_noalloc(g, m, T, None, None, 0, d_n.data_ptr())
        torch.cuda.synchronize()
        assert int(d_n.cpu()[0]) == len(cls)
        gb.free()
        gs.free()
    finally:
        ctx.close()


def test_noalloc_refusals():
    import torch
    torch.cuda.set_device(0)
    ctx = mm.context_create(0)
    try:
        s = synth.plain(60, seed=911)
        g = mm.load_system(ctx, s)
        mm.compute_metrics(g)
        m, T = _busiest_move(s)
        d_n = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        L = mm.lib()
        assert L.mm_move_affected_noalloc(g.handle, m, T, None, None, 0, None) == mm.MM_EINVAL
        assert L.mm_move_affected_noalloc(g.handle, m, T, None, None, 5, d_n.data_ptr()) == mm.MM_EINVAL
        assert L.mm_move_affected_noalloc(g.handle, m, int(s.method_class[m]), None, None, 0,
                                          d_n.data_ptr()) == mm.MM_EINVAL
        # after a move the metrics are stale until recomputed
        mm.apply_move(g, m, T)
        assert L.mm_move_affected_noalloc(g.handle, m, int(s.method_class[m]), None, None, 0,
                                          d_n.data_ptr()) == mm.MM_EINVAL
        assert b"not current" in L.mm_last_error()
        mm.compute_metrics(g)
        assert L.mm_move_affected_noalloc(g.handle, m, int(s.method_class[m]), None, None, 0,
                                          d_n.data_ptr()) == mm.MM_OK
        torch.cuda.synchronize()
        g.free()
        # more classes than the scratch array holds
        c = 1048576 + 1
        huge = synth.from_lists(c, [0, 1], [], [[], []], [[1], []])
        gh = mm.load_system(ctx, huge)
        mm.compute_metrics(gh)
        rc = L.mm_move_affected_noalloc(gh.handle, 1, 2, None, None, 0, d_n.data_ptr())
        assert rc == mm.MM_EINVAL and b"at most 1048576" in L.mm_last_error(), L.mm_last_error()
        gh.free()
    finally:
        ctx.close()

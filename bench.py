#!/usr/bin/env python
"""Throughput of the Move-Method metric engine on one MI355X.

A step is one pass of the whole hot path over a resident synthetic system:
recompute every metric (fan-in/out, CBO, LCOM both forms, RFC), generate the
REFERENCED candidates, score each by its exact deltas on every affected class,
apply the keep rule and compact the kept moves into a device buffer. Inputs are
in HBM before the timed region starts.

The default workload is the 50,000-class system (the largest single system).
Beside the step throughput the line carries: the dominant kernel's roofline
(HIP events in the timed region), the metric recompute's algorithmic bytes over
its measured time with a cold last-level cache (a 1 GiB streaming copy before
every repetition) and a warm one, the CPU oracle timed on the host on the same
system, p50/p99 latencies of a short served leg (64 resident systems under
Poisson edit streams at 50/80/95% of saturated throughput), the recompute after
one move and after a 500-method edit on the same system (only what the change
touched is recomputed) beside the full recompute, and WMC/NOC/DIT of every class.

Prints one JSON line (rank 0). Options: --gpus (1 only), --steps, --warmup,
--workload {plain200, medium5k, large50k, batch256, served64, similar5k},
--no-cpu-baseline, --no-served.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "move candidates scored/sec + metric recompute HBM GB/s; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
METRIC_KERNELS = ["k_method_basic", "k_map_tab_wc", "k_map_tab_mid", "k_big_stage", "k_big_build", "k_in_runs",
                  "k_map_tab_in", "k_big_in_flags", "k_coaccess", "k_coaccess_big",
                  "k_coaccess_small", "k_finalize"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_schedule(text):
    """'fill_chunk=2048,fill_group=2' -> {'fill_chunk': 2048, 'fill_group': 2}"""
    out = {}
    for item in filter(None, (x.strip() for x in text.split(","))):
        k, v = item.split("=")
        out[k.strip()] = int(v)
    return out


def unique_pairs(a, b):
    return int(len(np.unique(a.astype(np.int64) * (1 << 31) + b.astype(np.int64))))


def dedup_rows(off, idx):
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    key = np.unique(rows.astype(np.int64) * (1 << 31) + idx)
    return (key >> 31).astype(np.int64), (key & ((1 << 31) - 1)).astype(np.int64)


def algorithmic_bytes(s, cls, n_cand, kept=0):
    """Bytes each kernel must move at least once (inputs read once, outputs
    written once); gathers through owner / attribute-class tables are cache
    traffic and are not counted."""
    n, c = s.n_methods, s.n_classes
    ar, aa = dedup_rows(s.acc_off, s.acc_idx)
    cr, cc = dedup_rows(s.call_off, s.call_idx)
    nacc, ncall = len(aa), len(cc)
    owner = s.method_class.astype(np.int64)
    acls = s.attr_class.astype(np.int64)
    w_entries = int(cls["cbo"].sum())
    cnt_entries = unique_pairs(owner[cr], cc)
    self_call = cr == cc
    in_entries = unique_pairs(cc[~self_call], owner[cr[~self_call]])
    out_entries = unique_pairs(np.concatenate([cr[~self_call], ar]),
                               np.concatenate([owner[cc[~self_call]], acls[aa]]))
    off = 4 * (n + 1)
    # Tables by size, as the library lays them out: W and CNT of up to 512
    # references grouped in LDS by waves (k_map_tab_wc), up to 2048 by a block
    # (k_map_tab_mid; systems of 2^17 methods or more, else these join the
    # next tier), more as hash tables built in two passes (k_big_stage reads
    # their rows, k_big_build writes their entries); caller rows of 1..32 by
    # k_in_runs, 33..512 by k_map_tab_in, more by the two passes.
    mid_hi = 2048 if n >= (1 << 17) else 512
    nmem = np.bincount(owner, minlength=c)
    wref = np.bincount(owner[cr], minlength=c) + np.bincount(owner[ar], minlength=c)
    cref = np.bincount(owner[cr], minlength=c)
    w_ent = cls["cbo"].astype(np.int64)
    cpair = np.unique(owner[cr] * (1 << 31) + cc)
    c_ent = np.bincount(cpair >> 31, minlength=c)
    # W: members, their offset pairs, their rows, the grouped entries; CNT:
    # members, call offsets, calls, grouped entries
    w_cost = 4 * nmem + 16 * nmem + 4 * wref + 8 * w_ent
    c_cost = 4 * nmem + 8 * nmem + 4 * cref + 8 * c_ent
    rlen = np.bincount(cc, minlength=n)
    ipair = np.unique(cc[~self_call] * (1 << 31) + owner[cr[~self_call]])
    i_ent = np.bincount(ipair >> 31, minlength=n)

    def tier(r, lo, hi):
        return (r > lo) & (r <= hi)
    big = 1 << 62
    # caller rows: list entry, offsets pair and header read, length and own
    # count written (36 bytes for runs, 28 for tables), callers read, entries written
    i_cost_run = 36 + 4 * rlen + 8 * i_ent
    i_cost_tab = 28 + 4 * rlen + 8 * i_ent
    b = {
        "k_method_basic": 3 * off + 4 * n + 4 * nacc + 16 * n + 8 * n,
        "k_map_tab_wc": int(w_cost[tier(wref, 0, 512)].sum() + c_cost[tier(cref, 0, 512)].sum()),
        "k_map_tab_mid": int(w_cost[tier(wref, 512, mid_hi)].sum() + c_cost[tier(cref, 512, mid_hi)].sum()),
        "k_in_runs": int(i_cost_run[tier(rlen, 0, 32)].sum()),
        "k_map_tab_in": int(i_cost_tab[tier(rlen, 32, 512)].sum()),
        # the hash-table segments: their rows read (the staged pairs between
        # the passes are the implementation's, not the method's), their grouped
        # entries written
        "k_big_stage": int((w_cost - 8 * w_ent)[tier(wref, mid_hi, big)].sum()
                           + (c_cost - 8 * c_ent)[tier(cref, mid_hi, big)].sum()
                           + (4 * rlen)[tier(rlen, 512, big)].sum()),
        "k_big_build": int(8 * w_ent[tier(wref, mid_hi, big)].sum() + 8 * c_ent[tier(cref, mid_hi, big)].sum()
                           + (8 * i_ent)[tier(rlen, 512, big)].sum()),
        "k_coaccess": 4 * n + 8 * n + 4 * n,
        "k_finalize": 4 * n + 8 * n + 48 * c,
        "k_prep": 2 * off + 4 * (nacc + ncall) + 12 * out_entries + 32 * n,
        # candidate (method, class, out entry) read, per-method and per-class
        # terms read once, keep flag written per candidate, kept records written
        "k_delta": 12 * n_cand + 32 * n + 12 * out_entries + 48 * c + 16 * n + 4 * n_cand,
    }
    b["k_delta"] += 96 * kept
    b["compute_metrics"] = sum(v for k, v in b.items() if k in METRIC_KERNELS)
    b["_sizes"] = {"acc_nnz": nacc, "call_nnz": ncall, "w_entries": w_entries, "cnt_entries": cnt_entries,
                   "in_entries": in_entries, "out_entries": out_entries}
    return b


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when it
    was taken on the same kernel sources and workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rows = json.load(open(path))
    except (OSError, ValueError):
        return None
    for r in rows:
        if r.get("kernel") == kernel and r.get("workload") == workload and r.get("src_digest") == digest:
            return r.get("hbm_bytes_per_launch")
    return None


def snapshot_sha256(s):
    """SHA-256 of a system's arrays (sizes, owners, rows), identifying the snapshot
    a CPU and a GPU figure were taken on."""
    h = hashlib.sha256()
    h.update(np.array([s.n_classes, s.n_methods, s.n_attrs], np.int64).tobytes())
    for arr, dt in zip(s.arrays(), (np.int32, np.int32, np.int64, np.int32, np.int64, np.int32)):
        h.update(np.ascontiguousarray(arr, dt).tobytes())
    return h.hexdigest()


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(s, n_cand, mask, rule, budget_s, gpu_kept):
    """The second CPU oracle (grouped counts and incremental delta formulas,
    POSIX threads) timed on the host over one whole step of the same system:
    the grouped counts of every class (one thread, the metric recompute), the
    REFERENCED candidate list, and every candidate scored on the host threads
    (at most 16: the CPU share of one GPU on these hosts). Whole steps repeat
    until about `budget_s` of wall time is used. A 1-thread rate on a sample of
    the candidates is reported beside it."""
    from oracle import incremental as I
    nt = I.host_threads()
    passes, t_total, kept = 0, 0.0, -1
    while passes == 0 or (t_total < budget_s * 0.7 and passes < 8):
        t0 = time.perf_counter()
        inc = I.Incremental(s)
        cm, ct = inc.referenced()
        recs = inc.score(cm, ct, mask, rule, threads=nt)
        t_total += time.perf_counter() - t0
        passes += 1
        kept = int(recs["keep"].sum())
        del recs
        if passes == 1:
            k = min(len(cm), 200_000)
            sel = np.sort(np.random.default_rng(0).choice(len(cm), k, replace=False))
            t0 = time.perf_counter()
            inc.score(cm[sel], ct[sel], mask, rule, threads=1)
            one_thread = k / max(time.perf_counter() - t0, 1e-9)
        inc.close()
    step_s = t_total / passes
    hi = host_info()
    return {"value": n_cand / step_s, "unit": "candidates/s", "cores": nt, "kind": "oracle",
            "sample": f"whole steps of the same system ({passes} passes, {step_s:.3f} s each): grouped counts of "
                      f"every class on one thread, then all {len(cm)} REFERENCED candidates scored on {nt} threads "
                      f"by the second (incremental) C oracle; one thread scores {one_thread:.3g} candidates/s "
                      f"({k} sampled); host {hi['cpu_model']}, nproc {hi['nproc']}, affinity {hi['affinity']}",
            "one_thread_candidates_per_s": one_thread, "step_s": step_s, "kept": kept,
            "kept_equals_gpu": kept == gpu_kept, "host": hi}


def metric_phase(torch, mm, g, d_cls, d_meth, stream, reps=20):
    """Time the metric recompute alone with HIP events on its stream: warm (back
    to back) and cold (a 1 GiB streaming copy, larger than the last-level cache,
    before each repetition)."""
    flush_src = torch.ones(128 << 20, dtype=torch.int32, device=stream.device)
    flush_dst = torch.empty_like(flush_src)
    out = {}
    for mode in ("warm", "cold"):
        times = []
        for _ in range(reps):
            if mode == "cold":
                flush_dst.copy_(flush_src)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mm.compute_metrics_device(g, d_cls.data_ptr(), d_meth.data_ptr())
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        out[mode + "_ms"] = float(np.median(times))
    out["flush_bytes"] = 2 * flush_src.numel() * 4
    del flush_src, flush_dst
    return out


def incremental_leg(torch, mm, synth, s, stream, full_ms, moves=20, edit_k=500, edits=3):
    """Recompute after changes on the same system, timed with HIP events on its
    stream: one move at a time (only the touched segments are recomputed), and
    `edits` edits of `edit_k` methods each (rows replaced, a quarter changing
    owner), each followed by a recompute, the last also by the rescoring of the
    edited methods' REFERENCED candidates."""
    ctx = mm.context_create(0, stream.cuda_stream)
    g = mm.load_system(ctx, s)
    mm.compute_metrics_device(g, None, None)
    torch.cuda.synchronize()
    rng = np.random.default_rng(synth.BASE_SEED + 77)
    cur = s.copy()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), (time.perf_counter() - t0) * 1000.0, out

    move_dev, move_host = [], []
    for _ in range(moves):
        m = int(rng.integers(0, s.n_methods))
        row = s.call_idx[s.call_off[m]:s.call_off[m + 1]]
        if not len(row):
            continue
        T = int(cur.method_class[row[rng.integers(0, len(row))]])
        if T == cur.method_class[m]:
            continue
        t0 = time.perf_counter()
        mm.apply_move(g, m, T)
        apply_ms = (time.perf_counter() - t0) * 1000.0
        cur.method_class[m] = T
        dev, host, _ = timed(lambda: mm.compute_metrics_device(g, None, None))
        move_dev.append(dev)
        move_host.append(host + apply_ms)
    # a few edits in a row: the first also pays for first-use buffers
    apply_all, rec_all = [], []
    for _ in range(edits):
        ed = synth.edit_batch(cur, rng, k=edit_k)
        t0 = time.perf_counter()
        mm.apply_edit(g, *ed)
        apply_all.append((time.perf_counter() - t0) * 1000.0)
        rec_dev, rec_host, _ = timed(lambda: mm.compute_metrics_device(g, None, None))
        rec_all.append((rec_dev, rec_host))
        cur = synth.apply_edit_arrays(cur, *ed)
    methods = np.asarray(ed[0])
    cm, ct = [], []
    for m in methods:
        refs = np.unique(np.concatenate([cur.method_class[cur.call_idx[cur.call_off[m]:cur.call_off[m + 1]]],
                                         cur.attr_class[cur.acc_idx[cur.acc_off[m]:cur.acc_off[m + 1]]]]))
        refs = refs[refs != cur.method_class[m]]
        cm += [int(m)] * len(refs)
        ct += refs.tolist()
    n_out = mm.score_moves_count(g, mm.EXPLICIT, cm, ct, keep_only=True)
    d_out = torch.empty(max(n_out, 1) * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device=stream.device)
    sc_dev, sc_host, kept = timed(lambda: mm.score_moves_device(g, d_out.data_ptr(), n_out, mm.EXPLICIT, cm, ct,
                                                                keep_only=True))
    g.free()
    ctx.close()
    return {"what": "recompute after changes on the same system (HIP events on its stream)",
            "full_recompute_ms": full_ms,
            "move": {"moves": len(move_dev), "recompute_ms_median": float(np.median(move_dev)),
                     "apply_plus_recompute_host_ms_median": float(np.median(move_host))},
            "edit": {"methods": int(len(methods)), "edits": edits,
                     "apply_host_ms_median": float(np.median(apply_all)), "apply_host_ms_first": apply_all[0],
                     "recompute_ms_median": float(np.median([r[0] for r in rec_all])),
                     "recompute_host_ms_median": float(np.median([r[1] for r in rec_all])),
                     "rescore_candidates": len(cm), "rescore_ms": sc_dev,
                     "rescore_host_ms": sc_host, "kept": int(kept),
                     "device_ms_total": float(np.median([r[0] for r in rec_all])) + sc_dev}}


def ck_leg(torch, mm, synth, s, stream, reps=20):
    """WMC, NOC and DIT of every class (the hierarchy set once; WMC summed per
    class on every call), timed with HIP events; algorithmic bytes: weights and
    membership read once, 16 B per class written."""
    ctx = mm.context_create(0, stream.cuda_stream)
    g = mm.load_system(ctx, s)
    parent, weight = synth.hierarchy(s.n_classes, s.n_methods, synth.BASE_SEED + 88)
    t0 = time.perf_counter()
    mm.set_hierarchy(g, parent, weight)
    set_ms = (time.perf_counter() - t0) * 1000.0
    d = torch.empty(s.n_classes * mm.CLASS_CK.itemsize, dtype=torch.uint8, device=stream.device)
    mm.compute_ck_device(g, d.data_ptr())
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mm.compute_ck_device(g, d.data_ptr())
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    g.free()
    ctx.close()
    ms = float(np.median(times))
    alg = 4 * s.n_methods * 2 + 8 * (s.n_classes + 1) + 8 * s.n_classes + 16 * s.n_classes
    return {"ms": ms, "set_hierarchy_host_ms": set_ms, "algorithmic_bytes": alg,
            "gbps": alg / (ms / 1000.0) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large50k",
                    choices=["plain200", "medium5k", "large50k", "batch256", "served64", "similar5k"])
    ap.add_argument("--served-systems", type=int, default=64)
    ap.add_argument("--requests", type=int, default=200, help="requests per load level (served)")
    ap.add_argument("--batch-systems", type=int, default=256)
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the schedule (scoring knobs and metric fill items) before timing; the batch "
                         "workload always does")
    ap.add_argument("--no-autotune", action="store_true", help="batch workload: time the default schedule")
    ap.add_argument("--schedule", default="",
                    help="time this schedule: comma-separated name=value over the defaults (caller_light, "
                         "heavy_chunk, delta_chunk, delta_grid, fill_chunk, fill_group)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-served", action="store_true", help="skip the short served leg of a single-system run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the incremental and WMC/NOC/DIT legs of a single-system run (profiling runs)")
    ap.add_argument("--served-requests", type=int, default=200, help="requests per load level of the served leg")
    ap.add_argument("--keep-all", action="store_true", help="output every scored record, not only kept ones")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scale for the HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the path has no multi-GPU form); run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_1308_4011_amd import mm, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # one stream of our own (default priority) for everything torch and the
    # library enqueue: the contexts borrow it, so HIP events recorded on it
    # bracket the library's kernels (torch's default stream has handle 0, with
    # which a context would create a stream of its own)
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    if a.calibrate_copy:
        n = a.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n, "calibrate_copy_bytes_written": n, "launches": 5}))
        return
    if a.workload == "batch256":
        return bench_batch(a, torch, mm, synth, dev)
    if a.workload == "served64":
        return bench_served(a, mm, synth)
    if a.workload == "similar5k":
        return bench_similar(a, torch, mm, synth, dev)
    s = synth.WORKLOADS[a.workload]()
    log(f"[bench] workload {a.workload}: {s.summary()}")
    stream = torch.cuda.current_stream(dev)
    ctx = mm.context_create(0, stream.cuda_stream)
    g = mm.load_system(ctx, s)
    mask, rule = mm.CBO | mm.LCOM_PQ, mm.PARETO
    if a.schedule:
        mm.context_set_tuning(ctx, {**mm.context_get_tuning(ctx), **parse_schedule(a.schedule)})
    tuning = mm.autotune(g, mm.REFERENCED, metric_mask=mask, rule=rule) if a.autotune else mm.context_get_tuning(ctx)
    n_cand = mm.score_moves_count(g, mm.REFERENCED, metric_mask=mask, rule=rule)
    d_out = torch.empty(max(n_cand, 1) * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device=dev)
    d_cls = torch.empty(max(s.n_classes, 1) * mm.CLASS_METRICS.itemsize, dtype=torch.uint8, device=dev)
    d_meth = torch.empty(max(s.n_methods, 1) * mm.METHOD_METRICS.itemsize, dtype=torch.uint8, device=dev)
    keep_only = not a.keep_all

    def step():
        mm.compute_metrics_device(g, d_cls.data_ptr(), d_meth.data_ptr())
        return mm.score_moves_device(g, d_out.data_ptr(), n_cand, mm.REFERENCED, metric_mask=mask, rule=rule,
                                     keep_only=keep_only)

    # census: every kernel timed for a few steps
    mm.context_set_timing(ctx, "*")
    for _ in range(3):
        kept = step()
    torch.cuda.synchronize()
    census = mm.context_timing(ctx, reset=True)
    mm.context_set_timing(ctx, None)
    per_step = {k: v[1] / 3.0 for k, v in census.items()}
    for k, v in sorted(per_step.items(), key=lambda kv: -kv[1]):
        log(f"[bench] census {k:18s} {v * 1000:9.1f} us/step ({census[k][0] // 3} launches/step)")
    dominant = max(per_step, key=per_step.get)

    cls_host = np.frombuffer(d_cls.cpu().numpy().tobytes(), mm.CLASS_METRICS)[:s.n_classes]
    alg = algorithmic_bytes(s, cls_host, n_cand, kept if keep_only else n_cand)

    mm.context_set_timing(ctx, dominant)
    for _ in range(a.warmup):
        step()
    mm.context_timing(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        kept = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = mm.context_timing(ctx, reset=True)
    mm.context_set_timing(ctx, None)
    launches, total_ms = kt.get(dominant, (0, 0.0))
    avg_s = total_ms / 1000.0 / max(launches, 1)
    elapsed = t1 - t0
    ms_per_step = elapsed * 1000.0 / a.steps

    dom_bytes = alg.get(dominant)
    digest = source_digest(["paper_1308_4011_amd/csrc/k_metrics.hip", "paper_1308_4011_amd/csrc/k_score.hip",
                            "paper_1308_4011_amd/csrc/mm_dev.h"])
    achieved = dom_bytes / avg_s / 1e9 if dom_bytes and avg_s > 0 else None
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic_for(dominant, a.workload, digest),
                "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": dom_bytes, "src_digest": digest}
    # the metric recompute on its own: every input read once (two offset arrays,
    # both row arrays, owners, attribute classes) and every output written once
    # (16 B per method, 48 B per class, 8 B per grouped count of w and cnt)
    sz = alg["_sizes"]
    m_, c_, a_ = s.n_methods, s.n_classes, s.n_attrs
    rec_bytes = (4 * (2 * (m_ + 1) + sz["acc_nnz"] + sz["call_nnz"] + m_ + a_) + 16 * m_ + 48 * c_
                 + 8 * (sz["w_entries"] + sz["cnt_entries"]))
    phase = metric_phase(torch, mm, g, d_cls, d_meth, stream)
    metric_ms = sum(per_step.get(k, 0.0) for k in METRIC_KERNELS)
    recompute = {"algorithmic_bytes": rec_bytes, "kernel_ms_per_step_census": metric_ms, **phase}
    for mode in ("warm", "cold"):
        gbps = rec_bytes / (phase[mode + "_ms"] / 1000.0) / 1e9
        recompute[f"gbps_{mode}"] = gbps
        recompute[f"frac_{mode}"] = gbps / HBM_PEAK_GBS
    roofline["traversal"] = {"what": "metric recompute (all its kernels, both streams) between HIP events, "
                                     "cold last-level cache", "achieved": recompute["gbps_cold"],
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": recompute["frac_cold"],
                             "algorithmic_bytes": rec_bytes, "ms": phase["cold_ms"]}

    out = {"metric": METRIC, "value": n_cand * a.steps / elapsed, "unit": "candidates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": a.workload, "classes": s.n_classes, "methods": s.n_methods,
                      "attrs": s.n_attrs, "acc_nnz": alg["_sizes"]["acc_nnz"], "call_nnz": alg["_sizes"]["call_nnz"],
                      "candidates": n_cand, "candidate_set": "REFERENCED", "rule": "PARETO",
                      "metric_mask": "CBO|LCOM_PQ", "kept": int(kept), "keep_only": keep_only,
                      "schedule": tuning, "autotuned": a.autotune, "snapshot_sha256": snapshot_sha256(s)},
           "roofline": roofline, "metric_recompute": recompute,
           "kernel_us_per_step": {k: round(v * 1000.0, 2) for k, v in per_step.items()},
           "served_latency_ms": None, "cpu_baseline": None}
    g.free()
    ctx.close()
    del d_out, d_cls, d_meth
    torch.cuda.empty_cache()
    if not a.no_extra:
        log("[bench] incremental leg ...")
        out["incremental"] = incremental_leg(torch, mm, synth, s, stream, phase["warm_ms"])
        log(f"[bench] incremental: {out['incremental']}")
        out["ck"] = ck_leg(torch, mm, synth, s, stream)
        log(f"[bench] WMC/NOC/DIT: {out['ck']}")
    if not a.no_served:
        log("[bench] served leg ...")
        sv = served_leg(a, mm, synth, a.served_requests)
        out["served_latency_ms"] = {**{k: level_summary(v) for k, v in sv["levels"].items()},
                                    "one_at_a_time": level_summary(sv["one_at_a_time"]),
                                    "workload": sv["workload"], "requests_per_level": a.served_requests,
                                    "saturated_req_per_s": sv["saturated"]["req_per_s"],
                                    "one_at_a_time_req_per_s": sv["one_at_a_time"]["req_per_s"]}
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on the same system ...")
        out["cpu_baseline"] = cpu_baseline(s, n_cand, mask, rule, a.cpu_seconds, int(kept))
    print(json.dumps(out))


def bench_batch(a, torch, mm, synth, dev):
    """Snapshots of uneven sizes scored as one batch (each phase one launch over
    every snapshot) against one launch sequence per snapshot."""
    t0 = time.perf_counter()
    systems = synth.batch(a.batch_systems)
    log(f"[bench] batch of {len(systems)} snapshots generated in {time.perf_counter() - t0:.1f} s: "
        f"classes {sum(x.n_classes for x in systems)}, methods {sum(x.n_methods for x in systems)}, "
        f"calls {sum(x.nnz_call for x in systems)}")
    stream = torch.cuda.current_stream(dev)
    ctx = mm.context_create(0, stream.cuda_stream)
    mask, rule = mm.CBO | mm.LCOM_PQ, mm.PARETO
    b = mm.load_batch(ctx, systems)
    tuned = not a.no_autotune
    t0 = time.perf_counter()
    tuning = mm.autotune(b, mm.REFERENCED, metric_mask=mask, rule=rule, keep_only=True, repeats=2) if tuned \
        else mm.context_get_tuning(ctx)
    log(f"[bench] schedule {tuning} ({'autotuned in %.1f s' % (time.perf_counter() - t0) if tuned else 'default'})")
    n_cand = mm.score_moves_count(b, mm.REFERENCED, metric_mask=mask, rule=rule)
    d_out = torch.empty(max(n_cand, 1) * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device=dev)
    d_cls = torch.empty(max(b.n_classes, 1) * mm.CLASS_METRICS.itemsize, dtype=torch.uint8, device=dev)
    d_meth = torch.empty(max(b.n_methods, 1) * mm.METHOD_METRICS.itemsize, dtype=torch.uint8, device=dev)

    def step_batch():
        mm.compute_metrics_device(b, d_cls.data_ptr(), d_meth.data_ptr())
        return mm.score_moves_device(b, d_out.data_ptr(), n_cand, mm.REFERENCED, metric_mask=mask, rule=rule,
                                     keep_only=True)

    mm.context_set_timing(ctx, "*")
    step_batch()
    torch.cuda.synchronize()
    census = mm.context_timing(ctx, reset=True)
    mm.context_set_timing(ctx, None)
    for k, v in sorted(census.items(), key=lambda kv: -kv[1][1]):
        log(f"[bench] batch census {k:18s} {v[1] * 1000:9.1f} us ({v[0]} launches)")
    for _ in range(a.warmup):
        step_batch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        kept = step_batch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / a.steps
    log(f"[bench] batch step {t_batch * 1e3:.2f} ms, {n_cand} candidates, {kept} kept")

    # the same snapshots, one launch sequence each
    gs = [mm.load_system(ctx, x) for x in systems]
    counts = [mm.score_moves_count(g, mm.REFERENCED, metric_mask=mask, rule=rule) for g in gs]
    assert sum(counts) == n_cand, (sum(counts), n_cand)
    outs = [torch.empty(max(k, 1) * mm.MOVE_SCORE.itemsize, dtype=torch.uint8, device=dev) for k in counts]

    def step_each():
        kept = 0
        for g, o, k, x in zip(gs, outs, counts, systems):
            mm.compute_metrics_device(g, None, None)
            kept += mm.score_moves_device(g, o.data_ptr(), k, mm.REFERENCED, metric_mask=mask, rule=rule,
                                          keep_only=True)
        return kept

    step_each()
    torch.cuda.synchronize()
    reps = max(1, a.steps // 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        kept_each = step_each()
    torch.cuda.synchronize()
    t_each = (time.perf_counter() - t0) / reps
    log(f"[bench] per-snapshot sequence {t_each * 1e3:.2f} ms, {kept_each} kept")
    assert kept_each == kept
    out = {"metric": METRIC, "value": n_cand / t_batch, "unit": "candidates/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"batch{len(systems)}", "snapshots": len(systems),
                      "classes": int(sum(x.n_classes for x in systems)),
                      "methods": int(sum(x.n_methods for x in systems)), "candidates": n_cand,
                      "candidate_set": "REFERENCED", "rule": "PARETO", "metric_mask": "CBO|LCOM_PQ",
                      "kept": int(kept), "schedule": tuning, "autotuned": tuned},
           "per_snapshot_launches": {"ms_per_step": t_each * 1e3, "value": n_cand / t_each,
                                     "speedup_of_batch": t_each / t_batch},
           "kernel_us_per_step": {k: round(v[1] * 1000.0, 1) for k, v in census.items()}}
    for g in gs:
        g.free()
    b.free()
    ctx.close()
    print(json.dumps(out))


def bench_similar(a, torch, mm, synth, dev):
    """Similarity of every method pair of the 5,000-class system (Sec. II-A and
    the all-pairs count of Sec. III-B) and the moves it suggests (Sec. III-A):
    one step = the similarity passes under the all-pairs average plus scoring the
    SIMILAR candidates with the paper's LCOM rule (kept records only)."""
    s = synth.medium(5000)
    log(f"[bench] similar5k: {s.summary()}")
    stream = torch.cuda.current_stream(dev)
    ctx = mm.context_create(0, stream.cuda_stream)
    g = mm.load_system(ctx, s)
    th, mask, rule = mm.SIM_ABOVE_AVG, mm.LCOM_PQ, mm.PAPER_LCOM
    mm.set_similarity_threshold(g, th)
    st = mm.similarity(g, th)
    n_cand = st["n_candidates"]
    log(f"[bench] similarity: {st}")
    n_kept = mm.score_moves_count(g, mm.SIMILAR, metric_mask=mask, rule=rule, keep_only=True)
    d_out = torch.empty(max(n_kept, 1) * mm.MOVE_SCORE.itemsize // 8, dtype=torch.int64, device=dev)

    def step():
        mm.similarity(g, th)
        return mm.score_moves_device(g, d_out.data_ptr(), n_kept, mm.SIMILAR, metric_mask=mask, rule=rule,
                                     keep_only=True)

    mm.context_set_timing(ctx, "*")
    kept = step()
    torch.cuda.synchronize()
    census = mm.context_timing(ctx, reset=True)
    mm.context_set_timing(ctx, None)
    for k, v in sorted(census.items(), key=lambda kv: -kv[1][1]):
        log(f"[bench] census {k:18s} {v[1] * 1000:11.1f} us/step ({v[0]} launches/step)")
    for _ in range(a.warmup):
        step()
    mm.context_set_timing(ctx, "k_sim_rows")
    mm.context_timing(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        kept = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = mm.context_timing(ctx, reset=True)
    mm.context_set_timing(ctx, None)
    launches, sim_ms = kt.get("k_sim_rows", (0, 0.0))
    pairs = st["n_pairs"]
    # one incidence = one (row, other user of a shared property) visit: a 4-byte
    # list read and a 4-byte counter update, twice per pass (add, then claim)
    deg_call = np.bincount(s.call_idx, minlength=s.n_methods).astype(np.int64)
    deg_acc = np.bincount(s.acc_idx, minlength=s.n_attrs).astype(np.int64)
    incid_all = int((deg_call * (deg_call - 1)).sum() + (deg_acc * (deg_acc - 1)).sum())
    out = {"metric": METRIC, "value": n_cand * a.steps / elapsed, "unit": "candidates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": elapsed * 1000.0 / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "similar5k", "classes": s.n_classes, "methods": s.n_methods,
                      "candidates": n_cand, "candidate_set": "SIMILAR (above the all-pairs average)",
                      "rule": "PAPER_LCOM", "metric_mask": "LCOM_PQ", "kept": int(kept)},
           "similarity": {"pairs": pairs, "pairs_sharing_a_property": st["n_nonzero"],
                          "similarity_values_per_s": pairs * a.steps / elapsed,
                          "k_sim_rows_ms_per_step": sim_ms / max(a.steps, 1),
                          "k_sim_rows_launches_per_step": launches / max(a.steps, 1),
                          "incidences_per_pass": {"stats_and_pairs": incid_all // 2, "count": incid_all}},
           "kernel_us_per_step": {k: round(v[1] * 1000.0, 1) for k, v in census.items()},
           "roofline": None, "served_latency_ms": None, "cpu_baseline": None}
    print(json.dumps(out))


def served_leg(a, mm, synth, n_requests):
    """Resident systems served under a Poisson stream of edits (98%) and loads
    (2%); latency from submission to host-visible result. The budget holds the
    resident systems with 15% to spare, so new loads evict idle systems, which
    the server reloads from their kept state when a later request names them
    (inside that request, whose latency counts from its submission). Every
    level runs on a fresh server holding the same resident systems."""
    import math
    rng = np.random.default_rng(synth.BASE_SEED + 5999)

    def wait(srv, ticket):  # a request unfinished after two minutes ends the run with an error
        return srv.wait(ticket, timeout_ms=120_000)
    counts = synth.served_class_counts(a.served_systems)
    t0 = time.perf_counter()
    systems = [synth.served_system(int(k), synth.BASE_SEED + 5000 + j) for j, k in enumerate(counts)]
    extra = [synth.served_system(int(k), synth.BASE_SEED + 5500 + j)
             for j, k in enumerate(np.rint(np.exp(rng.uniform(math.log(1000), math.log(50000), 8))).astype(int))]
    log(f"[bench] {len(systems)} resident systems generated in {time.perf_counter() - t0:.1f} s: "
        f"classes {int(sum(x.n_classes for x in systems))}, methods {int(sum(x.n_methods for x in systems))}")

    def make_requests(n):
        reqs = []
        for _ in range(n):
            if rng.random() < 0.02:
                reqs.append(("load", int(rng.integers(0, len(extra)))))
            else:
                j = int(rng.integers(0, len(systems)))
                k = int(round(math.exp(rng.uniform(0, math.log(500)))))
                reqs.append(("edit", j, synth.edit_batch(systems[j], rng, k=k)))
        return reqs

    def submit(srv, r, load_id):
        if r[0] == "load":
            return srv.load(load_id, extra[r[1]])
        return srv.edit(r[1], *r[2])

    # residency: load everything, then cap memory at 1.15x so new loads evict
    srv = mm.Server(n_slots=4)
    t0 = time.perf_counter()
    for t in [srv.load(j, x) for j, x in enumerate(systems)]:
        res = wait(srv, t)
        assert res["status"] == mm.MM_OK, res["error"]
    load_s = time.perf_counter() - t0
    st = srv.stats()
    resident_bytes = st["device_bytes"]
    srv.close()
    log(f"[bench] all systems loaded in {load_s:.1f} s (load latency p50 {st['p50_ms']:.1f} ms, "
        f"p99 {st['p99_ms']:.1f} ms), {resident_bytes / 2**30:.2f} GiB resident")

    def breakdown(results):
        """Latency (submission to result), queueing and service percentiles per
        request kind, from the server's own clock."""
        out = {}
        for kind in ("edit", "load"):
            rs = [res for r, res in results if r[0] == kind]
            if not rs:
                continue
            lat = np.array([x["end_ms"] - x["submit_ms"] for x in rs])
            que = np.array([x["start_ms"] - x["submit_ms"] for x in rs])
            svc = np.array([x["end_ms"] - x["start_ms"] for x in rs])
            out[kind] = {"n": len(rs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                         "queue_p50_ms": float(np.percentile(que, 50)), "queue_p99_ms": float(np.percentile(que, 99)),
                         "service_p50_ms": float(np.percentile(svc, 50)),
                         "service_p99_ms": float(np.percentile(svc, 99)), "max_ms": float(lat.max())}
        return out

    def run_level(srv, reqs, rate, next_id):
        """Submit the stream: Poisson arrivals at `rate` on an absolute schedule
        (a late submission does not delay the ones after it), or all at once.
        A load's submission copies a whole system (up to 50k classes), so loads
        are submitted from a helper thread and do not hold up the arrivals
        behind them (they name new systems, so their order does not matter)."""
        from concurrent.futures import ThreadPoolExecutor
        srv.stats(reset=True)
        tickets, t_start = [], time.perf_counter()
        due = t_start
        with ThreadPoolExecutor(max_workers=2) as helper:
            for r in reqs:
                if rate:
                    due += rng.exponential(1.0 / rate)
                    ahead = due - time.perf_counter()
                    if ahead > 0:
                        time.sleep(ahead)
                if r[0] == "load":
                    next_id += 1
                    tickets.append((r, helper.submit(submit, srv, r, next_id)))
                else:
                    tickets.append((r, submit(srv, r, next_id)))
            tickets = [(r, t if isinstance(t, int) else t.result()) for r, t in tickets]
        results = [(r, wait(srv, t)) for r, t in tickets]
        srv.drain()
        wall = time.perf_counter() - t_start
        codes = {}
        for _, res in results:
            codes[res["status"]] = codes.get(res["status"], 0) + 1
        st = srv.stats()
        return {"requests": len(reqs), "offered_req_per_s": rate, "wall_s": wall, "req_per_s": len(reqs) / wall,
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                "kept_records": st["records"], "status_counts": {str(k): v for k, v in codes.items()},
                "evicted": st["evicted"], "reloaded": st["reloaded"], "by_kind": breakdown(results)}, next_id

    def fresh_server(slots):
        """Every level starts from the same state: the resident systems just
        loaded under the budget (systems loaded by an earlier level's stream do
        not carry over)."""
        srv = mm.Server(n_slots=slots, mem_budget=int(resident_bytes * 1.15))
        for t in [srv.load(j, x) for j, x in enumerate(systems)]:
            wait(srv, t)
        return srv

    # one stream of requests, replayed at every arrival rate and one at a time
    # (each on a fresh server), so the levels differ only in the rate
    stream = make_requests(n_requests)
    srv = fresh_server(4)
    sat, _ = run_level(srv, stream, 0, 10_000)
    srv.close()
    log(f"[bench] saturated: {sat}")
    levels = {}
    for f in (0.5, 0.8, 0.95):
        srv = fresh_server(4)
        levels[f"{int(f * 100)}%"], _ = run_level(srv, stream, f * sat["req_per_s"], 10_000)
        srv.close()
        log(f"[bench] load {f}: {levels[f'{int(f * 100)}%']}")
    srv = fresh_server(1)
    srv.stats(reset=True)
    seq, next_id = stream, 10_000
    t0 = time.perf_counter()
    results = []
    for r in seq:
        if r[0] == "load":
            next_id += 1
        results.append((r, wait(srv, submit(srv, r, next_id))))
    wall = time.perf_counter() - t0
    st = srv.stats()
    one = {"requests": len(seq), "req_per_s": len(seq) / wall, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
           "evicted": st["evicted"], "reloaded": st["reloaded"], "by_kind": breakdown(results)}
    srv.close()
    log(f"[bench] one at a time: {one}")
    return {"workload": f"served{len(systems)}", "resident_systems": len(systems),
            "classes": int(sum(x.n_classes for x in systems)), "resident_gib": resident_bytes / 2**30,
            "levels": levels, "saturated": sat, "one_at_a_time": one}


def level_summary(v):
    """p50/p99 of every request of a load level, the rate reached, evictions,
    and p50/p99 of its edits and loads on their own."""
    out = {"p50": v["p50_ms"], "p99": v["p99_ms"], "req_per_s": v["req_per_s"],
           "evicted": v.get("evicted"), "reloaded": v.get("reloaded")}
    if v.get("offered_req_per_s"):
        out["offered_req_per_s"] = v["offered_req_per_s"]
    for kind, b in v.get("by_kind", {}).items():
        out[kind] = {"n": b["n"], "p50": b["p50_ms"], "p99": b["p99_ms"], "queue_p99": b["queue_p99_ms"],
                     "service_p99": b["service_p99_ms"]}
    return out


def bench_served(a, mm, synth):
    sv = served_leg(a, mm, synth, a.requests)
    out = {"metric": METRIC, "value": sv["saturated"]["req_per_s"], "unit": "requests/s", "n_gpus": 1,
           "steps": a.requests, "warmup": 0, "ms_per_step": 1000.0 / sv["saturated"]["req_per_s"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": sv["workload"], "resident_systems": sv["resident_systems"],
                      "classes": sv["classes"], "slots": 4,
                      "mix": "98% edit (1-500 methods, log-uniform), 2% load (1k-50k classes)",
                      "resident_gib": sv["resident_gib"]},
           "served_latency_ms": {**{k: level_summary(v) for k, v in sv["levels"].items()},
                                 "one_at_a_time": level_summary(sv["one_at_a_time"])},
           "levels": sv["levels"], "saturated": sv["saturated"], "one_at_a_time": sv["one_at_a_time"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()

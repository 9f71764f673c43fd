// mm_internal.h -- launch plans shared by the host engine and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm_dev.h"

namespace mm {

struct MapOut {
    const MapSeg *seg;
    int32_t *plen;      // per partition: number of keys written
    int32_t *pforeign;  // per partition (call-count map only): keys owned by another class
    int32_t *keys;
    int32_t *vals;
};

struct MetricsPlan {
    MethodAgg *meth;
    ClassAgg *cls;
    MapOut w, cnt, in;
    const int2 *w_items;
    int n_w_items;
    const int2 *cnt_items;
    int n_cnt_items;
    const int2 *in_items;        // every (method, partition) of the callers map
    const int32_t *in_wave_list; // the items grouped by a wave (long caller rows)
    int n_in_wave;
    const int2 *co_items;        // (class, row tile)
    int n_co_items;
    int *err;
};

struct ScorePlan {
    int32_t mode;          // MM_CAND_*
    int64_t n_cand;
    int32_t cm1;           // n_classes - 1 (ALL mode)
    const int32_t *cand_m; // EXPLICIT / REFERENCED
    const int32_t *cand_t;
    const int32_t *cand_e; // REFERENCED: index of the destination in the method's out run
    uint32_t mask;
    int32_t rule;
    const MethodAgg *meth;
    const ClassAgg *cls;
    MapView w, cnt, in;
    MethodPrep *prep;
    int32_t *outk, *outc, *outa;  // per-method out runs (class, references, accesses)
    int64_t *cand_off;            // [n + 1] REFERENCED offsets
    MoveRec *rec;
    int32_t *gcnt;                // [c + 1] candidates per destination needing co-access
    int64_t *goff;                // [c + 1]
    int32_t *gslot;               // [n_cand]
    int32_t *glist;               // [n_cand]
    int2 *heavy;                  // (candidate, partition) items for long caller lists
    int64_t heavy_cap;
    int32_t *heavy_count;
    int32_t *flags;               // [n_cand] keep flags for compaction
    int64_t *kpos;                // [n_cand + 1]
    int *err;
};

// scans (k_util.hip): out[i] = sum of in[0..i), out[n] = total; tmp >= scan_tmp_elems(n)
int64_t scan_tmp_elems(int64_t n);
void scan_i32(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);

void launch_compute_metrics(const DevSys &d, const MetricsPlan &p, hipStream_t st);

// score_moves phases (k_score.hip)
void launch_prep(const DevSys &d, const ScorePlan &p, int32_t *ref_count, hipStream_t st);
void launch_ref_fill(const DevSys &d, const ScorePlan &p, int32_t *cm, int32_t *ct, int32_t *ce, hipStream_t st);
void launch_deltas(const DevSys &d, const ScorePlan &p, int64_t *tmp, hipStream_t st);
void launch_keep(const DevSys &d, const ScorePlan &p, int keep_only, hipStream_t st);
void launch_compact(const ScorePlan &p, MoveRec *out, hipStream_t st);

}  // namespace mm

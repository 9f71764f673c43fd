// mm_internal.h -- launch plans shared by the host engine and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm_dev.h"

namespace mm {

// Optional per-kernel timing: HIP events recorded around a launch on its stream.
struct KTimer {
    virtual ~KTimer() {}
    virtual bool begin(const char *name, hipStream_t st) = 0;  // false: not timed
    virtual void end(hipStream_t st) = 0;
};

#define MM_TIMED(timer, name, st, ...)                              \
    do {                                                            \
        bool on_ = (timer) && (timer)->begin((name), (st));         \
        __VA_ARGS__;                                                \
        if (on_) (timer)->end(st);                                  \
    } while (0)

struct MapOut {
    MapHdr *hdr;
    int32_t *foreign;  // call-count map: keys owned by another class, per segment; caller map:
                       // callers in the method's own class, per method
    int32_t *keys;
    int32_t *vals;
};

// block ranges of lists of methods grouped by row length: group g holds
// methods [off[g], off[g+1]) of the list and blocks [blk[g], blk[g+1])
struct SegGrid {
    int off[6];
    int blk[6];
};

// the destination counts (c + 1 entries) are followed by the work-list counters
// (c + 2, c + 3), the kept-list length (c + 4) and its overflow mark (c + 5):
// one fill clears them all
constexpr int GCNT_TAIL = 6;

// Hash-table segments of more references than the LDS tiers take, built in two
// passes (k_big_stage, k_big_build). A fill item takes at most one item's worth
// of entries: entries [a, b) of the caller row of method seg (caller maps);
// members mem_idx[a .. b) of class seg (y < 0); or entries [a, b) of member y's
// row (its calls, then its accesses for W). j is its index among the segment's
// nI items; its distinct (key, count) pairs go to stage[stage ..] (room for b - a
// or the batch's entries), bucketed by partition; the segment's partition table
// holds np + 1 rows of nI words from word bt: row p, where bucket p starts in
// each item; row np, each item's total.
struct BigItem {
    int32_t seg, a, b, y, j, nI;
    int64_t stage, bt;
};
// partition p of segment seg, whose items are items[i0 .. i0 + nI)
struct BigPart {
    int32_t seg, p, i0, nI;
    int64_t bt;
};
struct BigMap {
    const BigItem *items;
    const BigPart *parts;
    int n_items, n_parts;
    int2 *stage;
    int32_t *bt;
    MapOut mo;
};
// the three maps' hash segments (W, CNT, caller maps) in one launch per pass
struct BigWork {
    BigMap m[3];
    int lds_slots;  // slots of an item's LDS table: a power of two >= 2 * the most entries of an item
    int np_max;     // most partitions of one segment
};
// LDS bytes k_big_stage takes beside its static arrays
inline size_t big_stage_lds(const BigWork &b) {
    return ((size_t)2 * b.lds_slots + (size_t)b.np_max + 1) * sizeof(int32_t);
}

// the W and CNT tables the full recompute groups in LDS by waves (k_map_tab_wc):
// items class * 4 + what (0: both tables of the class, 1: its W table, 2: its
// CNT table), those needing both LDS regions of a block first (n_large), then
// those fitting one (n_small)
struct MapWcWork {
    const int32_t *list;
    int n_large, n_small;
};

struct MetricsPlan {
    MethodAgg *meth;
    ClassAgg *cls;
    MethodAgg *meth_out;  // NULL, or a caller's buffer that also receives the method metrics
    ClassAgg *cls_out;    // NULL, or a caller's buffer that also receives the class metrics
    uint64_t *own_mask;
    MapOut w, cnt, in;
    const int32_t *in_wave;                      // caller tables grouped in LDS by a block
    int n_in_wave;
    MapWcWork wc;                                // W and CNT tables grouped in LDS by waves
    const int32_t *w_mid, *cnt_mid;              // W and CNT tables of MAP_CAP..MID_CAP references, grouped in LDS
    int n_w_mid, n_cnt_mid;                      //   by a block each
    BigWork big;                                 // hash-table segments of the three maps
    const int32_t *in_runs;                      // methods with 1..IN_SMALL callers, four groups by row
    int in_run_off[5];                           //   length (<=4, <=8, <=16, <=32); group g = [off[g], off[g+1])
    const int4 *in_flag_items;                   // {method, first slot, end slot} of large caller maps
    int n_in_flag;
    const int2 *co_items;                        // (class, row tile) of classes with more than 64 own attributes
    int n_co_items;
    const int2 *co_groups;                       // (class, first of four row tiles): more than 64 methods,
    int n_co_groups;                             //   at most 64 own attributes
    const int32_t *co_small;                     // classes of at most 64 methods and 1..64 own attributes
    int n_co_small;
    const int32_t *fin_list;                     // every class: those of at most 64 members, then the others
    int n_fin_small, n_fin_large;
    int *err;
    KTimer *timer;
};

// Device arrays a patch may write (k_scatter): op {target, index, value}
enum { PATCH_OWNER = 0, PATCH_MEM_IDX = 1, PATCH_MEM_OFF = 2, PATCH_MEM_END = 3, PATCH_W_HDR = 4, PATCH_CNT_HDR = 5,
       PATCH_IN_HDR = 6, PATCH_PREP = 7, PATCH_TARGETS = 8 };
struct PatchTargets {
    int32_t *t[PATCH_TARGETS];  // owner, mem_idx, mem_off, mem_end, W / CNT / caller-map headers as int32
                                // words, the methods grouped by row length
};

// Rows of edited methods replaced on the device: the new row lengths of every
// method (launch_edit_lengths), their prefix sums (pa, pc), then every row
// copied to its new place from the old rows or the uploaded new ones
// (launch_edit_copy, which also writes the new int32 offsets).
struct EditRows {
    int n, k;
    const int32_t *meth;                   // edited methods, ascending
    const int32_t *e_acc_off, *e_acc_idx;  // their new rows (k + 1 offsets into the uploaded rows)
    const int32_t *e_call_off, *e_call_idx;
    const int32_t *acc_off, *acc_idx, *call_off, *call_idx;  // rows before the edit
    int32_t *len_acc, *len_call;           // [n] row lengths after the edit
};
void launch_edit_lengths(const EditRows &e, hipStream_t st);
// caller maps an incremental recompute reaches (k_incr.hip): marks from a list,
// marks of the loss flags that W changes reach, then the marked methods filed
// by caller-map kind (lists at q * stride: q = 0 hash-table segments, 1..4 run
// groups, 5 tables grouped in LDS; counts[q] their lengths,
// zero on entry; marks cleared)
void launch_incr_mark(const int32_t *list, int n, uint8_t *mark, hipStream_t st);
void launch_incr_flag_walk(const DevSys &d, const int32_t *classes, int n_classes, const uint8_t *key_class,
                           uint8_t *mark, hipStream_t st);
void launch_incr_in_lists(const DevSys &d, const MapHdr *in_hdr, uint8_t *mark, int32_t *lists, int64_t stride,
                          int32_t *counts, hipStream_t st);

// flag[X] = 1 for the classes owning a caller of methods[0 .. k) (flag cleared by the caller)
void launch_caller_classes(const DevSys &d, const int32_t *methods, int k, int32_t *flag, hipStream_t st);
void launch_edit_copy(const EditRows &e, const int64_t *pa, const int64_t *pc, int32_t *acc_off, int32_t *acc_idx,
                      int32_t *call_off, int32_t *call_idx, hipStream_t st);

// Recompute of the segments, methods and classes a set of moves touched
// (launch_dirty_metrics). The W and CNT tables of at most MAP_HMAX slots are
// grouped in LDS by waves (lists as for k_map_tab_sep, larger tables first),
// those of at most MID_HMAX by a block each (*_mid); larger ones are built by
// the fill items and partitions in `big`. Caller maps: runs by length group
// (in_runs, in_run_off), tables grouped in LDS (in_wave), larger tables built
// in `big` and flagged (in_flag).
struct DirtyPlan {
    MethodAgg *meth;
    ClassAgg *cls;
    uint64_t *own_mask;
    MapOut w, cnt, in;
    const int32_t *w_list, *c_list;
    int n_w, n_w_large, n_c, n_c_large;
    const int32_t *w_mid, *c_mid;
    int n_w_mid, n_c_mid;
    BigWork big;
    const int32_t *basic;
    int n_basic, n_basic_zero;
    const int32_t *co_small;
    int n_co_small;
    const int2 *co_groups, *co_items;
    int n_co_groups, n_co_items;
    const int32_t *in_wave;
    int n_in_wave;
    const int32_t *in_runs;
    int in_run_off[5];
    const int4 *in_flag;
    int n_in_flag;
    const int32_t *fin;
    int n_fin;
    int *err;
    KTimer *timer;
};

// apply n patch ops (k_scatter); then the recompute of a DirtyPlan
void launch_patch(const int4 *ops, int n, const PatchTargets &t, hipStream_t st);
void launch_dirty_metrics(const DevSys &d, const DirtyPlan &p, hipStream_t st);

struct ScorePlan {
    int32_t mode;          // MM_CAND_*
    int32_t rule;
    uint32_t mask;
    int32_t keep_only;
    int64_t n_cand;
    int32_t cm1;           // n_classes - 1 (ALL mode)
    const MethodAgg *meth;
    const ClassAgg *cls;
    const uint64_t *own_mask;
    MapView w, cnt, in;
    const int32_t *in_own;        // [n] callers of each method in its own class
    MethodPrep *prep;
    const int32_t *prep_runs;     // methods by row length (calls + accesses): <= 8, 16, 32, 64, longer
    int32_t prep_run_off[6];      //   group g = [prep_run_off[g], prep_run_off[g + 1])
    int32_t *outk, *outc, *outa;  // per-method out runs (class, references, accesses)
    int64_t *cand_off;            // [n + 1] REFERENCED offsets
    int32_t *cm, *ct, *ce;        // EXPLICIT / REFERENCED candidates (ce: place of (cm, ct)'s out entry in the out arrays)
    int32_t *gcnt;                // [c + 1] candidates per destination needing co-access
    int64_t *goff;                // [c + 1]
    int32_t *gslot;               // [n_cand] slot in the destination's list, or, when grouped, [out entries]
    int32_t grouped;              // 1: k_prep counted and k_ref_fill filled the destination lists
    int64_t compact_cap;          // k_compact writes nothing when more than this many records are kept
    int32_t origin;               // 0: any origin; 1 / 2: only origins whose LCOM / CBO is above the class average
    const long long *origin_sum;  // sum of that metric over the classes (device)
    int32_t lazy_src;             // 1: the origin-class CBO/RFC terms are left to k_delta's survivors
    int32_t prep_in_late;         // 1: k_prep leaves the caller terms to k_prep_in (it runs before the caller maps)
    int32_t *glist;               // [n_cand]
    int32_t *hval;                // [n_cand] h_T(m) of the grouped candidates
    MoveRec *rec;
    int32_t *flags;               // [n_cand] keep flags (keep_only)
    int64_t *kpos;                // [n_cand + 1]
    long long *kept_out;          // NULL, or where k_compact / k_kept_order store the kept count
    int32_t *status_dev;          // NULL, or host-mapped {err, pad, kept (int64)} that k_kept_order fills
    int32_t *kept_idx;            // NULL, or the unordered list of kept candidates (keep_only into a caller buffer)
    int32_t *kept_count;          //   its length
    int32_t *kept_over;           //   set when a kept candidate found the list full
    int64_t kept_cap;
    int2 *heavy;                  // (candidate, chunk) items for long caller-class lists
    int64_t heavy_cap;
    int32_t *heavy_count;
    int32_t *hcand;               // candidates with long caller-class lists
    int64_t hcand_cap;
    int32_t *hcand_count;
    int *err;
    KTimer *timer;
    // schedule (autotuned; results do not depend on it)
    int32_t caller_light;         // caller classes handled inline by the delta kernel
    int32_t heavy_chunk;          // caller-class slots per heavy work item
    int32_t delta_chunk;          // 0: one lane per candidate; else candidates per dynamic fetch
    int32_t delta_grid;           // workgroups of the persistent delta kernel
    int32_t *delta_next;          // fetch counter of the persistent delta kernel
};

// Similarity of method pairs (k_sim.hip).
enum { SIM_STATS = 0, SIM_COUNT = 1, SIM_PAIRS = 2 };
constexpr int SIM_HIST = 1024;        // union sizes binned in LDS (larger ones: global atomics)
constexpr int SIM_BITS_WORDS = 8192;  // LDS bitmap: classes (count) or partner methods (pairs), 2^18 bits

struct SimPlan {
    int32_t mode;                  // SIM_*
    int32_t cw;                    // bitmap words per row of cand_bits
    const int64_t *at_off;         // [na + 1] accessors of each attribute
    const int32_t *at_idx;
    const int32_t *deg;            // [n] properties of each method
    int32_t *dense;                // [grid * n] per-workgroup counters, zero between rows
    int32_t *cnt2;                 // [grid * n] per-workgroup shared counts of high partners (pairs)
    int32_t *ticket;               // row counter of the persistent grid
    unsigned long long *hist;      // [umax + 1] sum of shared counts by union size (stats)
    unsigned long long *nnz;       // pairs with a shared property (stats)
    const int32_t *imin;           // [umax + 1] least shared count of a high pair, by union size
    int32_t *row_pairs;            // [n] high pairs (r, y > r) per row
    int32_t *row_cands;            // [n] candidate classes per row
    uint32_t *cand_bits;           // [n * cw] candidate classes per row
    const int64_t *pair_off;       // [n + 1] output offsets of the rows' pairs
    int4 *pairs;                   // (m1, m2, shared, union)
    int64_t out_cap;               // entries of `pairs` (pairs) or of the candidate lists (emit)
    KTimer *timer;
};

void launch_at_build(const DevSys &d, const int64_t *at_off, int32_t *cnt_or_cur, int32_t *at_idx, int pass,
                     hipStream_t st);
void launch_sim_deg(const DevSys &d, int32_t *deg, hipStream_t st);
void launch_sim_rows(const DevSys &d, const SimPlan &p, int grid, hipStream_t st);
void launch_sim_emit(const DevSys &d, const SimPlan &p, const int64_t *cand_off, int32_t *cm, int32_t *ct,
                     hipStream_t st);

// Work area of the single-pass scan (k_util.hip): a ticket word, then one
// status word per tile; the host side keeps the ticket base and the epoch.
struct ScanArea {
    int64_t *dev = nullptr;
    int64_t cap_words = 0;
    uint32_t scans = 0;        // scans launched since the area was cleared (the device epoch)
    bool need_clear = true;    // a new area, or one a failed scan left behind
    int *err = nullptr;        // ERR_SCAN is or-ed here
};
constexpr uint32_t SCAN_EPOCHS = 0xff00u;  // scans between clears (the status words carry 16 epoch bits)

// scans: out[i] = sum of in[0..i), out[n] = total; the area holds >= scan_area_elems(n) words
int64_t scan_area_elems(int64_t n);
void scan_i32(const int32_t *in, int64_t *out, int64_t n, ScanArea &a, hipStream_t st, KTimer *t = nullptr);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, ScanArea &a, hipStream_t st, KTimer *t = nullptr);
// two independent scans in one launch; the area holds >= scan_area_elems(n1) + scan_area_elems(n2) words
void scan2_i32(const int32_t *in1, int64_t *out1, int64_t n1, const int32_t *in2, int64_t *out2, int64_t n2,
               ScanArea &a, hipStream_t st, KTimer *t = nullptr);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);

// Streams that run independent kernels of a phase beside the calling stream
// (all at the default priority), and the events that fork and join them.
struct AuxStreams {
    hipStream_t s[3];
    hipEvent_t ev[8];
};

// reverse call rows: pass 0 counts callers into cnt; pass 1 (after the prefix
// sum off64 of cnt) writes rc_off and fills rc_idx, using cnt as the cursor
void launch_edge_rows(const DevSys &d, int32_t *rows, hipStream_t st);
void launch_rc_bounds(const int32_t *callee_sorted, int64_t nnz, int n, int32_t *rc_off, hipStream_t st);
hipError_t callers_sort(void *tmp, size_t &tmp_bytes, const int32_t *callee_in, int32_t *callee_out,
                        const int32_t *caller_in, int32_t *caller_out, int64_t nnz, int n, hipStream_t st);

// ax == nullptr: every kernel on st, in order
void launch_compute_metrics(const DevSys &d, const MetricsPlan &p, hipStream_t st, const AuxStreams *ax = nullptr);

// score_moves phases (k_score.hip)
void launch_prep(const DevSys &d, const ScorePlan &p, int32_t *ref_count, hipStream_t st);
// the class of every call, access and caller entry, and the rank of every
// access's attribute in its class (DevSys::call_cls, acc_cls, rc_cls, acc_rank)
void launch_entry_classes(const DevSys &d, int64_t ncall, int64_t nacc, int32_t *call_cls, int32_t *acc_cls,
                          int32_t *rc_cls, int32_t *acc_rank, hipStream_t st);
// after moves (owners changed, rows not): the entries naming each moved method
// take its current class, call_cls in its callers' rows and rc_cls in its
// callees' caller rows
constexpr int ENTRY_MOVES_MAX = 256;
struct EntryMoves {
    int32_t n;
    int32_t m[ENTRY_MOVES_MAX];
};
void launch_entry_moves(const DevSys &d, const EntryMoves &mv, int32_t *call_cls, int32_t *rc_cls, hipStream_t st);
// the caller terms of the prep records (after launch_prep and the caller maps)
void launch_prep_in(const DevSys &d, const ScorePlan &p, hipStream_t st);
void launch_ref_fill(const DevSys &d, const ScorePlan &p, hipStream_t st);
void launch_score(const DevSys &d, const ScorePlan &p, ScanArea &scan, hipStream_t st);
void launch_compact(const ScorePlan &p, MoveRec *out, hipStream_t st);
// kept records of a short kept list, in candidate order, into out (nothing when
// they do not fit); the count goes to kept_out
constexpr int KEPT_FAST_MAX = 2048;
void launch_kept_order(const ScorePlan &p, MoveRec *out, hipStream_t st);
// ranked suggestions (k_rank.hip)
void launch_class_sum(const ClassAgg *cls, int c, int which, long long *sum, hipStream_t st);
void launch_rank_keys(const MoveRec *rec, int64_t n, const MethodAgg *meth, int kind, uint32_t *key, int32_t *idx,
                      hipStream_t st);
void launch_rank_gather(const MoveRec *rec, const int32_t *idx, int64_t n, MoveRec *out, hipStream_t st);
constexpr int IND_MAX_CLASSES = 16384 * 32;
void launch_independent(const MoveRec *rec, int64_t n, const MapView &in, int c, MoveRec *out, int64_t *count,
                        hipStream_t st);
hipError_t rank_sort(void *tmp, size_t &tmp_bytes, const uint32_t *key_in, uint32_t *key_out, const int32_t *idx_in,
                     int32_t *idx_out, int64_t n, hipStream_t st);
void launch_affected_mark(const ScorePlan &p, int m, int S, int T, int n_slots, int32_t *flag, int32_t *dval,
                          hipStream_t st);
// WMC, NOC, DIT (k_ck.hip). launch_ck_hierarchy: NOC and DIT of a hierarchy
// (anc, anc2, dep2: c-entry work arrays; ERR_CYCLE or-ed into err on a cycle).
int ck_rounds(int64_t c);
void launch_ck_hierarchy(const int32_t *parent, int c, int32_t *noc, int32_t *dit, int32_t *anc, int32_t *anc2,
                         int32_t *dep2, int *err, hipStream_t st);
void launch_ck_class(const DevSys &d, const int32_t *weight, const int32_t *noc, const int32_t *dit, CkOut *out,
                     hipStream_t st);

// classes with flag set go to cls/dcbo[pos[X]] when below cap; n_out (NULL:
// not written) receives pos[c], the number of flagged classes
void launch_affected_out(const int32_t *flag, const int32_t *dval, const int64_t *pos, int c, int64_t cap,
                         int32_t *cls, int32_t *dcbo, int64_t *n_out, hipStream_t st);

}  // namespace mm

/*
 * mm.h -- C ABI of the MI355X Move-Method metric engine.
 *
 * The library follows the paper's statement of the problem ("Using Modularity
 * Metrics to assist Move Method Refactoring of Large Systems"):
 *   input  -- the classes of a system with their methods and attributes, and for
 *             every method the methods it invokes and the attributes it accesses,
 *             all as numeric ids (Sec. IV-B, the Inspector's lists; Sec. IV-C, the
 *             cls and dpnd arrays handed to the GPU);
 *   output -- per-method and per-class modularity metrics (Sec. II: fan-in,
 *             fan-out, CBO, LCOM in its original pair-count form and in its later
 *             ratio form, and RFC from the CK suite named there), and candidate
 *             Move Method refactorings scored by their exact metric deltas, kept
 *             when they improve some classes and worsen none (abstract, Sec. III-A,
 *             Sec. IV-A).
 *
 * Conventions
 *   - Every call returns mm_status: MM_OK (0) or a negative error code. No C++
 *     exception crosses this boundary. mm_last_error() returns a thread-local
 *     message describing the last failure on the calling thread.
 *   - All ids are int32 and 0-based. Host arrays passed in are copied; the caller
 *     keeps ownership and may free them when the call returns.
 *   - A system is used by one host thread at a time. Work is ordered on the
 *     context's HIP stream; host-output calls return after their results are in
 *     host memory, device-output calls return once their work is enqueued (and,
 *     for variable-size outputs, once the count is known).
 *   - Lower is better for every metric: "improve" is a delta < 0, "worsen" > 0.
 *
 * Metric definitions (rows are read as sets; a self-call is kept)
 *   fan_in(m)   number of methods calling m                        Sec. II-A
 *   fan_out(m)  number of methods m calls                          Sec. II-A
 *   CBO(C)      number of other classes whose methods C's methods call or whose
 *               attributes they access (efferent)                  Sec. II-B
 *   LCOM(C)     P - Q, P = pairs of C's methods sharing no attribute of C,
 *               Q = pairs sharing at least one; not clamped at 0    Sec. II-B
 *   LCOM_HS(C)  (n*a - U) / (n*a), U = sum over C's methods of the number of C's
 *               attributes each uses; returned as the exact integer pair
 *               (hs_num, hs_den), (0, 1) when n*a = 0               Sec. II-B
 *   RFC(C)      |M_C union (methods called by M_C)|, one level      Sec. II-B
 *
 * A move (m -> T) changes only the owner of m: attributes stay where they are,
 * ids do not change, m keeps its calls and accesses, nothing is left behind in
 * the origin class S. The classes it can affect are S, T and the classes owning
 * a caller of m (whose CBO may change); fan-in and fan-out never change.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mm_status;

#define MM_OK 0
#define MM_EINVAL (-1)      /* bad argument: NULL, id out of range, bad offsets, dst == src, bad mask/rule */
#define MM_EOVERFLOW (-2)   /* a count does not fit the library's int32 / int64 fields */
#define MM_ENOMEM (-3)      /* device allocation failed or the context's memory budget would be exceeded */
#define MM_EHIP (-4)        /* a HIP runtime call failed */
#define MM_ERANGE (-5)      /* output capacity too small; *n_out holds the required count */
#define MM_EBUSY (-6)       /* the server refused a request (queue full or admission) */
#define MM_EINTERNAL (-7)   /* an internal limit was hit (message says which) */
#define MM_ENOTFOUND (-8)   /* unknown ticket or system handle */

/* metric_mask bits */
#define MM_CBO 1u
#define MM_LCOM_PQ 2u
#define MM_LCOM_HS 4u
#define MM_RFC 8u

/* rules */
#define MM_RULE_PARETO 0     /* every affected (class, masked metric) delta <= 0 and one < 0 */
#define MM_RULE_PAPER_LCOM 1 /* each masked LCOM form improves in both origin and destination (Sec. III-A) */
#define MM_RULE_PAPER_CBO 2  /* origin CBO lowered, destination CBO not higher (Sec. III-A), no caller class worse */

/* candidate sets */
#define MM_CAND_EXPLICIT 0   /* caller-supplied (method, class) pairs */
#define MM_CAND_ALL 1        /* every method into every other class (the worst case of Sec. III-B) */
#define MM_CAND_REFERENCED 2 /* every class owning a method m calls or an attribute m accesses (Sec. III-A) */
#define MM_CAND_SIMILAR 3    /* moves suggested by high-similarity method pairs (Sec. III-A; see
                                mm_similarity); the threshold is mm_set_similarity_threshold's */

typedef struct mm_context mm_context;
typedef struct mm_system mm_system;

/* A system in CSR form. acc_off / call_off have n_methods + 1 entries, start at 0
 * and are non-decreasing; row i of acc_idx lists attribute ids accessed by method
 * i, row i of call_idx the method ids it calls. Rows may be unsorted and may
 * repeat ids (they are read as sets). Every class id is in [0, n_classes). */
typedef struct {
    int32_t n_classes, n_methods, n_attrs;
    const int32_t *method_class; /* [n_methods] owner class of every method */
    const int32_t *attr_class;   /* [n_attrs]   owner class of every attribute */
    const int64_t *acc_off;      /* [n_methods + 1] */
    const int32_t *acc_idx;      /* [acc_off[n_methods]] */
    const int64_t *call_off;     /* [n_methods + 1] */
    const int32_t *call_idx;     /* [call_off[n_methods]] */
} mm_system_desc;

typedef struct {               /* 48 bytes */
    int32_t n_methods, n_attrs, cbo, rfc;
    int64_t lcom_p, lcom_q;    /* LCOM = lcom_p - lcom_q */
    int64_t hs_num, hs_den;    /* LCOM_HS = hs_num / hs_den */
} mm_class_metrics;

typedef struct {               /* 16 bytes */
    int32_t fan_in, fan_out;
    int32_t own_attr_uses;          /* attributes of its own class the method accesses */
    int32_t own_coaccess_partners;  /* other methods of its class sharing one of them */
} mm_method_metrics;

typedef struct {               /* 96 bytes; deltas are after - before */
    int32_t method, src, dst;
    int32_t d_cbo_src, d_cbo_dst, d_rfc_src, d_rfc_dst;
    int32_t n_caller_cls;      /* classes other than src/dst owning a caller of method */
    int32_t n_caller_worse;    /* ... whose CBO rises */
    int32_t n_caller_better;   /* ... whose CBO falls */
    int32_t keep, pad;
    int64_t d_lcom_src, d_lcom_dst;
    int64_t hs_num_src, hs_den_src, hs_num_dst, hs_den_dst; /* LCOM_HS after the move */
} mm_move_score;

/* Replace the rows (and optionally the owner) of k methods. */
typedef struct {
    int32_t k;
    const int32_t *method;     /* [k] distinct method ids */
    const int32_t *new_class;  /* [k] new owner, or NULL to keep the owners */
    const int64_t *acc_off;    /* [k + 1] */
    const int32_t *acc_idx;
    const int64_t *call_off;   /* [k + 1] */
    const int32_t *call_idx;
} mm_edit_desc;

typedef struct {
    int32_t n_classes, n_methods, n_attrs, pad;
    int64_t nnz_acc, nnz_call;   /* after removing repeated ids */
    int64_t device_bytes;        /* device memory held by the system */
    int64_t version;             /* bumped by every apply_move / apply_edit */
} mm_system_info;

/* ---- context --------------------------------------------------------------
 * mm_context_create: selects HIP device `device`. If hip_stream is non-NULL the
 * context borrows that stream (e.g. torch.cuda.current_stream().cuda_stream);
 * otherwise it creates and owns one. mem_budget_bytes caps the device memory
 * all systems of the context may hold (0 = no cap). Errors: MM_EINVAL (NULL out,
 * bad device), MM_EHIP. */
mm_status mm_context_create(int32_t device, void *hip_stream, uint64_t mem_budget_bytes, mm_context **out);
/* Frees the context. Its systems must have been freed first (MM_EBUSY if not). */
mm_status mm_context_destroy(mm_context *ctx);
/* Message of the last failure on this thread ("" if none). Valid until the next
 * failing call on this thread. */
const char *mm_last_error(void);
/* Device memory currently held by the context's systems and work buffers. */
mm_status mm_context_memory(mm_context *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* ---- kernel timing (tracing) ------------------------------------------------
 * mm_context_set_timing: records HIP events around the launches of the named
 * kernels on the context stream. kernels: NULL or "" turns timing off, "*" times
 * every kernel, otherwise a comma-separated list of kernel names (e.g.
 * "k_delta,k_map_tab_wc"). Timing adds two event records per timed launch.
 * With "*" a metric recompute runs its two kernel chains one after the other on
 * the context stream, so each kernel's time is its own execution; with a list of
 * names the chains stay concurrent (a timed kernel's time then includes waiting
 * behind kernels of the other chain).
 * mm_context_timing: per-kernel totals since the last reset; writes up to cap
 * entries to out (may be NULL to count), *n = number of kernels with samples.
 * Synchronizes with the timed work. name points to static storage. */
typedef struct {
    const char *name;
    int64_t launches;
    double total_ms;
} mm_kernel_time;
mm_status mm_context_set_timing(mm_context *ctx, const char *kernels);
mm_status mm_context_timing(mm_context *ctx, mm_kernel_time *out, int32_t cap, int32_t *n, int32_t reset);

/* ---- schedule tuning ---------------------------------------------------------
 * Knobs of the scoring schedule. They change speed only: every result is the
 * same under any valid setting.
 *   caller_light  caller classes of a method handled inline per candidate; more
 *                 go to a wave-parallel pass (>= 0)
 *   heavy_chunk   caller-class slots per work item of that pass (>= 1)
 *   delta_chunk   0: one lane per candidate; > 0: a persistent grid of
 *                 delta_grid workgroups fetching this many candidates at a time
 *   delta_grid    workgroups of the persistent form (0: 8 per compute unit)
 * and of the metric recompute's layout (taken at the next full recompute):
 *   fill_chunk    most entries per fill item of the hash-table segments
 *                 (the tables of the largest classes and caller lists; 0:
 *                 automatic, about 2,048 items in all of 256-1,024 entries;
 *                 else 64..2048)
 *   fill_group    no effect (>= 0): every fill item groups its keys in LDS
 * mm_context_set_tuning(ctx, NULL) restores the defaults. mm_autotune times the
 * scoring call described by its arguments (as for mm_score_moves) under a set of
 * scoring schedules, then the whole step (a full metric recompute and that call)
 * under a set of fill schedules, `repeats` times each, keeps the fastest in the
 * context and returns it in *best (may be NULL). Errors: as mm_score_moves. */
typedef struct {
    int32_t caller_light, heavy_chunk, delta_chunk, delta_grid;
    int32_t fill_chunk, fill_group;
} mm_tuning;
mm_status mm_context_set_tuning(mm_context *ctx, const mm_tuning *t);
mm_status mm_context_get_tuning(mm_context *ctx, mm_tuning *t);
mm_status mm_autotune(mm_system *sys, int32_t cand_mode, const int32_t *cand_method, const int32_t *cand_class,
                      int64_t n_cand, uint32_t metric_mask, int32_t rule, int32_t keep_only, int32_t repeats,
                      mm_tuning *best);

/* ---- load_system ----------------------------------------------------------
 * Validates and copies a system to the device (Sec. IV-C: one upload, then the
 * data stays resident), removing repeated ids from rows and building the callers
 * of every method. Errors: MM_EINVAL (NULL pointers with non-zero sizes, ids out
 * of range, offsets not starting at 0, decreasing, or not matching the arrays),
 * MM_EOVERFLOW (more than 2^31-1 ids in a row array), MM_ENOMEM, MM_EHIP. */
mm_status mm_load_system(mm_context *ctx, const mm_system_desc *desc, mm_system **out);
mm_status mm_free_system(mm_system *sys);

/* ---- batches ----------------------------------------------------------------
 * mm_load_batch loads n_sys independent systems as one system handle: their
 * disjoint union, with the classes, methods and attributes of part i shifted to
 * start after those of parts 0..i-1. Every metric and every score equals that of
 * the part on its own (no reference crosses parts), while each kernel phase runs
 * once over all parts. Records use the shifted ids; mm_system_parts returns the
 * offsets ([n_parts + 1] each; arrays may be NULL) to map them back. Scoring a
 * batch accepts MM_CAND_REFERENCED and MM_CAND_EXPLICIT (pairs within one part);
 * MM_CAND_ALL is refused (MM_EINVAL) since it would pair parts. A plain system
 * reports one part. Errors: as mm_load_system, per part. */
mm_status mm_load_batch(mm_context *ctx, const mm_system_desc *descs, int32_t n_sys, mm_system **out);
mm_status mm_system_parts(mm_system *sys, int32_t *n_parts, int32_t *class_off, int32_t *method_off,
                          int32_t *attr_off);
mm_status mm_system_info_get(mm_system *sys, mm_system_info *out);

/* ---- compute_metrics ------------------------------------------------------
 * Computes every metric of Sec. II for all classes and methods of the system's
 * current state (after any moves and edits). out_cls ([n_classes]) and out_m
 * ([n_methods]) are host buffers owned by the caller; either may be NULL to skip
 * the copy. Errors: MM_EINVAL, MM_EHIP, MM_EINTERNAL. */
mm_status mm_compute_metrics(mm_system *sys, mm_class_metrics *out_cls, mm_method_metrics *out_m);
/* Same, writing caller-owned device buffers (either may be NULL) on the context
 * stream; returns once the work is enqueued. */
mm_status mm_compute_metrics_device(mm_system *sys, mm_class_metrics *d_cls, mm_method_metrics *d_m);

/* ---- score_moves ----------------------------------------------------------
 * Scores candidate moves by their exact deltas on every affected class (Sec.
 * III-A; Sec. IV-C assesses a move by re-running the metrics on the changed
 * membership, which these deltas equal). Metrics are recomputed first if the
 * system changed since the last compute.
 *   cand_mode     MM_CAND_EXPLICIT (cand_method/cand_class, n_cand entries, every
 *                 dst different from the method's current class), MM_CAND_ALL,
 *                 MM_CAND_REFERENCED or MM_CAND_SIMILAR (cand_* ignored; order:
 *                 method ascending, then class ascending).
 *   metric_mask   subset of MM_CBO | MM_LCOM_PQ | MM_LCOM_HS | MM_RFC used by rule.
 *   rule          MM_RULE_*; PAPER_LCOM needs an LCOM bit, PAPER_CBO needs MM_CBO.
 *   keep_only     0: one record per candidate, in candidate order, keep = 0/1;
 *                 1: only kept records, still in candidate order.
 *   out           host array of out_capacity records, or NULL to query the count.
 *   n_out         receives the number of records the call produces.
 * Errors: MM_EINVAL, MM_ERANGE (out non-NULL and out_capacity < *n_out; nothing
 * written), MM_ENOMEM, MM_EHIP, MM_EINTERNAL. A query with out == NULL followed by
 * the same call with a buffer reuses the device results of the query. */
mm_status mm_score_moves(mm_system *sys, int32_t cand_mode, const int32_t *cand_method,
                         const int32_t *cand_class, int64_t n_cand, uint32_t metric_mask,
                         int32_t rule, int32_t keep_only, mm_move_score *out,
                         int64_t out_capacity, int64_t *n_out);
/* Same, writing a caller-owned device buffer d_out; cand_method / cand_class stay
 * host arrays. Returns once the results are enqueued on the context stream. */
mm_status mm_score_moves_device(mm_system *sys, int32_t cand_mode, const int32_t *cand_method,
                                const int32_t *cand_class, int64_t n_cand, uint32_t metric_mask,
                                int32_t rule, int32_t keep_only, mm_move_score *d_out,
                                int64_t out_capacity, int64_t *n_out);

/* Per-class detail behind a record's caller counts (Sec. II-B defines CBO; Sec.
 * IV-A asks that no other class gets worse): for the move of `method` to
 * dst_class, every class X other than the method's class and dst_class that
 * holds a caller of the method, in ascending class order, with the change of X's
 * CBO (-1, 0 or +1). Their number equals the record's n_caller_cls, the +1 and
 * -1 entries its n_caller_worse and n_caller_better.
 *   cls, d_cbo  host arrays of `capacity` entries, or cls == NULL to query *n.
 *   n           receives the number of caller classes.
 * Errors: MM_EINVAL (NULL n, id out of range, dst_class == current owner, cls
 * without d_cbo), MM_ERANGE (capacity < *n; nothing written), MM_ENOMEM, MM_EHIP. */
mm_status mm_move_affected(mm_system *sys, int32_t method, int32_t dst_class, int32_t *cls,
                           int32_t *d_cbo, int64_t capacity, int64_t *n);

/* For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The result of
 * mm_move_affected, written to caller-owned DEVICE buffers, by a call that
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and
 * does not wait for the device: the work is enqueued on the context's stream
 * and the call returns.
 *   d_cls, d_cbo  device arrays of `capacity` entries (may be NULL when capacity
 *                 is 0): the caller classes in ascending order and each one's CBO
 *                 change; entries past `capacity` are not written.
 *   d_n           device int64 receiving the number of caller classes (compare
 *                 it with capacity once the stream has reached this point).
 * Working memory is one library-wide array of MM_NOALLOC_SCRATCH_BYTES per GPU,
 * held by each GPU the library runs on until the process ends. Every call on a
 * GPU uses that GPU's array, so calls that overlap on one GPU (from two host
 * threads, or on two streams not ordered against each other) race and give
 * wrong results; calls ordered on one stream do not.
 * The system's metrics must be current (mm_compute_metrics, which may allocate,
 * after the last load, move or edit).
 * Errors: MM_EINVAL (NULL d_n, capacity < 0, NULL arrays with capacity > 0, id
 * out of range, dst_class == current owner, more than MM_NOALLOC_MAX_CLASSES
 * classes, metrics not current), MM_EHIP (the array's device address is
 * unknown, or a launch failed). Kernel errors are reported by the next call
 * that waits for the device. */
#define MM_NOALLOC_MAX_CLASSES 1048576
#define MM_NOALLOC_SCRATCH_BYTES 16781824
mm_status mm_move_affected_noalloc(mm_system *sys, int32_t method, int32_t dst_class, int32_t *d_cls,
                                   int32_t *d_cbo, int64_t capacity, int64_t *d_n);

/* ---- similarity of method pairs ------------------------------------------
 * The properties of a method are the methods it calls and the attributes it
 * accesses (its two rows, as sets; a self-call is a property like any other
 * call). The Jaccard similarity of two methods is |shared| / |union| of their
 * property sets, 0 when the union is empty (Sec. II-A; the all-pairs count of
 * Sec. III-B). A pair is "high" (Sec. III-A and its footnote) under threshold
 *   MM_SIM_NONZERO       similarity > 0 (the pairs that share a property)
 *   MM_SIM_ABOVE_AVG     similarity > the average over all n(n-1)/2 pairs,
 *                        zeros included (the default)
 *   MM_SIM_ABOVE_AVG_NZ  similarity > the average over the pairs with similarity > 0
 * The averages are exact fractions and the comparison is exact (no rounding).
 * MM_CAND_SIMILAR: for every high pair whose methods sit in different classes,
 * each method may move to the other's class or to a class owning a method it
 * calls; (method, class) ascending, each once. A batch (mm_load_batch) refuses
 * similarity: its average would mix systems. */
#define MM_SIM_NONZERO 0
#define MM_SIM_ABOVE_AVG 1
#define MM_SIM_ABOVE_AVG_NZ 2

typedef struct {
    int32_t m1, m2;              /* m1 < m2 */
    int32_t shared, uni;         /* |shared| and |union| of the property sets */
} mm_sim_pair;

typedef struct {
    int64_t n_pairs;             /* n(n-1)/2 */
    int64_t n_nonzero;           /* pairs sharing a property */
    int64_t n_high;              /* pairs above the threshold */
    int64_t n_candidates;        /* MM_CAND_SIMILAR moves under the threshold */
    int32_t threshold;
    int32_t max_union;           /* bound on |union| (twice the longest property set) */
    double average;              /* the threshold's average, rounded to double (0 for NONZERO) */
} mm_sim_stats;

/* Counts of the similarity pairs and candidates under `threshold`; always
 * recomputed (MM_CAND_SIMILAR reuses the last computation of the same version).
 * Errors: MM_EINVAL (bad threshold, batch), MM_EOVERFLOW (more than 2^18
 * classes, or union sizes so varied that the exact average exceeds 8192 bits),
 * MM_ENOMEM, MM_EHIP. */
mm_status mm_similarity(mm_system *sys, int32_t threshold, mm_sim_stats *out);
/* The high pairs under `threshold`, (m1, m2) ascending; out == NULL queries *n.
 * Errors as mm_similarity, plus MM_ERANGE (capacity < *n; nothing written) and
 * MM_EOVERFLOW for more than 2^18 methods. */
mm_status mm_similarity_pairs(mm_system *sys, int32_t threshold, mm_sim_pair *out, int64_t capacity,
                              int64_t *n);
/* Threshold used by MM_CAND_SIMILAR from now on (default MM_SIM_ABOVE_AVG). */
mm_status mm_set_similarity_threshold(mm_system *sys, int32_t threshold);

/* ---- ranked suggestions ------------------------------------------------------
 * The suggestion procedures of Sec. III-A, each a scoring pass with the paper's
 * rule followed by an order (kept records only):
 *   MM_SUGGEST_LCOM     moves out of classes with a high LCOM (P - Q) to the
 *                       classes the method references, kept when LCOM improves
 *                       in both (MM_RULE_PAPER_LCOM); methods with the highest
 *                       fan-out first
 *   MM_SUGGEST_CBO      moves out of classes with a high CBO to the classes the
 *                       method uses, kept when the origin's CBO drops, the
 *                       destination's does not rise and no caller class gets
 *                       worse (MM_RULE_PAPER_CBO); highest fan-in + fan-out first
 *   MM_SUGGEST_SIMILAR  the MM_CAND_SIMILAR moves kept by MM_RULE_PAPER_LCOM, in
 *                       candidate order
 * threshold: MM_THRESH_AVERAGE (origin classes above the average of the metric
 * over all classes, compared exactly: value * c > sum) or MM_THRESH_NONE; it is
 * ignored for MM_SUGGEST_SIMILAR. Equal keys keep candidate order ((method,
 * class) ascending). out == NULL queries *n.
 * Errors: MM_EINVAL (bad kind or threshold; MM_THRESH_AVERAGE on a batch, whose
 * average would mix systems), MM_ERANGE (capacity < *n; nothing written), and
 * those of mm_score_moves / mm_similarity. */
#define MM_SUGGEST_LCOM 0
#define MM_SUGGEST_CBO 1
#define MM_SUGGEST_SIMILAR 2
#define MM_THRESH_NONE 0
#define MM_THRESH_AVERAGE 1
mm_status mm_suggest(mm_system *sys, int32_t kind, int32_t threshold, mm_move_score *out, int64_t capacity,
                     int64_t *n);
/* The ranked suggestions reduced, in rank order, to a conflict-free set: a move
 * is taken when none of its affected classes (its class, its destination and
 * every class owning a caller of the method) belongs to a move taken before.
 * All moves of the set can be applied together, each changing the metrics
 * exactly as its record predicts. Arguments and errors as mm_suggest, plus
 * MM_EOVERFLOW for more than 2^19 classes. */
mm_status mm_suggest_independent(mm_system *sys, int32_t kind, int32_t threshold, mm_move_score *out,
                                 int64_t capacity, int64_t *n);
/* Greedy plan: up to max_moves times, apply the best suggestion of `kind` and
 * re-evaluate (as Sec. IV-C re-runs the metrics after a change). out receives
 * each step's record as scored on the system of that step (capacity >=
 * max_moves) and *n the number of steps. keep_applied = 0 restores the system
 * (the moves are undone in reverse order); 1 leaves them applied. On an error
 * the system is restored. Errors: MM_EINVAL (NULL out or n, negative max_moves,
 * keep_applied not 0/1), and those of mm_suggest / mm_apply_move. */
mm_status mm_plan(mm_system *sys, int32_t kind, int32_t threshold, int32_t max_moves, int32_t keep_applied,
                  mm_move_score *out, int64_t *n);

/* ---- apply_move / apply_edit ----------------------------------------------
 * mm_apply_move moves one method to class dst_class (only the owner changes; Sec.
 * III-A / IV-C). Errors: MM_EINVAL (id out of range, dst_class == current owner).
 * mm_apply_edit replaces the rows, and optionally the owners, of k methods, as
 * when the system evolves (Sec. I: data gathered continuously while the system
 * changes). Errors as mm_load_system, plus MM_EINVAL for repeated methods. */
mm_status mm_apply_move(mm_system *sys, int32_t method, int32_t dst_class);
mm_status mm_apply_edit(mm_system *sys, const mm_edit_desc *edit);
/* After mm_apply_move the next metric request recomputes only what the moves
 * since the last one touched: the grouped counts of the origin and destination
 * classes and of the classes holding callers of a moved method, the caller
 * groups of the moved methods, of the methods they call and of the methods whose
 * loss flags those changes reach, the moved methods' own counts, the co-access
 * of origin and destination, and those classes' aggregates. The results equal a
 * full recompute. enabled = 0 makes every move rebuild the layout and
 * recompute everything instead (the default is 1). Errors: MM_EINVAL. */
mm_status mm_system_set_incremental(mm_system *sys, int32_t enabled);

/* ---- WMC, NOC, DIT ----------------------------------------------------------
 * Sec. II-B names the whole Chidamber-Kemerer suite (WMC, NOC, DIT, CBO, RFC,
 * LCOM) and then works with CBO and LCOM. The other three need what the call and
 * access graph does not hold: the class hierarchy and a complexity weight per
 * method. With the suite's definitions:
 *   wmc  weighted methods per class: the sum of the weights of the class's
 *        methods (the class's method count when every weight is 1);
 *   noc  number of children: classes whose parent is this class;
 *   dit  depth of inheritance: the class's proper ancestors, i.e. the steps up
 *        the parent chain to a class with no parent inside the system (0 for
 *        such a class).
 * mm_set_hierarchy copies
 *   parent  [n_classes] host array: the class each class extends, or -1 when it
 *           extends no class of the system (single inheritance, no cycle);
 *   weight  [n_methods] host array of weights >= 0 (e.g. cyclomatic
 *           complexity), or NULL: every method weighs 1.
 * The caller keeps its arrays. Without a call every class has no parent and
 * every weight is 1. A method keeps its weight when it moves (mm_apply_move,
 * mm_apply_edit): WMC follows the membership, NOC and DIT do not change.
 * Errors: MM_EINVAL (NULL parent with classes, parent id outside [-1,
 * n_classes), a negative weight, a cycle -- then no hierarchy is set -- or, on a
 * batch, a parent in another part), MM_ENOMEM, MM_EHIP. */
typedef struct mm_class_ck {
    int64_t wmc;
    int32_t noc, dit;
} mm_class_ck; /* 16 bytes */
mm_status mm_set_hierarchy(mm_system *sys, const int32_t *parent, const int32_t *weight);
/* WMC, NOC and DIT of every class: out is a host array of n_classes entries
 * (the call waits for the device); mm_compute_ck_device writes a caller-owned
 * device array and returns once the work is enqueued on the context stream.
 * Errors: MM_EINVAL (NULL out with classes), MM_ENOMEM, MM_EHIP. */
mm_status mm_compute_ck(mm_system *sys, mm_class_ck *out);
mm_status mm_compute_ck_device(mm_system *sys, mm_class_ck *d_out);

/* ---- serving ---------------------------------------------------------------
 * A server keeps systems resident on one device and runs requests from several
 * host threads. n_slots worker threads, each with its own HIP stream, take the
 * oldest queued request whose system is idle: requests on different systems run
 * concurrently (their kernels overlap on the GPU), requests on one system keep
 * their submission order, and a request that arrives while others run starts as
 * soon as a slot frees. Loads are admitted by device memory: least recently used
 * idle systems are evicted to make room; a load that cannot fit waits while
 * other requests run, else fails with MM_ENOMEM. An evicted system keeps its
 * current state (after its edits) in host memory: the next request that names
 * it loads it again first, as part of that request (its latency, counted from
 * submission, includes the reload). Loads and reloads, which upload a whole
 * system, run on at most half of the slots at once (at least one), so that the
 * other slots stay free for edits and scores. The server owns its context.
 * Requests (their arrays are copied at submission):
 *   MM_REQ_LOAD   load a system under the caller-chosen id system_id
 *   MM_REQ_EDIT   apply an edit to system_id, then score the REFERENCED
 *                 candidates of the edited methods (with metric_mask, rule,
 *                 keep_only); the records are the result
 *   MM_REQ_SCORE  score system_id (cand_mode MM_CAND_REFERENCED or EXPLICIT)
 *   MM_REQ_FREE   free system_id
 * Each result equals the result of running that system's requests in order
 * without the others. Latency = completion - submission, in milliseconds. */
#define MM_REQ_LOAD 1
#define MM_REQ_EDIT 2
#define MM_REQ_SCORE 3
#define MM_REQ_FREE 4

typedef struct mm_server mm_server;

typedef struct {
    int32_t device;
    int32_t n_slots;             /* worker threads / streams, 1..16 */
    int32_t queue_capacity;      /* queued requests beyond this are refused (MM_EBUSY) */
    int32_t pad;
    uint64_t mem_budget_bytes;   /* device memory cap of all resident systems (0 = none) */
} mm_server_opts;

typedef struct {
    int32_t kind, system_id;
    const mm_system_desc *load;  /* LOAD */
    const mm_edit_desc *edit;    /* EDIT */
    int32_t cand_mode;           /* SCORE */
    int32_t pad;
    const int32_t *cand_method, *cand_class;
    int64_t n_cand;
    uint32_t metric_mask;        /* EDIT and SCORE */
    int32_t rule, keep_only;
    int32_t pad2;
} mm_request;

typedef struct {
    int32_t state;               /* 0 queued, 1 running, 2 done */
    int32_t status;              /* MM_OK or the request's error */
    int32_t slot;                /* worker that ran it */
    int32_t pad;
    int64_t n_records;
    const mm_move_score *records;  /* valid until mm_server_release of this ticket */
    double submit_ms, start_ms, end_ms;  /* since the server started or its stats were reset */
    const char *error;           /* message when status != MM_OK */
} mm_result;

typedef struct {
    int64_t submitted, completed, failed, refused, evicted, records;
    double p50_ms, p99_ms, mean_ms, max_ms, elapsed_s;
    int32_t resident, queued;
    uint64_t device_bytes;
    int64_t reloaded;            /* evicted systems loaded again for a request that named them */
    uint64_t peak_bytes;         /* most device bytes held at once (the reset starts from the current use) */
} mm_server_counters;

mm_status mm_server_create(const mm_server_opts *opts, mm_server **out);
/* Finishes queued requests, then frees every resident system and the server. */
mm_status mm_server_destroy(mm_server *srv);
/* Queue a request; returns at once with its ticket. MM_EBUSY: queue full. */
mm_status mm_server_submit(mm_server *srv, const mm_request *req, uint64_t *ticket);
/* Wait up to timeout_ms (< 0: no limit) for a request; MM_EBUSY if unfinished
 * (out->state tells where it is), MM_ENOTFOUND for an unknown ticket. */
mm_status mm_server_wait(mm_server *srv, uint64_t ticket, int32_t timeout_ms, mm_result *out);
/* Forget a finished request and its records. */
mm_status mm_server_release(mm_server *srv, uint64_t ticket);
/* Block until no request is queued or running. */
mm_status mm_server_drain(mm_server *srv);
/* Counters and latency percentiles since start or the last reset. */
mm_status mm_server_stats(mm_server *srv, int32_t reset, mm_server_counters *out);

#ifdef __cplusplus
}
#endif
#endif /* MM_H */

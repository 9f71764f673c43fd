// mm_api.hip -- host engine behind the C ABI of include/mm.h.
//
// The host keeps a mirror of each system's structure (owners, rows, class
// membership) and derives from it the device layout: which (segment, partition)
// work items exist and where every grouped-count run lives. All per-edge and
// per-pair work runs in the gfx950 kernels; the host does O(n + c) bookkeeping,
// validation and the uploads of Sec. IV-C (data copied once, then resident).
#include <algorithm>
#include <exception>
#include <atomic>
#include <future>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/mm.h"
#include "mm_internal.h"

using namespace mm;

namespace {

thread_local std::string g_last_error;

struct MmError {
    mm_status code;
    std::string msg;
};

[[noreturn]] void fail(mm_status code, const std::string &msg) { throw MmError{code, msg}; }

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) fail(MM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

namespace {

// HIP events around selected kernel launches; totals per kernel name.
struct Timer final : KTimer {
    std::string pattern;  // "" off, "*" every kernel, else ",name,name,"
    struct Pend {
        const char *name;
        hipEvent_t a, b;
    };
    struct Stat {
        const char *name = nullptr;
        int64_t n = 0;
        double ms = 0;
    };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> pool;
    std::map<std::string, Stat> stats;
    const char *cur = nullptr;
    hipEvent_t ca = nullptr;

    bool enabled() const { return !pattern.empty(); }
    bool match(const char *name) const {
        return pattern == "*" || pattern.find("," + std::string(name) + ",") != std::string::npos;
    }
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
        }
        return e;
    }

    bool begin(const char *name, hipStream_t st) override {
        if (!enabled() || !match(name)) return false;
        ca = get();
        if (!ca) return false;
        cur = name;
        (void)hipEventRecord(ca, st);
        return true;
    }
    void end(hipStream_t st) override {
        hipEvent_t b = get();
        if (!b) {
            pool.push_back(ca);
            return;
        }
        (void)hipEventRecord(b, st);
        pend.push_back({cur, ca, b});
        if (pend.size() >= 4096) resolve();
    }
    void add(const Pend &p) {
        float ms = 0;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            Stat &t = stats[p.name];
            t.name = p.name;
            t.n++;
            t.ms += ms;
        } else {
            (void)hipGetLastError();
        }
    }
    void resolve() {
        for (auto &p : pend) {
            add(p);
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pend.clear();
    }
    ~Timer() override {
        resolve();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace

struct mm_context {
    Timer timer;
    std::mutex mem_mu;  // guards `used` (systems of one context may run on several threads)
    mm_tuning tuning{CALLER_LIGHT, HEAVY_CHUNK, 0, 0, 0, 0};
    int32_t n_cu = 256;
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    uint64_t used = 0;    // bytes held by live buffers
    uint64_t peak = 0;    // most bytes held at once since creation or the last reset of server statistics
    uint64_t pooled = 0;  // bytes of released blocks kept for reuse (pool and deferred lists)
    std::multimap<size_t, void *> pool;
    int32_t n_systems = 0;
    std::mutex aux_mu;
    std::map<hipStream_t, AuxStreams> aux;  // per calling stream
};

namespace {

// Released blocks of a context are kept for reuse instead of freed: hipFree
// waits for the whole device, which would stall every other stream. Reuse is
// ordered by the context's stream; a server worker, whose stream differs from
// the other workers', sets tl_defer so that its releases reach the pool only
// after its stream has finished (flush_deferred).
thread_local std::vector<std::pair<size_t, void *>> *tl_defer = nullptr;

// Blocks kept for reuse: under a budget every released block is kept (pooled
// bytes count against the budget, and an allocation that needs room frees
// pooled blocks first), so a release never waits in hipFree for the device;
// without one, up to 1 GiB.
uint64_t pool_limit(const mm_context *c) { return c->budget ? c->budget : (uint64_t)1 << 30; }

void flush_deferred(mm_context *c, std::vector<std::pair<size_t, void *>> &v) {
    std::lock_guard<std::mutex> lk(c->mem_mu);
    for (auto &e : v) c->pool.emplace(e.first, e.second);
    v.clear();
}

// free pooled blocks, largest first, until `need` more bytes fit the budget
// (caller holds mem_mu)
void trim_pool(mm_context *c, uint64_t need) {
    while (!c->pool.empty() && c->used + c->pooled + need > c->budget) {
        auto it = std::prev(c->pool.end());
        (void)hipFree(it->second);
        c->pooled -= it->first;
        c->pool.erase(it);
    }
}

// auxiliary streams for the kernels that run beside `st` (created on first use)
const AuxStreams *aux_for(mm_context *c, hipStream_t st) {
    std::lock_guard<std::mutex> lk(c->aux_mu);
    auto it = c->aux.find(st);
    if (it != c->aux.end()) return &it->second;
    AuxStreams a{};
    for (auto &x : a.s)
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;  // run the phase in order on st
        }
    for (auto &e : a.ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    return &c->aux.emplace(st, a).first->second;
}

// device buffer charged against the context budget
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    mm_context *ctx = nullptr;
    int64_t *sys_bytes = nullptr;

    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }

    void release() {
        if (p) {
            std::lock_guard<std::mutex> lk(ctx->mem_mu);
            ctx->used -= bytes;
            if (sys_bytes) *sys_bytes -= (int64_t)bytes;
            if (ctx->pooled + bytes > pool_limit(ctx)) {
                (void)hipFree(p);  // waits for pending work on the block
            } else {
                ctx->pooled += bytes;
                if (tl_defer) tl_defer->emplace_back(bytes, p);
                else ctx->pool.emplace(bytes, p);
            }
        }
        p = nullptr;
        bytes = 0;
    }
    // at least `want` bytes (rounded to 256; a pooled block up to 25% larger may
    // serve), old content dropped
    void alloc(mm_context *c, int64_t *counter, size_t want) {
        if (want < 256) want = 256;
        want = (want + 255) & ~(size_t)255;
        if (p && bytes == want) return;
        release();
        ctx = c;
        sys_bytes = counter;
        std::lock_guard<std::mutex> lk(c->mem_mu);
        auto it = c->pool.lower_bound(want);
        if (it != c->pool.end() && it->first <= want + want / 4) {
            if (c->budget && c->used + it->first > c->budget)
                fail(MM_ENOMEM, "device memory budget exceeded (" + std::to_string(c->used + it->first) + " > " +
                                    std::to_string(c->budget) + " bytes)");
            p = it->second;
            bytes = it->first;
            c->pooled -= bytes;
            c->pool.erase(it);
            c->used += bytes;
            c->peak = std::max(c->peak, c->used);
            if (counter) *counter += (int64_t)bytes;
            return;
        }
        if (c->budget) {
            trim_pool(c, want);
            if (c->used + c->pooled + want > c->budget)
                fail(MM_ENOMEM, "device memory budget exceeded (" + std::to_string(c->used + want) + " > " +
                                    std::to_string(c->budget) + " bytes)");
        }
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            // give the pool back to the device and try once more
            for (auto &e : c->pool) (void)hipFree(e.second);
            for (auto &e : c->pool) c->pooled -= e.first;
            c->pool.clear();
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                fail(MM_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
            }
        }
        bytes = want;
        c->used += want;
        c->peak = std::max(c->peak, c->used);
        if (counter) *counter += (int64_t)want;
    }
    // at least `want` bytes for data that is rewritten whole: exact on first
    // use; later kept while within 25% above `want`, else reallocated with 1/8
    // headroom so that small growth (edits) does not reallocate every time
    void fit(mm_context *c, int64_t *counter, size_t want) {
        if (want < 256) want = 256;
        want = (want + 255) & ~(size_t)255;
        if (p && bytes >= want && bytes - want <= want / 4 + 4096) return;
        alloc(c, counter, p ? want + want / 8 : want);
    }
    // at least `want` bytes, kept when already large enough
    void reserve(mm_context *c, int64_t *counter, size_t want) {
        if (p && bytes >= want) return;
        size_t grow = want + want / 4;
        alloc(c, counter, grow);
    }
    template <typename T>
    T *as() const { return (T *)p; }
    void swap(DBuf &o) {  // exchange blocks (and their accounting) with another buffer
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(ctx, o.ctx);
        std::swap(sys_bytes, o.sys_bytes);
    }
};

template <typename T>
void upload(mm_context *ctx, int64_t *counter, DBuf &b, const std::vector<T> &v, hipStream_t st) {
    b.fit(ctx, counter, v.size() * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Layout of one grouped-count map over its segments (see mm_dev.h).
// Fill items and partitions of the hash-table segments of one map (the host
// side of k_big_stage / k_big_build).
struct BigHost {
    std::vector<BigItem> items;
    std::vector<BigPart> parts;
    int64_t stage = 0, bt = 0;  // staging pairs and partition-table words the items need
    int32_t np_max = 1;
    int64_t n_segs = 0;
    void clear() {
        items.clear();
        parts.clear();
        stage = bt = 0;
        np_max = 1;
        n_segs = 0;
    }
    void push(int32_t seg, int32_t a, int32_t b, int32_t y, int64_t entries) {
        items.push_back(BigItem{seg, a, b, y, 0, 0, stage, 0});
        stage += entries;
    }
    // the items of segment seg pushed from index i0 on: their numbering, the
    // segment's partition table and one block per partition
    void close(int32_t seg, int32_t cap, size_t i0) {
        const int32_t nI = (int32_t)(items.size() - i0);
        const int32_t np = cap > PART_SLOTS ? cap / PART_SLOTS : 1;
        if (np > PART_MAX) fail(MM_EOVERFLOW, "a grouped-count table of more than 2^24 slots");
        for (size_t i = i0; i < items.size(); ++i) {
            items[i].j = (int32_t)(i - i0);
            items[i].nI = nI;
            items[i].bt = bt;
        }
        for (int32_t p = 0; p < np; ++p) parts.push_back(BigPart{seg, p, (int32_t)i0, nI, bt});
        bt += (int64_t)(np + 1) * nI;
        np_max = std::max(np_max, np);
        ++n_segs;
    }
};

struct MapLayout {
    std::vector<MapHdr> hdr;
    std::vector<int32_t> wave;      // table segments grouped in LDS, those of more than MAP_HSMALL slots first
    int n_wave_large = 0;
    std::vector<int32_t> mid;       // table segments of MAP_CAP..MID_CAP references, grouped in LDS by a block
    std::vector<int32_t> big_segs;  // hash-table segments built in two passes
    BigHost big;                    //   their fill items and partitions
    int64_t slots = 0;
};

// R[s] = references of segment s (an upper bound of its distinct keys), keyspace
// = number of possible keys. Table size: a power of two >= 2 * distinct bound.
// Segments with at most run_max references become sorted runs grouped by one
// lane; up to MAP_CAP, tables grouped in LDS by a wave (or a block, for caller
// maps); up to mid_max (W and CNT: MID_CAP), tables grouped in LDS by a block;
// larger ones, tables built by fill items and partitions (k_big_stage,
// k_big_build). Every kind is written whole by its builder.
// smallest power of two >= max(need, lo), lo a power of two
inline int64_t pow2_at_least(int64_t need, int64_t lo) {
    if (need <= lo) return lo;
    return (int64_t)1 << (64 - __builtin_clzll((uint64_t)(need - 1)));
}

void make_map(const std::vector<int64_t> &R, int64_t keyspace, int64_t run_max, int64_t mid_max, MapLayout &L) {
    const size_t ns = R.size();
    L.hdr.resize(ns);
    L.wave.clear();
    L.mid.clear();
    L.big.clear();
    L.big_segs.clear();
    int64_t cur = 0;
    // runs (and empty headers) in one pass without data-dependent branches: a
    // segment with 1..run_max references is a run, the others are empty here
    // and become tables below
    for (size_t q = 0; q < ns; ++q) {
        const int64_t r = R[q];
        const bool run = (uint64_t)(r - 1) < (uint64_t)run_max;
        L.hdr[q] = MapHdr{run ? (int32_t)cur : 0, 0, run ? MAP_RUN : MAP_EMPTY, run ? (int32_t)r : 0};
        cur += run ? r : 0;
    }
    std::vector<int32_t> small;
    for (size_t q = 0; q < ns; ++q) {
        if (R[q] <= run_max || R[q] > MAP_CAP) continue;
        const int64_t cap = pow2_at_least(2 * std::min<int64_t>(R[q], keyspace), 4);
        L.hdr[q] = MapHdr{(int32_t)cur, 0, MAP_TABLE, (int32_t)cap};
        cur += cap;
        (cap > MAP_HSMALL ? L.wave : small).push_back((int32_t)q);
    }
    L.n_wave_large = (int)L.wave.size();
    L.wave.insert(L.wave.end(), small.begin(), small.end());
    for (size_t q = 0; q < ns; ++q) {
        if (R[q] <= MAP_CAP || R[q] > mid_max) continue;
        const int64_t cap = pow2_at_least(2 * std::min<int64_t>(R[q], keyspace), 1024);
        L.hdr[q] = MapHdr{(int32_t)cur, 0, MAP_TABLE, (int32_t)cap};
        cur += cap;
        L.mid.push_back((int32_t)q);
    }
    for (size_t q = 0; q < ns; ++q) {
        if (R[q] <= std::max<int64_t>(mid_max, MAP_CAP)) continue;
        const int64_t cap = pow2_at_least(2 * std::min<int64_t>(R[q], keyspace), 1024);
        L.hdr[q] = MapHdr{(int32_t)cur, 0, MAP_TABLE, (int32_t)cap};
        cur += cap;
        L.big_segs.push_back((int32_t)q);
        if (cur > INT32_MAX) fail(MM_EOVERFLOW, "grouped-count layout exceeds 2^31 slots");
    }
    if (cur > INT32_MAX) fail(MM_EOVERFLOW, "grouped-count layout exceeds 2^31 slots");
    L.slots = cur;
}

struct DevMap {
    DBuf hdr, foreign, keys, vals, wave, mid, flag_items;
    DBuf big_items, big_parts, big_stage, big_bt;  // hash-table segments: fill items, partitions, their work areas
    int n_wave = 0, n_wave_large = 0, n_mid = 0, n_flag_items = 0;
    int n_big_items = 0, n_big_parts = 0, np_max = 1;
    int64_t slots = 0;
    int64_t pool_cap = 0;  // slots the keys/vals buffers hold (tables that outgrow theirs move to the end)
    std::vector<MapHdr> host_hdr;  // kinds and capacities (lengths live on the device)
};

// a small pinned host block: device-to-host reads into it need no staging copy
struct PinnedBlock {
    void *p = nullptr;
    void *dev = nullptr;  // the block's address in device code (NULL: not mapped, read it back by a copy)
    PinnedBlock() = default;
    PinnedBlock(const PinnedBlock &) = delete;
    PinnedBlock &operator=(const PinnedBlock &) = delete;
    ~PinnedBlock() {
        if (p) (void)hipHostFree(p);
    }
    void *get(size_t bytes) {  // NULL when pinned memory is unavailable (the caller uses pageable memory)
        if (!p) {
            if (hipHostMalloc(&p, bytes, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
            } else if (hipHostGetDevicePointer(&dev, p, 0) != hipSuccess) {
                (void)hipGetLastError();
                dev = nullptr;
            }
        }
        return p;
    }
};


}  // namespace

// State of the incremental recompute after moves (mm_incr_impl.h).
struct Incr {
    std::vector<uint8_t> fc, fm;     // dirty bits per class / method since the last metric recompute
    std::vector<int32_t> lc, lm;     // the classes / methods with bits set
    std::vector<int64_t> Rw, Rc;     // references per class (W, CNT), current
    std::vector<int32_t> mem_lim;    // end of each class's region of the membership pool
    int64_t mem_used = 0, mem_cap = 0;
    std::vector<int32_t> h_flags;    // caller classes read back from the device
    DBuf d_flags;
    DBuf d_mark, d_inl, d_key;       // device marks of caller maps to rebuild, their filed lists, the changed W keys
    void *mark_block = nullptr;      // the d_mark block last cleared (a pass clears the marks it files)
    std::vector<uint8_t> key_host;
    std::vector<int32_t> inl_host;
    bool active = false;             // moves wait for their recompute
    bool base = false;               // every metric was computed on this layout (moves may then patch them)
    bool stale = false;              // the layout's full work lists describe an older membership
    std::vector<int4> ops, ops_stage;
    std::vector<int32_t> plan_stage, edit_stage;
    DBuf d_ops, d_plan, d_edit;
    BigHost big[3];                  // fill items and partitions of the hash-table segments to rebuild (W, CNT, callers)
    DBuf d_big_items[3], d_big_parts[3];
    hipEvent_t ops_ev = nullptr, plan_ev = nullptr, edit_ev = nullptr;  // last copy out of the staging buffers
    bool ops_ev_set = false, plan_ev_set = false, edit_ev_set = false;
    struct {
        int64_t classes = 0, w = 0, cnt = 0, in = 0, basic = 0;
    } last_dirty;                    // sizes of the last incremental recompute
    Incr() = default;
    Incr(const Incr &) = delete;
    Incr &operator=(const Incr &) = delete;
    ~Incr() {
        if (ops_ev) (void)hipEventDestroy(ops_ev);
        if (plan_ev) (void)hipEventDestroy(plan_ev);
        if (edit_ev) (void)hipEventDestroy(edit_ev);
    }
};

struct mm_system {
    mm_context *ctx = nullptr;
    hipStream_t stream = nullptr;  // the context's stream, or a server slot's while it runs a request
    int32_t c = 0, n = 0, na = 0;
    // a batch is the disjoint union of its parts; part i owns classes
    // [part_cls[i], part_cls[i+1]) and likewise methods and attributes
    std::vector<int32_t> part_cls, part_meth, part_attr;
    int64_t bytes = 0;
    int64_t version = 0;

    // host mirror
    std::vector<int32_t> owner, acls, alocal, acnt;
    std::vector<int32_t> acc_off, acc_idx, call_off, call_idx, rc_off;  // rc_off: caller offsets (lists on the device)
    // the rows an edit replaced, kept as the next edit's output (no fresh, zeroed
    // allocation per edit)
    std::vector<int32_t> spare_acc_off, spare_acc_idx, spare_call_off, spare_call_idx;
    std::vector<int32_t> mem_off, mem_end, mem_idx;  // class C's methods: mem_idx[mem_off[C] .. mem_end[C])

    // device copy of the structure
    DBuf d_owner, d_acls, d_alocal, d_acnt, d_acc_off, d_acc_idx, d_call_off, d_call_idx, d_rc_off, d_rc_idx;
    DBuf d_mem_off, d_mem_end, d_mem_idx;
    DBuf d_call_cls, d_acc_cls, d_rc_cls;  // class of every call, access and caller entry
    DBuf d_acc_rank;                       // rank of every access's attribute in its class
    bool entry_classes_valid = false;      // they match the device rows (and owners, but for entry_moved)
    std::vector<int32_t> entry_moved;      // methods moved since, rows unchanged: patched, not gathered again
    DevMap w, cnt, in;
    DBuf d_co_items;     // co-access groups, then single row tiles of wide classes
    int n_co_items = 0, n_co_groups = 0;
    DBuf d_co_small;     // classes whose co-access fits one wave
    int n_co_small = 0;
    DBuf d_fin_list;     // every class for the aggregates: at most 64 members first, then the others
    int n_fin_small = 0;
    DBuf d_wc_list;      // W and CNT tables grouped by waves, as work items (MapWcWork)
    int n_wc_large = 0, n_wc_small = 0;
    DBuf d_in_runs;      // methods with 1..IN_SMALL callers grouped by row length
    int in_run_off[5] = {0, 0, 0, 0, 0};
    DBuf d_prep_runs;    // every method grouped by its row length (calls + accesses)
    int prep_run_off[6] = {0, 0, 0, 0, 0, 0};
    std::vector<int32_t> prep_host, prep_pos;  // host copy of that list, and each method's place in it
    bool structure_valid = false;  // device structure matches the host mirror
    bool layout_valid = false;
    int64_t structure_version = 0;  // counts uploads of the structure
    Incr incr;
    bool incr_enabled = true;  // moves recompute only what they touch (else a full layout rebuild)
    int32_t layout_fill = 0;  // fill_chunk of the schedule the layout used
    int32_t big_chunk = BIG_CHUNK;  // most entries of a fill item of the hash-table segments

    // metrics
    DBuf d_meth, d_cls, d_err, d_own_mask;
    bool metrics_valid = false;
    // the last work on maps_stream is a full metric launch whose W and CNT maps
    // have their own event (ev[5] of that stream's aux set); the next score
    // consumes it
    bool maps_event = false;
    hipStream_t maps_stream = nullptr;

    // score scratch
    DBuf s_prep, s_outk, s_outc, s_outa, s_refcnt, s_candoff, s_cm, s_ct, s_ce, s_rec;
    DBuf s_gcnt, s_goff, s_gslot, s_glist, s_hval;
    DBuf s_heavy, s_hcand, s_counts, s_flags, s_kpos, s_tmp, s_kept, s_kept_idx;
    DBuf s_aff_flag, s_aff_val, s_aff_pos, s_aff_cls, s_aff_d;  // per-caller detail of one move
    DBuf s_rank_rec, s_rank_key, s_rank_key2, s_rank_idx, s_rank_idx2, s_rank_tmp;  // ranked suggestions

    // similarity of method pairs (k_sim.hip) and its candidates
    DBuf sim_at_off, sim_at_idx, sim_at_cur, sim_deg, sim_dense, sim_cnt2, sim_ctr, sim_hist, sim_imin;
    DBuf sim_row_pairs, sim_row_cands, sim_cand_bits, sim_cand_off, sim_pair_off, sim_pairs;
    struct {
        int64_t at_version = -1, stats_version = -1, count_version = -1;
        int32_t count_threshold = -1, umax = 0, grid = 0, cw = 0;
        std::vector<uint64_t> hist;  // sum of shared counts by union size
        uint64_t nnz = 0;            // pairs with a shared property
        std::vector<int32_t> imin, row_cands;
        int64_t n_kept = 0, n_cands = 0;
        double average = 0;
    } sim;
    int32_t sim_threshold = MM_SIM_ABOVE_AVG;  // threshold of MM_CAND_SIMILAR

    // per-version host bookkeeping reused across scoring calls
    struct {
        int64_t version = -1;
        int32_t mode = -1, caller_light = -1, heavy_chunk = -1;
        int64_t heavy_items = 0, heavy_cands = 0;
    } hb_cache;
    int64_t ref_version = -1, ref_count = 0;  // REFERENCED candidate count of that version

    // class hierarchy and method weights (WMC, NOC, DIT); NOC and DIT are
    // computed when the hierarchy is set
    DBuf ck_weight, ck_noc, ck_dit, ck_out;
    bool ck_hier = false, ck_weighted = false;

    ScanArea scan;  // host side of the prefix-sum work area in s_tmp
    PinnedBlock status_host;       // where the error bits and the kept count are read back

    struct {
        bool valid = false;
        int64_t version = -1;
        int32_t mode = -1, rule = -1, keep_only = -1;
        uint32_t mask = 0;
        std::vector<int32_t> cm, ct;
        int64_t n_cand = 0, n_out = 0;
        bool rec_external = false;  // records were written straight to a caller buffer
        int32_t sim_threshold = -1;
        int32_t origin = 0;
    } cache;

    DevSys view() const {
        DevSys d;
        d.c = c;
        d.n = n;
        d.na = na;
        d.pad = 0;
        d.owner = d_owner.as<int32_t>();
        d.acls = d_acls.as<int32_t>();
        d.alocal = d_alocal.as<int32_t>();
        d.acnt = d_acnt.as<int32_t>();
        d.acc_off = d_acc_off.as<int32_t>();
        d.acc_idx = d_acc_idx.as<int32_t>();
        d.call_off = d_call_off.as<int32_t>();
        d.call_idx = d_call_idx.as<int32_t>();
        d.rc_off = d_rc_off.as<int32_t>();
        d.rc_idx = d_rc_idx.as<int32_t>();
        d.mem_off = d_mem_off.as<int32_t>();
        d.mem_end = d_mem_end.as<int32_t>();
        d.mem_idx = d_mem_idx.as<int32_t>();
        d.call_cls = d_call_cls.as<int32_t>();
        d.acc_cls = d_acc_cls.as<int32_t>();
        d.rc_cls = d_rc_cls.as<int32_t>();
        d.acc_rank = d_acc_rank.as<int32_t>();
        return d;
    }
};

namespace {

template <typename F>
mm_status guarded(F &&f) {
    try {
        f();
        return MM_OK;
    } catch (const MmError &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return MM_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return MM_EINTERNAL;
    }
}

void set_device(mm_context *ctx) { HIPCHK(hipSetDevice(ctx->device)); }

// Validate one CSR block (offsets [rows + 1], ids in [0, id_limit)).
void check_csr(const char *what, const int64_t *off, const int32_t *idx, int64_t rows, int64_t id_limit) {
    if (!off) fail(MM_EINVAL, std::string(what) + " offsets are NULL");
    if (off[0] != 0) fail(MM_EINVAL, std::string(what) + " offsets must start at 0");
    for (int64_t i = 0; i < rows; ++i)
        if (off[i + 1] < off[i]) fail(MM_EINVAL, std::string(what) + " offsets decrease at row " + std::to_string(i));
    int64_t nnz = off[rows];
    if (nnz > INT32_MAX) fail(MM_EOVERFLOW, std::string(what) + " has more than 2^31-1 entries");
    if (nnz > 0 && !idx) fail(MM_EINVAL, std::string(what) + " ids are NULL");
    for (int64_t e = 0; e < nnz; ++e)
        if (idx[e] < 0 || idx[e] >= id_limit)
            fail(MM_EINVAL, std::string(what) + " id out of range at entry " + std::to_string(e));
}

// rows read as sets: sort and drop repeats
void canonical_rows(const int64_t *off, const int32_t *idx, int64_t rows, std::vector<int32_t> &o,
                    std::vector<int32_t> &v) {
    o.assign(rows + 1, 0);
    v.clear();
    v.reserve(off[rows]);
    std::vector<int32_t> tmp;
    for (int64_t i = 0; i < rows; ++i) {
        tmp.assign(idx + off[i], idx + off[i + 1]);
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        v.insert(v.end(), tmp.begin(), tmp.end());
        o[i + 1] = (int32_t)v.size();
    }
}

ScanArea &scan_area(mm_system *s, int64_t n);
void rebuild_callers(mm_system *s);

void upload_structure(mm_system *s) {
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    ++s->structure_version;
    upload(ctx, cb, s->d_owner, s->owner, s->stream);
    upload(ctx, cb, s->d_acls, s->acls, s->stream);
    upload(ctx, cb, s->d_alocal, s->alocal, s->stream);
    upload(ctx, cb, s->d_acnt, s->acnt, s->stream);
    upload(ctx, cb, s->d_acc_off, s->acc_off, s->stream);
    upload(ctx, cb, s->d_acc_idx, s->acc_idx, s->stream);
    upload(ctx, cb, s->d_call_off, s->call_off, s->stream);
    upload(ctx, cb, s->d_call_idx, s->call_idx, s->stream);
    rebuild_callers(s);
    // the caller offsets come back to the host
    s->rc_off.resize((size_t)s->n + 1);
    HIPCHK(hipMemcpyAsync(s->rc_off.data(), s->d_rc_off.p, ((size_t)s->n + 1) * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipGetLastError());
}

// Callers of every method (the reverse call rows), built on the device from the
// device rows: the edges tagged with their caller, stably sorted by callee, then
// the row offsets from the sorted callees. Enqueued on the system's stream.
void rebuild_callers(mm_system *s) {
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    s->entry_classes_valid = false;
    const int32_t n = s->n;
    const int64_t nnz = (int64_t)s->call_idx.size();
    s->d_rc_off.fit(ctx, cb, ((size_t)n + 1) * 4);
    s->d_rc_idx.fit(ctx, cb, (size_t)std::max<int64_t>(nnz, 1) * 4);
    DBuf rows, callee_sorted, tmp;
    const DevSys d = s->view();
    if (nnz > 0) {
        rows.alloc(ctx, nullptr, (size_t)nnz * 4);
        callee_sorted.alloc(ctx, nullptr, (size_t)nnz * 4);
        launch_edge_rows(d, rows.as<int32_t>(), s->stream);
        size_t tmp_bytes = 0;
        HIPCHK(callers_sort(nullptr, tmp_bytes, nullptr, nullptr, nullptr, nullptr, nnz, n, s->stream));
        tmp.alloc(ctx, nullptr, std::max<size_t>(tmp_bytes, 1));
        HIPCHK(callers_sort(tmp.p, tmp_bytes, s->d_call_idx.as<int32_t>(), callee_sorted.as<int32_t>(),
                            rows.as<int32_t>(), s->d_rc_idx.as<int32_t>(), nnz, n, s->stream));
    }
    launch_rc_bounds(callee_sorted.as<int32_t>(), nnz, n, s->d_rc_off.as<int32_t>(), s->stream);
    HIPCHK(hipGetLastError());
}

// The class of every call, access and caller entry (DevSys::call_cls and the
// others), gathered once on the system's stream whenever the rows or the owners
// have changed since the last gathering.
void ensure_entry_classes(mm_system *s) {
    if (s->entry_classes_valid && s->entry_moved.empty()) return;
    if (s->entry_classes_valid) {
        // a few moves: patch the entries naming the moved methods (each once,
        // with its current owner), unless that is more work than gathering all
        std::vector<int32_t> &mv = s->entry_moved;
        std::sort(mv.begin(), mv.end());
        mv.erase(std::unique(mv.begin(), mv.end()), mv.end());
        int64_t work = 0;
        for (int32_t m : mv)
            work += (s->rc_off[m + 1] - s->rc_off[m]) + (s->call_off[m + 1] - s->call_off[m]);
        if ((int64_t)mv.size() <= ENTRY_MOVES_MAX && work <= std::max<int64_t>((int64_t)s->call_idx.size() / 16, 4096)) {
            EntryMoves em;
            em.n = (int32_t)mv.size();
            std::copy(mv.begin(), mv.end(), em.m);
            launch_entry_moves(s->view(), em, s->d_call_cls.as<int32_t>(), s->d_rc_cls.as<int32_t>(), s->stream);
            HIPCHK(hipGetLastError());
            mv.clear();
            return;
        }
    }
    s->entry_moved.clear();
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    const int64_t ncall = (int64_t)s->call_idx.size(), nacc = (int64_t)s->acc_idx.size();
    s->d_call_cls.fit(ctx, cb, (size_t)std::max<int64_t>(ncall, 1) * 4);
    s->d_rc_cls.fit(ctx, cb, (size_t)std::max<int64_t>(ncall, 1) * 4);
    s->d_acc_cls.fit(ctx, cb, (size_t)std::max<int64_t>(nacc, 1) * 4);
    s->d_acc_rank.fit(ctx, cb, (size_t)std::max<int64_t>(nacc, 1) * 4);
    launch_entry_classes(s->view(), ncall, nacc, s->d_call_cls.as<int32_t>(), s->d_acc_cls.as<int32_t>(),
                         s->d_rc_cls.as<int32_t>(), s->d_acc_rank.as<int32_t>(), s->stream);
    HIPCHK(hipGetLastError());
    s->entry_classes_valid = true;
}

// the fill items and partitions of a map's hash-table segments, with room for
// their staging pairs and partition tables
void upload_big(mm_system *s, DevMap &dm, const BigHost &bh) {
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    upload(ctx, cb, dm.big_items, bh.items, s->stream);
    upload(ctx, cb, dm.big_parts, bh.parts, s->stream);
    dm.big_stage.reserve(ctx, cb, (size_t)std::max<int64_t>(bh.stage, 1) * sizeof(int2));
    dm.big_bt.reserve(ctx, cb, (size_t)std::max<int64_t>(bh.bt, 1) * sizeof(int32_t));
    dm.n_big_items = (int)bh.items.size();
    dm.n_big_parts = (int)bh.parts.size();
    dm.np_max = bh.np_max;
}

void upload_map(mm_system *s, DevMap &dm, const MapLayout &L, bool foreign) {
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    upload(ctx, cb, dm.hdr, L.hdr, s->stream);
    if (foreign) {
        dm.foreign.fit(ctx, cb, std::max<size_t>(L.hdr.size(), 1) * sizeof(int32_t));
        fill_i32(dm.foreign.as<int32_t>(), 0, (int64_t)L.hdr.size(), s->stream);
    }
    upload(ctx, cb, dm.wave, L.wave, s->stream);
    upload(ctx, cb, dm.mid, L.mid, s->stream);
    dm.n_mid = (int)L.mid.size();
    upload_big(s, dm, L.big);
    dm.n_wave = (int)L.wave.size();
    dm.n_wave_large = L.n_wave_large;
    // room for tables that outgrow theirs after moves (they move to the end)
    const int64_t pool = L.slots + L.slots / 4 + 1024;
    dm.keys.fit(ctx, cb, (size_t)pool * sizeof(int32_t));
    dm.vals.fit(ctx, cb, (size_t)pool * sizeof(int32_t));
    dm.pool_cap = (int64_t)std::min(dm.keys.bytes, dm.vals.bytes) / (int64_t)sizeof(int32_t);
    dm.slots = L.slots;
    dm.host_hdr = L.hdr;
}

// fill items of class segment C: batches of members holding at most `chunk`
// row entries; a member with a longer row gets items of `chunk` entries of it
void big_class_items(const mm_system *s, BigHost &bh, int32_t C, int32_t cap, bool calls_only, int32_t chunk) {
    const size_t i0 = bh.items.size();
    int32_t j0 = s->mem_off[C];
    int64_t acc = 0;
    for (int32_t j = s->mem_off[C]; j < s->mem_end[C]; ++j) {
        const int32_t y = s->mem_idx[(size_t)j];
        const int64_t L =
            (s->call_off[y + 1] - s->call_off[y]) + (calls_only ? 0 : s->acc_off[y + 1] - s->acc_off[y]);
        if (acc + L > chunk && j0 < j) {  // the batch before y is full
            bh.push(C, j0, j, -1, acc);
            j0 = j;
            acc = 0;
        }
        if (L > chunk) {  // y alone, in pieces
            for (int64_t e = 0; e < L; e += chunk)
                bh.push(C, (int32_t)e, (int32_t)std::min<int64_t>(e + chunk, L), y, std::min<int64_t>(chunk, L - e));
            j0 = j + 1;
        } else {
            acc += L;
        }
    }
    if (j0 < s->mem_end[C] || bh.items.size() == i0) bh.push(C, j0, s->mem_end[C], -1, acc);
    bh.close(C, cap, i0);
}

// fill items of the caller map of method m: pieces of `chunk` callers
void big_caller_items(const mm_system *s, BigHost &bh, int32_t m, int32_t cap, int32_t chunk) {
    const size_t i0 = bh.items.size();
    const int32_t lo = s->rc_off[m], hi = s->rc_off[m + 1];
    for (int32_t a = lo; a < hi; a += std::min(chunk, hi - a)) bh.push(m, a, a + std::min(chunk, hi - a), -1, std::min(chunk, hi - a));
    if (bh.items.size() == i0) bh.push(m, lo, lo, -1, 0);
    bh.close(m, cap, i0);
}

// slots of k_big_stage's LDS table for items of at most `chunk` entries
inline int32_t big_lds_slots(int32_t chunk) { return (int32_t)pow2_at_least(2 * (int64_t)chunk, 64); }


void incr_reset(mm_system *s, const std::vector<int64_t> &Rw, const std::vector<int64_t> &Rc);  // mm_incr_impl.h

// class membership, grouped-count layouts and MFMA tile lists from the mirror
constexpr int32_t LAYOUT_THREADS_MIN = 100000;  // methods from which the layout passes run on host threads

void build_layout(mm_system *s) {
    const int32_t c = s->c, n = s->n;
    s->mem_off.assign(c + 1, 0);
    for (int32_t m = 0; m < n; ++m) s->mem_off[s->owner[m] + 1]++;
    for (int32_t k = 0; k < c; ++k) s->mem_off[k + 1] += s->mem_off[k];
    s->mem_idx.assign(n, 0);
    {
        std::vector<int32_t> fill(s->mem_off.begin(), s->mem_off.end() - 1);
        for (int32_t m = 0; m < n; ++m) s->mem_idx[fill[s->owner[m]]++] = m;
    }
    s->mem_end.assign(s->mem_off.begin() + 1, s->mem_off.end());
    s->incr.mem_cap = (int64_t)n + n / 4 + 256;  // room for class rows that outgrow theirs after moves
    s->mem_idx.resize((size_t)s->incr.mem_cap, 0);
    std::vector<int64_t> Rw(c, 0), Rc(c, 0), Ri(n, 0);
    for (int32_t m = 0; m < n; ++m) {
        int64_t nc = s->call_off[m + 1] - s->call_off[m], na = s->acc_off[m + 1] - s->acc_off[m];
        Rw[s->owner[m]] += nc + na;
        Rc[s->owner[m]] += nc;
        Ri[m] = s->rc_off[m + 1] - s->rc_off[m];
    }
    // The passes below read the system and write disjoint outputs, so on a
    // large system they run on their own host threads (milliseconds each);
    // on a small one they run in turn when joined. get() joins them and passes
    // on the first failure.
    const std::launch pol = n >= LAYOUT_THREADS_MIN ? std::launch::async : std::launch::deferred;
    MapLayout Lw, Lc, Li;
    std::vector<int4> flag_items;
    // Fill items of the hash-table segments: about BIG_ITEMS_TARGET of them in
    // all (enough blocks to fill the chip, each lane with one or two entries),
    // between BIG_CHUNK_MIN and BIG_CHUNK references each.
    int64_t big_refs = 0;
    // W and CNT tables of MAP_CAP..MID_CAP references are grouped in LDS by a
    // block on large systems; on small ones (bound by issuing launches) they
    // join the hash-table segments, which saves a launch on the side chain
    const int64_t mid_max = n >= MID_TIER_MIN ? MID_CAP : MAP_CAP;
    for (int32_t q = 0; q < c; ++q) big_refs += (Rw[q] > mid_max ? Rw[q] : 0) + (Rc[q] > mid_max ? Rc[q] : 0);
    for (int32_t m = 0; m < n; ++m) big_refs += Ri[m] > MAP_CAP ? Ri[m] : 0;
    // (the schedule may fix the item size and the item count from which a
    // segment's items are grouped in LDS; both change speed only)
    const mm_tuning &tu = s->ctx->tuning;
    const int32_t chunk = tu.fill_chunk > 0 ? tu.fill_chunk
                          : (int32_t)std::min<int64_t>(BIG_CHUNK, pow2_at_least(big_refs / BIG_ITEMS_TARGET,
                                                                                BIG_CHUNK_MIN));
    s->layout_fill = tu.fill_chunk;
    s->big_chunk = chunk;
    auto f_w = std::async(pol, [&] {
        make_map(Rw, c, 0, mid_max, Lw);
        for (int32_t C : Lw.big_segs) big_class_items(s, Lw.big, C, Lw.hdr[(size_t)C].cap, false, chunk);
    });
    auto f_c = std::async(pol, [&] {
        make_map(Rc, n, 0, mid_max, Lc);
        for (int32_t C : Lc.big_segs) big_class_items(s, Lc.big, C, Lc.hdr[(size_t)C].cap, true, chunk);
    });
    auto f_i = std::async(pol, [&] {
        make_map(Ri, c, IN_SMALL, MAP_CAP, Li);
        for (int32_t m : Li.big_segs) {
            big_caller_items(s, Li.big, m, Li.hdr[(size_t)m].cap, chunk);
            for (int32_t a = 0; a < Li.hdr[m].cap; a += BIG_CHUNK)
                flag_items.push_back(make_int4(m, a, std::min(a + BIG_CHUNK, Li.hdr[m].cap), 0));
        }
    });
    // Two work lists from one classifying pass over the methods (group from a
    // small table, no data-dependent branches), then one placing pass:
    //   runs: the short caller rows by length, up to 4, 8, 16 and IN_SMALL callers
    //   prep_runs: every method by its row length (calls + accesses), up to 8,
    //              16, 32 and 64 entries (lane segments of that width), or longer
    static_assert(IN_SMALL == 32, "caller-row groups of 4, 8, 16, 32");
    std::vector<int32_t> runs((size_t)n), prep_runs((size_t)n);
    auto f_r = std::async(pol, [&] {
        int8_t g_in[IN_SMALL + 2], g_row[66];
        for (int r = 0; r <= IN_SMALL + 1; ++r)
            g_in[r] = (r < 1 || r > IN_SMALL) ? 4 : r <= 4 ? 0 : r <= 8 ? 1 : r <= 16 ? 2 : 3;
        for (int r = 0; r <= 65; ++r) g_row[r] = r <= 8 ? 0 : r <= 16 ? 1 : r <= 32 ? 2 : r <= 64 ? 3 : 4;
        std::vector<int8_t> ga((size_t)n), gb((size_t)n);
        int64_t ca[5] = {0, 0, 0, 0, 0}, cr[5] = {0, 0, 0, 0, 0};
        for (int32_t m = 0; m < n; ++m) {
            const int64_t ri = Ri[m];
            const int64_t rw = (s->call_off[m + 1] - s->call_off[m]) + (s->acc_off[m + 1] - s->acc_off[m]);
            const int8_t qa = g_in[ri < IN_SMALL + 1 ? ri : IN_SMALL + 1], qb = g_row[rw < 65 ? rw : 65];
            ga[m] = qa;
            gb[m] = qb;
            ca[qa]++;
            cr[qb]++;
        }
        int64_t pa[5], pb[5];
        s->in_run_off[0] = 0;
        s->prep_run_off[0] = 0;
        for (int q = 0; q < 5; ++q) {
            pa[q] = q == 0 ? 0 : pa[q - 1] + ca[q - 1];
            pb[q] = s->prep_run_off[q];
            s->prep_run_off[q + 1] = s->prep_run_off[q] + (int)cr[q];
        }
        for (int q = 0; q < 4; ++q) s->in_run_off[q + 1] = s->in_run_off[q] + (int)ca[q];
        for (int32_t m = 0; m < n; ++m) {
            runs[pa[ga[m]]++] = m;  // group 4 (not a short caller row) lands after the four groups
            prep_runs[pb[gb[m]]++] = m;
        }
        runs.resize(s->in_run_off[4]);
    });
    // co-access work of the classes with own attributes: up to 64 attributes
    // (one MFMA k-block) and up to 64 methods, one wave each; up to 64
    // attributes and more methods, groups of four row tiles with the masks
    // staged in LDS; more than 64 attributes, single row tiles. The groups come
    // first in one buffer, the row tiles after them.
    std::vector<int2> co, co_wide;
    std::vector<int32_t> co_small;
    for (int32_t C = 0; C < c; ++C) {
        if (s->acnt[C] == 0) continue;
        int32_t nm = s->mem_end[C] - s->mem_off[C];
        if (nm == 0) continue;
        if (s->acnt[C] <= 64 && nm <= 64)
            co_small.push_back(C);
        else if (s->acnt[C] <= 64)
            for (int32_t t = 0; t * 16 < nm; t += 4) co.push_back(make_int2(C, t));
        else
            for (int32_t t = 0; t * 16 < nm; ++t) co_wide.push_back(make_int2(C, t));
    }
    s->n_co_groups = (int)co.size();
    co.insert(co.end(), co_wide.begin(), co_wide.end());
    {
        // join every pass before the first failure propagates (their captures live on this frame)
        std::exception_ptr first;
        for (auto *f : {&f_w, &f_c, &f_i, &f_r}) {
            try {
                f->get();
            } catch (...) {
                if (!first) first = std::current_exception();
            }
        }
        if (first) std::rethrow_exception(first);
    }
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    upload(ctx, cb, s->d_mem_off, s->mem_off, s->stream);
    upload(ctx, cb, s->d_mem_end, s->mem_end, s->stream);
    upload(ctx, cb, s->d_mem_idx, s->mem_idx, s->stream);
    upload_map(s, s->w, Lw, false);
    upload_map(s, s->cnt, Lc, true);
    upload_map(s, s->in, Li, true);
    upload(ctx, cb, s->in.flag_items, flag_items, s->stream);
    s->in.n_flag_items = (int)flag_items.size();
    upload(ctx, cb, s->d_co_items, co, s->stream);
    s->n_co_items = (int)co.size() - s->n_co_groups;
    upload(ctx, cb, s->d_co_small, co_small, s->stream);
    s->n_co_small = (int)co_small.size();
    // the W and CNT tables grouped by waves, as work items: a class whose W
    // table groups by a wave has its CNT table there too (its calls are a part of
    // its references), and one wave builds both when they fit MAP_HMAX slots;
    // otherwise each alone, as is the CNT table of a class whose W table is
    // filled elsewhere. Items of more than MAP_HSMALL slots first.
    std::vector<int32_t> wc;
    {
        std::vector<uint8_t> w_wave((size_t)c, 0);
        for (int32_t C : Lw.wave) w_wave[(size_t)C] = 1;
        std::vector<int32_t> small;
        auto put = [&](int32_t C, int what, int64_t need) { (need > MAP_HSMALL ? wc : small).push_back(C * 4 + what); };
        for (int32_t C : Lw.wave) {
            const MapHdr &hc = Lc.hdr[(size_t)C];
            const int64_t hw = Lw.hdr[(size_t)C].cap, hcap = hc.kind == MAP_TABLE ? hc.cap : 0;
            if (hw + hcap <= MAP_HMAX) {
                put(C, 0, hw + hcap);
            } else {
                put(C, 1, hw);
                if (hcap) put(C, 2, hcap);
            }
        }
        for (int32_t C : Lc.wave)
            if (!w_wave[(size_t)C]) put(C, 2, Lc.hdr[(size_t)C].cap);
        if ((int64_t)c * 4 > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^29 classes");
        s->n_wc_large = (int)wc.size();
        s->n_wc_small = (int)small.size();
        wc.insert(wc.end(), small.begin(), small.end());
        upload(ctx, cb, s->d_wc_list, wc, s->stream);
    }
    // the classes by member count for the aggregates (16 lanes, or a wave);
    // kept until the synchronization below, like the other uploaded lists
    std::vector<int32_t> fin((size_t)c);
    {
        int32_t lo = 0, hi = c;
        for (int32_t C = 0; C < c; ++C)
            fin[(size_t)(s->mem_end[C] - s->mem_off[C] <= FIN_SMALL ? lo++ : --hi)] = C;
        s->n_fin_small = lo;
        upload(ctx, cb, s->d_fin_list, fin, s->stream);
    }
    upload(ctx, cb, s->d_in_runs, runs, s->stream);
    upload(ctx, cb, s->d_prep_runs, prep_runs, s->stream);
    s->prep_pos.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) s->prep_pos[(size_t)prep_runs[(size_t)i]] = i;
    s->prep_host.swap(prep_runs);  // kept after the synchronization below
    s->d_meth.fit(ctx, cb, (size_t)n * sizeof(MethodAgg));
    s->d_own_mask.fit(ctx, cb, (size_t)n * sizeof(uint64_t));
    s->d_cls.fit(ctx, cb, (size_t)c * sizeof(ClassAgg));
    s->d_err.fit(ctx, cb, 16);  // error bits (int) at 0, kept count (int64) at 8
    fill_i32(s->d_err.as<int32_t>(), 0, 4, s->stream);  // error bits stay set until reported
    HIPCHK(hipStreamSynchronize(s->stream));
    incr_reset(s, Rw, Rc);
    s->layout_valid = true;
}

MapOut map_out(DevMap &m) {
    return MapOut{m.hdr.as<MapHdr>(), m.foreign.as<int32_t>(), m.keys.as<int32_t>(), m.vals.as<int32_t>()};
}
MapView map_view(DevMap &m) { return MapView{m.hdr.as<MapHdr>(), m.keys.as<int32_t>(), m.vals.as<int32_t>()}; }
BigWork big_work(mm_system *s) {
    BigWork b;
    DevMap *dm[3] = {&s->w, &s->cnt, &s->in};
    b.np_max = 1;
    for (int q = 0; q < 3; ++q) {
        b.m[q] = BigMap{dm[q]->big_items.as<BigItem>(), dm[q]->big_parts.as<BigPart>(), dm[q]->n_big_items,
                        dm[q]->n_big_parts, dm[q]->big_stage.as<int2>(), dm[q]->big_bt.as<int32_t>(), map_out(*dm[q])};
        b.np_max = std::max(b.np_max, dm[q]->np_max);
    }
    b.lds_slots = big_lds_slots(s->big_chunk);
    return b;
}

// The error word and the kept count, as the host reads them back.
struct StatusWords {
    int32_t err, pad;
    int64_t kept;
};

// Where the last kernel of a pass may store the status words itself (the
// mapped pinned block), or NULL: then they are copied back from the device.
int32_t *status_device_slot(mm_system *s) {
    return s->status_host.get(sizeof(StatusWords)) ? static_cast<int32_t *>(s->status_host.dev) : nullptr;
}

// device_wrote: the pass's last kernel stored both words in the pinned block
// (status_device_slot), so only the stream has to finish.
void check_kernel_errors(mm_system *s, int64_t *kept = nullptr, bool device_wrote = false) {
    // the error word and, when asked, the kept count k_compact stored beside it
    StatusWords local{0, 0, 0};
    StatusWords *st = static_cast<StatusWords *>(s->status_host.get(sizeof(StatusWords)));
    if (!st) {
        st = &local;
        device_wrote = false;
    }
    if (!device_wrote)
        HIPCHK(hipMemcpyAsync(st, s->d_err.p, kept ? 16 : sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int err = *static_cast<volatile int32_t *>(&st->err);
    if (kept) *kept = *static_cast<volatile int64_t *>(&st->kept);
    if (err) fill_i32(s->d_err.as<int32_t>(), 0, 1, s->stream);  // reported once, then cleared
    if (err & ERR_MAP_OVERFLOW) {
        s->metrics_valid = false;
        s->incr.base = false;
        fail(MM_EINTERNAL, "grouped-count table overflow");
    }
    if (err & ERR_CYCLE) fail(MM_EINVAL, "the class hierarchy has a cycle");
    if (err & ERR_HEAVY_OVERFLOW) fail(MM_EINTERNAL, "caller-class work list overflow");
    if (err & ERR_SCAN) {
        s->scan.need_clear = true;  // clear the work area before its next use
        fail(MM_EINTERNAL, "prefix sum gave up waiting for a tile");
    }
    if (err) fail(MM_EINTERNAL, "kernel reported error bits " + std::to_string(err));
}

}  // namespace

#include "mm_incr_impl.h"

namespace {

void ensure_metrics(mm_system *s, ClassAgg *cls_dst = nullptr, MethodAgg *meth_dst = nullptr) {
    if (!s->structure_valid) {  // an earlier upload stopped part way (out of memory)
        upload_structure(s);
        s->structure_valid = true;
    }
    if (!s->metrics_valid && s->incr.active && s->layout_valid) {
        dirty_recompute(s, cls_dst, meth_dst);  // only what the moves since the last recompute touched
        s->metrics_valid = true;
        return;
    }
    if (!s->layout_valid) build_layout(s);
    hipStream_t st = s->stream;
    if (s->metrics_valid) {
        if (cls_dst && s->c)
            HIPCHK(hipMemcpyAsync(cls_dst, s->d_cls.p, (size_t)s->c * sizeof(ClassAgg), hipMemcpyDeviceToDevice, st));
        if (meth_dst && s->n)
            HIPCHK(hipMemcpyAsync(meth_dst, s->d_meth.p, (size_t)s->n * sizeof(MethodAgg), hipMemcpyDeviceToDevice,
                                  st));
        return;
    }
    // a full recompute needs work lists of the current membership, made with the
    // schedule's fill items
    if (s->incr.stale || s->layout_fill != s->ctx->tuning.fill_chunk)
        build_layout(s);
    ensure_entry_classes(s);
    MetricsPlan p;
    memset(&p, 0, sizeof(p));
    p.meth = s->d_meth.as<MethodAgg>();
    p.cls = s->d_cls.as<ClassAgg>();
    p.own_mask = s->d_own_mask.as<uint64_t>();
    p.w = map_out(s->w);
    p.cnt = map_out(s->cnt);
    p.in = map_out(s->in);
    p.in_wave = s->in.wave.as<int32_t>();
    p.n_in_wave = s->in.n_wave;
    p.w_mid = s->w.mid.as<int32_t>();
    p.n_w_mid = s->w.n_mid;
    p.cnt_mid = s->cnt.mid.as<int32_t>();
    p.n_cnt_mid = s->cnt.n_mid;
    p.big = big_work(s);
    p.in_runs = s->d_in_runs.as<int32_t>();
    for (int q = 0; q < 5; ++q) p.in_run_off[q] = s->in_run_off[q];
    p.in_flag_items = s->in.flag_items.as<int4>();
    p.n_in_flag = s->in.n_flag_items;
    p.co_groups = s->d_co_items.as<int2>();
    p.n_co_groups = s->n_co_groups;
    p.co_items = s->d_co_items.as<int2>() + s->n_co_groups;
    p.n_co_items = s->n_co_items;
    p.co_small = s->d_co_small.as<int32_t>();
    p.n_co_small = s->n_co_small;
    p.wc = MapWcWork{s->d_wc_list.as<int32_t>(), s->n_wc_large, s->n_wc_small};
    p.fin_list = s->d_fin_list.as<int32_t>();
    p.n_fin_small = s->n_fin_small;
    p.n_fin_large = s->c - s->n_fin_small;
    p.err = s->d_err.as<int>();
    p.timer = s->ctx->timer.enabled() ? &s->ctx->timer : nullptr;
    p.cls_out = cls_dst;
    p.meth_out = meth_dst;
    const DevSys d = s->view();
    // timing every kernel (a per-kernel census) runs the two chains one after
    // the other on the context stream, so each event pair holds its own kernel
    // only; timing named kernels keeps the chains concurrent
    const AuxStreams *ax = s->ctx->timer.pattern == "*" ? nullptr : aux_for(s->ctx, st);
    launch_compute_metrics(d, p, st, ax);  // k_finalize also fills the caller's buffers
    HIPCHK(hipGetLastError());
    s->metrics_valid = true;
    s->incr.base = true;
    s->maps_event = ax != nullptr;  // this launch's fork and W/CNT events (ev[0], ev[5] of st's aux set)
    s->maps_stream = st;
}

void invalidate(mm_system *s, bool structure) {
    ++s->version;
    s->metrics_valid = false;
    s->maps_event = false;
    s->cache.valid = false;
    if (structure) s->layout_valid = false;
}

// the system's prefix-sum work area, large enough for n elements
ScanArea &scan_area(mm_system *s, int64_t n) {
    void *before = s->s_tmp.p;
    s->s_tmp.reserve(s->ctx, &s->bytes, (size_t)scan_area_elems(std::max<int64_t>(n, 1)) * 8);
    if (s->s_tmp.p != before || s->scan.dev != s->s_tmp.as<int64_t>()) {
        s->scan.dev = s->s_tmp.as<int64_t>();
        s->scan.need_clear = true;  // new block: cleared before its first scan
    }
    s->scan.cap_words = (int64_t)(s->s_tmp.bytes / 8);
    s->scan.err = s->d_err.as<int>();
    return s->scan;
}

mm_system *checked_sys(mm_system *s) {
    if (!s) fail(MM_EINVAL, "system handle is NULL");
    set_device(s->ctx);
    return s;
}

void load_impl(mm_context *ctx, const mm_system_desc *dsc, mm_system **out, hipStream_t st = nullptr) {
    if (!ctx || !dsc || !out) fail(MM_EINVAL, "NULL argument");
    set_device(ctx);
    const int64_t c = dsc->n_classes, n = dsc->n_methods, na = dsc->n_attrs;
    if (c < 0 || n < 0 || na < 0) fail(MM_EINVAL, "negative size");
    if (c >= (1 << 30)) fail(MM_EOVERFLOW, "more than 2^30 classes");
    if (n > 0 && !dsc->method_class) fail(MM_EINVAL, "method_class is NULL");
    if (na > 0 && !dsc->attr_class) fail(MM_EINVAL, "attr_class is NULL");
    for (int64_t i = 0; i < n; ++i)
        if (dsc->method_class[i] < 0 || dsc->method_class[i] >= c)
            fail(MM_EINVAL, "method_class out of range at method " + std::to_string(i));
    for (int64_t i = 0; i < na; ++i)
        if (dsc->attr_class[i] < 0 || dsc->attr_class[i] >= c)
            fail(MM_EINVAL, "attr_class out of range at attribute " + std::to_string(i));
    check_csr("acc", dsc->acc_off, dsc->acc_idx, n, na);
    check_csr("call", dsc->call_off, dsc->call_idx, n, n);
    if (dsc->acc_off[n] + dsc->call_off[n] > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 references");

    mm_system *s = new mm_system();
    try {
        s->ctx = ctx;
        s->stream = st ? st : ctx->stream;
        s->c = (int32_t)c;
        s->n = (int32_t)n;
        s->na = (int32_t)na;
        s->owner.assign(dsc->method_class, dsc->method_class + n);
        s->acls.assign(dsc->attr_class, dsc->attr_class + na);
        s->acnt.assign(c, 0);
        s->alocal.assign(na, 0);
        for (int64_t a = 0; a < na; ++a) s->alocal[a] = s->acnt[s->acls[a]]++;
        canonical_rows(dsc->acc_off, dsc->acc_idx, n, s->acc_off, s->acc_idx);
        canonical_rows(dsc->call_off, dsc->call_idx, n, s->call_off, s->call_idx);
        upload_structure(s);
        s->structure_valid = true;
        build_layout(s);
    } catch (...) {
        delete s;
        throw;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        ctx->n_systems++;
    }
    *out = s;
}

void load_batch_impl(mm_context *ctx, const mm_system_desc *descs, int32_t n_sys, mm_system **out) {
    if (!ctx || !descs || !out || n_sys <= 0) fail(MM_EINVAL, "bad batch arguments");
    int64_t C = 0, N = 0, A = 0, NA = 0, NC = 0;
    for (int32_t i = 0; i < n_sys; ++i) {
        const mm_system_desc &d = descs[i];
        if (d.n_classes < 0 || d.n_methods < 0 || d.n_attrs < 0) fail(MM_EINVAL, "negative size in batch part");
        if (!d.acc_off || !d.call_off) fail(MM_EINVAL, "batch part offsets are NULL");
        C += d.n_classes;
        N += d.n_methods;
        A += d.n_attrs;
        NA += d.acc_off[d.n_methods];
        NC += d.call_off[d.n_methods];
    }
    if (C >= (1 << 30) || N > INT32_MAX || A > INT32_MAX || NA > INT32_MAX || NC > INT32_MAX)
        fail(MM_EOVERFLOW, "batch exceeds the id ranges of one system");
    std::vector<int32_t> mc(N), ac(A), ai(NA), ci(NC);
    std::vector<int64_t> ao(N + 1, 0), co(N + 1, 0);
    std::vector<int32_t> pc(n_sys + 1, 0), pm(n_sys + 1, 0), pa(n_sys + 1, 0);
    int64_t c0 = 0, m0 = 0, a0 = 0, e0 = 0, f0 = 0;
    for (int32_t i = 0; i < n_sys; ++i) {
        const mm_system_desc &d = descs[i];
        if ((d.n_methods > 0 && !d.method_class) || (d.n_attrs > 0 && !d.attr_class))
            fail(MM_EINVAL, "batch part " + std::to_string(i) + " has NULL arrays");
        for (int32_t k = 0; k < d.n_methods; ++k) {
            int32_t x = d.method_class[k];
            if (x < 0 || x >= d.n_classes) fail(MM_EINVAL, "batch part " + std::to_string(i) + ": method_class out of range");
            mc[m0 + k] = (int32_t)(x + c0);
        }
        for (int32_t k = 0; k < d.n_attrs; ++k) {
            int32_t x = d.attr_class[k];
            if (x < 0 || x >= d.n_classes) fail(MM_EINVAL, "batch part " + std::to_string(i) + ": attr_class out of range");
            ac[a0 + k] = (int32_t)(x + c0);
        }
        check_csr("batch acc", d.acc_off, d.acc_idx, d.n_methods, d.n_attrs);
        check_csr("batch call", d.call_off, d.call_idx, d.n_methods, d.n_methods);
        for (int64_t k = 0; k < d.acc_off[d.n_methods]; ++k) ai[e0 + k] = (int32_t)(d.acc_idx[k] + a0);
        for (int64_t k = 0; k < d.call_off[d.n_methods]; ++k) ci[f0 + k] = (int32_t)(d.call_idx[k] + m0);
        for (int32_t k = 0; k <= d.n_methods; ++k) {
            ao[m0 + k] = e0 + d.acc_off[k];
            co[m0 + k] = f0 + d.call_off[k];
        }
        c0 += d.n_classes;
        m0 += d.n_methods;
        a0 += d.n_attrs;
        e0 += d.acc_off[d.n_methods];
        f0 += d.call_off[d.n_methods];
        pc[i + 1] = (int32_t)c0;
        pm[i + 1] = (int32_t)m0;
        pa[i + 1] = (int32_t)a0;
    }
    mm_system_desc u{(int32_t)C, (int32_t)N, (int32_t)A, mc.data(), ac.data(), ao.data(), ai.data(), co.data(), ci.data()};
    load_impl(ctx, &u, out);
    (*out)->part_cls = std::move(pc);
    (*out)->part_meth = std::move(pm);
    (*out)->part_attr = std::move(pa);
}

struct ScoreArgs {
    int32_t mode;
    const int32_t *cm, *ct;
    int64_t n_cand;
    uint32_t mask;
    int32_t rule, keep_only;
    int32_t origin = 0;  // ranked suggestions: 1 / 2 keep only origins above the average LCOM / CBO
};

void validate_score_args(mm_system *s, const ScoreArgs &a) {
    if (a.mode < 0 || a.mode > 3) fail(MM_EINVAL, "bad candidate mode");
    if (a.mode == MM_CAND_ALL && s->part_cls.size() > 2)
        fail(MM_EINVAL, "ALL candidates would cross systems of a batch; use REFERENCED or EXPLICIT");
    if (a.mode == MM_CAND_SIMILAR && s->part_cls.size() > 2)
        fail(MM_EINVAL, "similarity of a batch would average over several systems");
    if (a.mask & ~15u) fail(MM_EINVAL, "bad metric mask");
    if (a.rule < 0 || a.rule > 2) fail(MM_EINVAL, "bad rule");
    if (a.rule == MM_RULE_PAPER_LCOM && !(a.mask & (MM_LCOM_PQ | MM_LCOM_HS)))
        fail(MM_EINVAL, "PAPER_LCOM needs MM_LCOM_PQ or MM_LCOM_HS in the mask");
    if (a.rule == MM_RULE_PAPER_CBO && !(a.mask & MM_CBO)) fail(MM_EINVAL, "PAPER_CBO needs MM_CBO in the mask");
    if (a.keep_only != 0 && a.keep_only != 1) fail(MM_EINVAL, "keep_only must be 0 or 1");
    if (a.mode == MM_CAND_EXPLICIT) {
        if (a.n_cand < 0) fail(MM_EINVAL, "negative candidate count");
        if (a.n_cand > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 candidates");
        if (a.n_cand > 0 && (!a.cm || !a.ct)) fail(MM_EINVAL, "candidate arrays are NULL");
        for (int64_t k = 0; k < a.n_cand; ++k) {
            int32_t m = a.cm[k], T = a.ct[k];
            if (m < 0 || m >= s->n) fail(MM_EINVAL, "candidate method out of range at " + std::to_string(k));
            if (T < 0 || T >= s->c) fail(MM_EINVAL, "candidate class out of range at " + std::to_string(k));
            if (s->owner[m] == T) fail(MM_EINVAL, "candidate " + std::to_string(k) + " moves a method to its own class");
            if (s->part_cls.size() > 2) {
                auto pm = std::upper_bound(s->part_meth.begin(), s->part_meth.end(), m) - s->part_meth.begin();
                auto pc = std::upper_bound(s->part_cls.begin(), s->part_cls.end(), T) - s->part_cls.begin();
                if (pm != pc) fail(MM_EINVAL, "candidate " + std::to_string(k) + " crosses systems of a batch");
            }
        }
    }
}

bool cache_hit(mm_system *s, const ScoreArgs &a) {
    auto &C = s->cache;
    if (!C.valid || C.version != s->version || C.mode != a.mode || C.mask != a.mask || C.rule != a.rule ||
        C.keep_only != a.keep_only || C.origin != a.origin)
        return false;
    if (a.mode == MM_CAND_SIMILAR && C.sim_threshold != s->sim_threshold) return false;
    if (a.mode == MM_CAND_EXPLICIT) {
        if (C.n_cand != a.n_cand) return false;
        if (a.n_cand && (memcmp(C.cm.data(), a.cm, a.n_cand * 4) || memcmp(C.ct.data(), a.ct, a.n_cand * 4)))
            return false;
    }
    return true;
}

int64_t map_slots_host(const MapHdr &h) {
    return h.kind == MAP_TABLE ? h.cap : (h.kind == MAP_RUN ? h.cap : 0);
}

// Bounds of the heavy caller-class work: (candidate, chunk) items and candidates.
}  // namespace

#include "mm_sim_impl.h"

namespace {

void heavy_bounds(mm_system *s, const ScoreArgs &a, int64_t &items, int64_t &cands) {
    items = cands = 0;
    const mm_tuning &tu = s->ctx->tuning;
    auto &hc = s->hb_cache;
    if (a.mode != MM_CAND_EXPLICIT && a.mode != MM_CAND_SIMILAR && hc.version == s->version && hc.mode == a.mode &&
        hc.caller_light == tu.caller_light && hc.heavy_chunk == tu.heavy_chunk) {
        items = hc.heavy_items;
        cands = hc.heavy_cands;
        return;
    }
    const int32_t n = s->n, c = s->c;
    std::vector<int64_t> ch(n, 0);
    bool any = false;
    for (int32_t m = 0; m < n; ++m) {
        if (s->rc_off[m + 1] - s->rc_off[m] <= tu.caller_light) continue;
        const MapHdr &h = s->in.host_hdr[m];
        ch[m] = ((int64_t)map_slots_host(h) + tu.heavy_chunk - 1) / tu.heavy_chunk;
        any = true;
    }
    if (any && a.mode == MM_CAND_SIMILAR) {
        for (int32_t m = 0; m < n; ++m)
            if (ch[m] && s->sim.row_cands[m]) {
                items += ch[m] * s->sim.row_cands[m];
                cands += s->sim.row_cands[m];
            }
        return;  // depends on the threshold: not cached here
    }
    for (int32_t m = 0; any && m < n && a.mode != MM_CAND_EXPLICIT; ++m) {
        if (!ch[m]) continue;
        int64_t k = c - 1;
        if (a.mode == MM_CAND_REFERENCED) {
            int64_t refs = (s->acc_off[m + 1] - s->acc_off[m]) + (s->call_off[m + 1] - s->call_off[m]);
            k = std::min<int64_t>(refs, c - 1);
        }
        items += ch[m] * k;
        cands += k;
    }
    if (any && a.mode == MM_CAND_EXPLICIT)
        for (int64_t k = 0; k < a.n_cand; ++k)
            if (ch[a.cm[k]]) {
                items += ch[a.cm[k]];
                cands += 1;
            }
    if (a.mode != MM_CAND_EXPLICIT) hc = {s->version, a.mode, tu.caller_light, tu.heavy_chunk, items, cands};
}

// Run the scoring pipeline. Records go to `direct` when it can hold every
// record (keep_only = 0), else to the scratch s_rec.
void score_run(mm_system *s, const ScoreArgs &a, MoveRec *direct, int64_t direct_cap) {
    mm_context *ctx = s->ctx;
    hipStream_t st = s->stream;
    int64_t *cb = &s->bytes;
    ensure_metrics(s);
    ensure_entry_classes(s);  // current already after any recompute
    const int32_t n = s->n, c = s->c;
    const int64_t nref = (int64_t)s->acc_idx.size() + (int64_t)s->call_idx.size();
    // Right after a full metric launch on this stream, the first pass (k_prep
    // and its prefix sums) needs only the W and CNT maps: it runs on a side
    // stream from the launch's event for them, beside the caller-map phase. A
    // keep_only pass leaves the origin's map terms to the candidates that need
    // them, so its first pass reads no map at all and starts from the launch's
    // fork instead, beside the whole recompute. All earlier work on the stream
    // precedes either event, so no buffer of an earlier call is still in use.
    // Any other time it runs on the stream itself.
    // (on a small system the step is bound by issuing launches, and the events
    // and the extra pass would cost more than the overlap gains)
    const AuxStreams *ax =
        s->maps_event && s->maps_stream == st && s->n >= PREP_SIDE_MIN ? aux_for(ctx, st) : nullptr;
    s->maps_event = false;
    const hipStream_t sp = ax ? ax->s[1] : st;

    s->s_prep.reserve(ctx, cb, (size_t)n * sizeof(MethodPrep));
    s->s_outk.reserve(ctx, cb, (size_t)nref * 4);
    s->s_outc.reserve(ctx, cb, (size_t)nref * 4);
    s->s_outa.reserve(ctx, cb, (size_t)nref * 4);
    s->s_counts.reserve(ctx, cb, 32);

    ScorePlan p;
    memset(&p, 0, sizeof(p));
    p.mode = a.mode;
    p.mask = a.mask;
    p.rule = a.rule;
    p.keep_only = a.keep_only;
    p.lazy_src = a.keep_only;  // few candidates get past the LCOM stage: their origin terms come later
    p.prep_in_late = ax != nullptr;  // then the caller terms come after the join
    p.cm1 = c - 1;
    p.meth = s->d_meth.as<MethodAgg>();
    p.cls = s->d_cls.as<ClassAgg>();
    p.own_mask = s->d_own_mask.as<uint64_t>();
    p.w = map_view(s->w);
    p.cnt = map_view(s->cnt);
    p.in = map_view(s->in);
    p.in_own = s->in.foreign.as<int32_t>();
    p.prep = s->s_prep.as<MethodPrep>();
    p.prep_runs = s->d_prep_runs.as<int32_t>();
    for (int q = 0; q < 6; ++q) p.prep_run_off[q] = s->prep_run_off[q];
    p.outk = s->s_outk.as<int32_t>();
    p.outc = s->s_outc.as<int32_t>();
    p.outa = s->s_outa.as<int32_t>();
    p.delta_next = s->s_counts.as<int32_t>() + 2;  // 8-byte counter at offset 8
    p.origin = a.origin;
    p.origin_sum = (const long long *)(s->s_counts.as<char>() + 16);
    p.caller_light = ctx->tuning.caller_light;
    p.heavy_chunk = ctx->tuning.heavy_chunk;
    p.delta_chunk = ctx->tuning.delta_chunk;
    p.delta_grid = ctx->tuning.delta_grid > 0 ? ctx->tuning.delta_grid : ctx->n_cu * 8;
    p.err = s->d_err.as<int>();
    p.timer = ctx->timer.enabled() ? &ctx->timer : nullptr;
    const DevSys d = s->view();
    const bool ref = a.mode == MM_CAND_REFERENCED;
    // The candidate count is known before any launch for ALL, and for REFERENCED
    // once counted on this structure: then every buffer is sized first and all
    // launches form one sequence. Otherwise
    // the count comes back from the device (REFERENCED), the similarity pass or
    // the caller between the two stages.
    int64_t n_cand = -1;
    if (ref && s->ref_version == s->version) n_cand = s->ref_count;
    if (a.mode == MM_CAND_ALL) {
        n_cand = (c > 1) ? (int64_t)n * (c - 1) : 0;
        if (n_cand > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 candidates in ALL mode");
    }
    const bool one_sequence = n_cand >= 0;
    // the candidate arrays read only the first pass's results: when their
    // buffers are sized before it (one sequence) and it reads no map, they are
    // filled on the side stream too, before the join
    const bool ref_early = ref && one_sequence && ax && p.lazy_src;
    if (ref) {
        // the destination lists of the co-access step are counted in k_prep
        // and filled in k_ref_fill
        s->s_refcnt.reserve(ctx, cb, (size_t)n * 4);
        s->s_candoff.reserve(ctx, cb, ((size_t)n + 1) * 8);
        s->s_gcnt.reserve(ctx, cb, ((size_t)c + GCNT_TAIL) * 4);
        s->s_goff.reserve(ctx, cb, ((size_t)c + 1) * 8);
        s->s_gslot.reserve(ctx, cb, (size_t)std::max<int64_t>({nref, n_cand, 1}) * 4);
        p.gcnt = s->s_gcnt.as<int32_t>();
        p.goff = s->s_goff.as<int64_t>();
        p.gslot = s->s_gslot.as<int32_t>();
        p.grouped = 1;
        p.cand_off = s->s_candoff.as<int64_t>();
    }
    ScanArea *sa = nullptr;
    bool compacted = false;
    auto stage1 = [&] {
        if (a.origin) {  // the class sum behind the above-average test
            fill_i32(s->s_counts.as<int32_t>() + 4, 0, 2, st);
            launch_class_sum(s->d_cls.as<ClassAgg>(), c, a.origin, (long long *)(s->s_counts.as<char>() + 16), st);
        }
        if (ax) HIPCHK(hipStreamWaitEvent(sp, p.lazy_src ? ax->ev[0] : ax->ev[5], 0));  // fork, or W and CNT done
        if (ref) {
            fill_i32(p.gcnt, 0, (int64_t)c + GCNT_TAIL, sp);  // destination counts and the counters after them
            launch_prep(d, p, s->s_refcnt.as<int32_t>(), sp);
            scan2_i32(s->s_refcnt.as<int32_t>(), s->s_candoff.as<int64_t>(), n, p.gcnt, p.goff, c, *sa, sp, p.timer);
            if (ref_early) launch_ref_fill(d, p, sp);
        } else {
            launch_prep(d, p, nullptr, sp);
        }
        if (ax) {  // join: the caller terms read the complete caller maps
            HIPCHK(hipEventRecord(ax->ev[6], sp));
            HIPCHK(hipStreamWaitEvent(st, ax->ev[6], 0));
            launch_prep_in(d, p, st);
        }
    };
    // buffers sized by the candidate count
    auto prepare2 = [&] {
        if (ref) {
            s->s_cm.reserve(ctx, cb, (size_t)n_cand * 4);
            s->s_ct.reserve(ctx, cb, (size_t)n_cand * 4);
            s->s_ce.reserve(ctx, cb, (size_t)n_cand * 4);
            p.cm = s->s_cm.as<int32_t>();
            p.ct = s->s_ct.as<int32_t>();
            p.ce = s->s_ce.as<int32_t>();
        }
        p.n_cand = n_cand;
        s->s_gcnt.reserve(ctx, cb, ((size_t)c + GCNT_TAIL) * 4);
        s->s_goff.reserve(ctx, cb, ((size_t)c + 1) * 8);
        s->s_gslot.reserve(ctx, cb, (size_t)n_cand * 4);
        s->s_glist.reserve(ctx, cb, (size_t)std::max<int64_t>(n_cand, 1) * 4);
        s->s_hval.reserve(ctx, cb, (size_t)n_cand * 4);
        p.gcnt = s->s_gcnt.as<int32_t>();
        p.goff = s->s_goff.as<int64_t>();
        p.gslot = s->s_gslot.as<int32_t>();
        p.glist = s->s_glist.as<int32_t>();
        p.hval = s->s_hval.as<int32_t>();
        // the two work-list counters sit after the destination counts, so that
        // one fill clears both
        p.heavy_count = p.gcnt + c + 2;
        p.hcand_count = p.gcnt + c + 3;

        int64_t heavy_items, heavy_cands;
        heavy_bounds(s, a, heavy_items, heavy_cands);
        s->s_heavy.reserve(ctx, cb, (size_t)std::max<int64_t>(heavy_items, 1) * sizeof(int2));
        s->s_hcand.reserve(ctx, cb, (size_t)std::max<int64_t>(heavy_cands, 1) * 4);
        p.heavy = s->s_heavy.as<int2>();
        p.heavy_cap = heavy_items;
        p.hcand = s->s_hcand.as<int32_t>();
        p.hcand_cap = heavy_cands;

        const bool external = !a.keep_only && direct && direct_cap >= n_cand;
        if (external) {
            p.rec = direct;
        } else {
            s->s_rec.reserve(ctx, cb, (size_t)n_cand * sizeof(MoveRec));
            p.rec = s->s_rec.as<MoveRec>();
        }
        if (a.keep_only) {
            s->s_flags.reserve(ctx, cb, (size_t)n_cand * 4);
            s->s_kpos.reserve(ctx, cb, ((size_t)n_cand + 1) * 8);
            p.flags = s->s_flags.as<int32_t>();
            p.kpos = s->s_kpos.as<int64_t>();
            if (direct && direct_cap > 0 && n_cand > 0) {
                // kept records straight into the caller's device buffer, before the
                // count comes back (nothing is written if they do not fit); the
                // count itself lands beside the error word
                p.compact_cap = direct_cap;
                p.kept_out = (long long *)(s->d_err.as<char>() + 8);
                compacted = true;
                // kept candidates also join a short list that one block puts in
                // order; the scan of the keep flags takes over when it overflows
                s->s_kept_idx.reserve(ctx, cb, (size_t)KEPT_FAST_MAX * 4);
                p.kept_idx = s->s_kept_idx.as<int32_t>();
                p.kept_count = p.gcnt + c + 4;
                p.kept_over = p.gcnt + c + 5;
                p.kept_cap = KEPT_FAST_MAX;
                p.status_dev = status_device_slot(s);  // k_kept_order stores the status words there
            }
        }
        return external;
    };
    auto stage2 = [&] {
        if (ref && !ref_early) launch_ref_fill(d, p, st);
        launch_score(d, p, *sa, st);
        if (a.keep_only) {
            if (compacted)
                launch_kept_order(p, direct, st);
            else
                scan_i32(p.flags, p.kpos, n_cand, *sa, st, p.timer);
        }
    };
    bool external = false;
    if (one_sequence) {
        external = prepare2();
        sa = &scan_area(s, std::max<int64_t>((int64_t)n + c, n_cand));  // n + c: both stage-1 scans in one launch
        stage1();
        stage2();
    } else {
        sa = &scan_area(s, (int64_t)n + c);  // both stage-1 scans in one launch
        stage1();
        if (ref) {
            HIPCHK(hipMemcpyAsync(&n_cand, s->s_candoff.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            s->ref_version = s->version;
            s->ref_count = n_cand;
            if (n_cand > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 REFERENCED candidates");
        } else if (a.mode == MM_CAND_SIMILAR) {
            n_cand = sim_candidates(s, s->sim_threshold, s->s_cm, s->s_ct);
            p.cm = s->s_cm.as<int32_t>();
            p.ct = s->s_ct.as<int32_t>();
            p.mode = MM_CAND_EXPLICIT;  // scored as a device-resident explicit list
        } else {
            n_cand = a.n_cand;
            s->s_cm.reserve(ctx, cb, (size_t)n_cand * 4);
            s->s_ct.reserve(ctx, cb, (size_t)n_cand * 4);
            if (n_cand) {
                HIPCHK(hipMemcpyAsync(s->s_cm.p, a.cm, n_cand * 4, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->s_ct.p, a.ct, n_cand * 4, hipMemcpyHostToDevice, st));
            }
            p.cm = s->s_cm.as<int32_t>();
            p.ct = s->s_ct.as<int32_t>();
        }
        external = prepare2();
        sa = &scan_area(s, std::max<int64_t>(c, n_cand));
        stage2();
    }
    int64_t n_out = n_cand;
    if (a.keep_only && !compacted) HIPCHK(hipMemcpyAsync(&n_out, p.kpos + n_cand, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipGetLastError());
    check_kernel_errors(s, compacted ? &n_out : nullptr, compacted && p.status_dev);  // synchronizes
    if (compacted && (n_out > p.kept_cap || n_out > direct_cap)) {
        // a long kept list, or one the caller's buffer cannot take: the ordered
        // scan of the keep flags lays the records out (and keeps them available
        // to a later call with a larger buffer)
        scan_i32(p.flags, p.kpos, n_cand, *sa, st, p.timer);
        launch_compact(p, direct, st);
        HIPCHK(hipGetLastError());
        check_kernel_errors(s, &n_out);
    }

    auto &C = s->cache;
    C.valid = true;
    C.version = s->version;
    C.mode = a.mode;
    C.mask = a.mask;
    C.rule = a.rule;
    C.keep_only = a.keep_only;
    C.n_cand = n_cand;
    C.n_out = n_out;
    C.rec_external = external || (compacted && n_out <= direct_cap);
    C.sim_threshold = s->sim_threshold;
    C.origin = a.origin;
    if (a.mode == MM_CAND_EXPLICIT) {
        C.cm.assign(a.cm, a.cm + n_cand);
        C.ct.assign(a.ct, a.ct + n_cand);
    } else {
        C.cm.clear();
        C.ct.clear();
    }
}

ScorePlan compact_plan(mm_system *s) {
    ScorePlan p;
    memset(&p, 0, sizeof(p));
    p.timer = s->ctx->timer.enabled() ? &s->ctx->timer : nullptr;
    p.n_cand = s->cache.n_cand;
    p.rec = s->s_rec.as<MoveRec>();
    p.flags = s->s_flags.as<int32_t>();
    p.kpos = s->s_kpos.as<int64_t>();
    p.compact_cap = INT64_MAX;
    return p;
}

void score_impl(mm_system *s, const ScoreArgs &a, mm_move_score *out, bool device_out, int64_t cap,
                int64_t *n_out) {
    if (!n_out) fail(MM_EINVAL, "n_out is NULL");
    validate_score_args(s, a);
    // A count query (out == NULL) always scores; the next call with a buffer and
    // the same arguments takes those results. Any other call scores afresh.
    if (!out || !cache_hit(s, a) || s->cache.rec_external)
        score_run(s, a, device_out ? (MoveRec *)out : nullptr, device_out ? cap : 0);
    const int64_t need = s->cache.n_out;
    *n_out = need;
    if (!out) return;
    s->cache.valid = false;
    if (cap < need) fail(MM_ERANGE, "output capacity " + std::to_string(cap) + " < " + std::to_string(need));
    if (need == 0 || s->cache.rec_external) return;
    mm_context *ctx = s->ctx;
    hipStream_t st = s->stream;
    const size_t bytes = (size_t)need * sizeof(MoveRec);
    if (a.keep_only) {
        if (device_out) {
            launch_compact(compact_plan(s), (MoveRec *)out, st);
            HIPCHK(hipGetLastError());
        } else {
            s->s_kept.reserve(ctx, &s->bytes, bytes);
            launch_compact(compact_plan(s), s->s_kept.as<MoveRec>(), st);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(out, s->s_kept.p, bytes, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
    } else {
        HIPCHK(hipMemcpyAsync(out, s->s_rec.p, bytes, device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (!device_out) HIPCHK(hipStreamSynchronize(st));
    }
}

// Time the scoring pipeline under a few schedules (coordinate search over the
// delta kernel's schedule, the inline caller-class threshold and the heavy
// chunk) and keep the fastest in the context. Results never depend on these.
void autotune_impl(mm_system *s, const ScoreArgs &a, int32_t repeats, mm_tuning *best) {
    validate_score_args(s, a);
    if (repeats < 1) repeats = 1;
    mm_context *ctx = s->ctx;
    ensure_metrics(s);
    check_kernel_errors(s);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_cfg = [&](const mm_tuning &t) {
        ctx->tuning = t;
        float bestms = 1e30f;
        for (int r = 0; r < repeats; ++r) {
            HIPCHK(hipEventRecord(e0, s->stream));
            score_run(s, a, nullptr, 0);
            HIPCHK(hipEventRecord(e1, s->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            bestms = std::min(bestms, ms);
        }
        return bestms;
    };
    mm_tuning cur = ctx->tuning;
    float tcur = 0;
    try {
        score_run(s, a, nullptr, 0);  // warm the scratch buffers
        tcur = time_cfg(cur);
        const int32_t g8 = ctx->n_cu * 8, g4 = ctx->n_cu * 4;
        const int32_t sched[][2] = {{0, 0}, {256, g8}, {1024, g8}, {4096, g4}};
        for (auto &sc : sched) {
            mm_tuning t = cur;
            t.delta_chunk = sc[0];
            t.delta_grid = sc[1];
            float ms = time_cfg(t);
            if (ms < tcur) { cur = t; tcur = ms; }
        }
        for (int32_t cl : {2, 4, 8, 16, 32}) {
            mm_tuning t = cur;
            t.caller_light = cl;
            float ms = time_cfg(t);
            if (ms < tcur) { cur = t; tcur = ms; }
        }
        for (int32_t hc : {64, 256, 1024}) {
            mm_tuning t = cur;
            t.heavy_chunk = hc;
            float ms = time_cfg(t);
            if (ms < tcur) { cur = t; tcur = ms; }
        }
        // the metric recompute's fill items: the whole step (a full recompute,
        // then the scoring call), the layout rebuilt untimed for each setting
        auto time_step = [&](const mm_tuning &t) {
            ctx->tuning = t;
            s->metrics_valid = false;
            ensure_metrics(s);  // rebuilds the layout when the fill items change
            float bestms = 1e30f;
            for (int r = 0; r < repeats; ++r) {
                s->metrics_valid = false;
                s->cache.valid = false;
                HIPCHK(hipEventRecord(e0, s->stream));
                ensure_metrics(s);
                score_run(s, a, nullptr, 0);
                HIPCHK(hipEventRecord(e1, s->stream));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                bestms = std::min(bestms, ms);
            }
            return bestms;
        };
        float tstep = time_step(cur);
        for (int32_t fc : {256, 512, 1024, 2048}) {
            mm_tuning t = cur;
            t.fill_chunk = fc;
            float ms = time_step(t);
            if (ms < tstep) { cur = t; tstep = ms; }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->tuning = cur;
        s->cache.valid = false;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuning = cur;
    s->cache.valid = false;
    if (best) *best = cur;
}

// part of a batch holding id x of a kind whose part offsets are `off` (0 for a
// plain system)
int64_t part_of(const std::vector<int32_t> &off, int32_t x) {
    return off.size() > 2 ? std::upper_bound(off.begin(), off.end(), x) - off.begin() : 0;
}

void apply_move_impl(mm_system *s, int32_t m, int32_t T) {
    if (m < 0 || m >= s->n) fail(MM_EINVAL, "method out of range");
    if (T < 0 || T >= s->c) fail(MM_EINVAL, "class out of range");
    if (s->owner[m] == T) fail(MM_EINVAL, "method already belongs to that class");
    if (part_of(s->part_meth, m) != part_of(s->part_cls, T))
        fail(MM_EINVAL, "the move crosses systems of a batch");
    bool done = false;
    try {
        done = s->layout_valid && s->structure_valid && s->incr_enabled && s->incr.base && move_incremental(s, m, T);
    } catch (...) {
        if (s->owner[m] == T) {  // the host mirror holds the move: rebuild the device copy from it
            s->incr.ops.clear();
            invalidate(s, true);
            s->structure_valid = false;
        }
        throw;
    }
    if (done) {
        invalidate(s, false);  // metrics of the touched segments are recomputed on the next request
        s->entry_moved.push_back(m);
        return;
    }
    s->owner[m] = T;
    invalidate(s, true);
    s->structure_valid = false;
    s->entry_moved.push_back(m);
    HIPCHK(hipMemcpyAsync(s->d_owner.as<int32_t>() + m, &s->owner[m], 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->structure_valid = true;
}

// the scoring scratch a system keeps between calls (ranked suggestions excluded)
#define MM_SCORE_SCRATCH(s)                                                                                     \
    &s->s_prep, &s->s_outk, &s->s_outc, &s->s_outa, &s->s_refcnt, &s->s_candoff, &s->s_cm, &s->s_ct, &s->s_ce,    \
        &s->s_rec, &s->s_gcnt, &s->s_goff, &s->s_gslot, &s->s_glist, &s->s_hval, &s->s_heavy, &s->s_hcand,          \
        &s->s_counts, &s->s_flags, &s->s_kpos, &s->s_tmp, &s->s_kept, &s->s_kept_idx, &s->s_aff_flag, &s->s_aff_val, \
        &s->s_aff_pos, &s->s_aff_cls, &s->s_aff_d, &s->sim_at_off, &s->sim_at_idx, &s->sim_at_cur, &s->sim_deg,     \
        &s->sim_dense, &s->sim_cnt2, &s->sim_ctr, &s->sim_hist, &s->sim_imin, &s->sim_row_pairs,                   \
        &s->sim_row_cands, &s->sim_cand_bits, &s->sim_cand_off, &s->sim_pair_off, &s->sim_pairs

// device bytes of the scoring scratch, ranked suggestions included
int64_t scratch_bytes(const mm_system *s) {
    const DBuf *b[] = {MM_SCORE_SCRATCH(s), &s->s_rank_rec, &s->s_rank_key, &s->s_rank_key2,
                       &s->s_rank_idx, &s->s_rank_idx2, &s->s_rank_tmp};
    int64_t t = 0;
    for (const DBuf *x : b) t += (int64_t)x->bytes;
    return t;
}

// free the scoring scratch (the next scoring call allocates it again); drops
// the cached records, which live in it
void release_scratch(mm_system *s) {
    DBuf *b[] = {MM_SCORE_SCRATCH(s)};
    for (DBuf *x : b) x->release();
    s->cache.valid = false;
    s->sim.at_version = s->sim.stats_version = s->sim.count_version = -1;
}

// Caller classes X of `m` other than S and T, ascending, with the CBO change of
// each when m moves to T (the per-class detail behind a record's caller counts).
void affected_impl(mm_system *s, int32_t m, int32_t T, int32_t *cls, int32_t *dcbo, int64_t cap, int64_t *n) {
    if (!n) fail(MM_EINVAL, "n is NULL");
    if (m < 0 || m >= s->n) fail(MM_EINVAL, "method out of range");
    if (T < 0 || T >= s->c) fail(MM_EINVAL, "class out of range");
    const int32_t S = s->owner[m];
    if (T == S) fail(MM_EINVAL, "destination is the method's own class");
    if (cls && (!dcbo || cap < 0)) fail(MM_EINVAL, "bad output buffers");
    ensure_metrics(s);
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    const int32_t c = s->c;
    s->s_aff_flag.reserve(ctx, cb, (size_t)c * 4);
    s->s_aff_val.reserve(ctx, cb, (size_t)c * 4);
    s->s_aff_pos.reserve(ctx, cb, ((size_t)c + 1) * 8);
    int32_t *flag = s->s_aff_flag.as<int32_t>();
    int32_t *val = s->s_aff_val.as<int32_t>();
    int64_t *pos = s->s_aff_pos.as<int64_t>();
    fill_i32(flag, 0, c, st);
    ScorePlan p;
    memset(&p, 0, sizeof(p));
    p.in = map_view(s->in);
    p.w = map_view(s->w);
    launch_affected_mark(p, m, S, T, map_slots_host(s->in.host_hdr[m]), flag, val, st);
    scan_i32(flag, pos, c, scan_area(s, c), st);
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, pos + c, 8, hipMemcpyDeviceToHost, st));
    check_kernel_errors(s);  // synchronizes
    *n = total;
    if (!cls) return;
    if (cap < total) fail(MM_ERANGE, "output capacity " + std::to_string(cap) + " < " + std::to_string(total));
    if (total == 0) return;
    s->s_aff_cls.reserve(ctx, cb, (size_t)total * 4);
    s->s_aff_d.reserve(ctx, cb, (size_t)total * 4);
    launch_affected_out(flag, val, pos, c, total, s->s_aff_cls.as<int32_t>(), s->s_aff_d.as<int32_t>(), nullptr,
                        st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(cls, s->s_aff_cls.p, (size_t)total * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(dcbo, s->s_aff_d.p, (size_t)total * 4, hipMemcpyDeviceToHost, st));
    check_kernel_errors(s);  // synchronizes
}

// The hierarchy and weights behind WMC, NOC and DIT: validated and copied, then
// NOC and DIT computed on the device (a cycle is found there and refused).
void set_hierarchy_impl(mm_system *s, const int32_t *parent, const int32_t *weight) {
    const int32_t c = s->c, n = s->n;
    if (!parent && c > 0) fail(MM_EINVAL, "parent is NULL");
    const bool batch = s->part_cls.size() > 2;
    for (int32_t C = 0; C < c; ++C) {
        const int32_t p = parent[C];
        if (p < -1 || p >= c) fail(MM_EINVAL, "parent of class " + std::to_string(C) + " out of range");
        if (batch && p >= 0 && part_of(s->part_cls, p) != part_of(s->part_cls, C))
            fail(MM_EINVAL, "class " + std::to_string(C) + " extends a class of another system of the batch");
    }
    if (weight)
        for (int32_t m = 0; m < n; ++m)
            if (weight[m] < 0) fail(MM_EINVAL, "negative weight of method " + std::to_string(m));
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    s->ck_hier = false;
    s->ck_weighted = false;
    if (!s->d_err.p) {
        s->d_err.fit(ctx, cb, 16);
        fill_i32(s->d_err.as<int32_t>(), 0, 4, st);
    }
    if (weight && n > 0) {
        s->ck_weight.fit(ctx, cb, (size_t)n * 4);
        HIPCHK(hipMemcpyAsync(s->ck_weight.p, weight, (size_t)n * 4, hipMemcpyHostToDevice, st));
    } else {
        s->ck_weight.release();
    }
    if (c > 0) {
        DBuf par, anc, anc2, dep2;
        par.alloc(ctx, nullptr, (size_t)c * 4);
        anc.alloc(ctx, nullptr, (size_t)c * 4);
        anc2.alloc(ctx, nullptr, (size_t)c * 4);
        dep2.alloc(ctx, nullptr, (size_t)c * 4);
        s->ck_noc.fit(ctx, cb, (size_t)c * 4);
        s->ck_dit.fit(ctx, cb, (size_t)c * 4);
        HIPCHK(hipMemcpyAsync(par.p, parent, (size_t)c * 4, hipMemcpyHostToDevice, st));
        launch_ck_hierarchy(par.as<int32_t>(), c, s->ck_noc.as<int32_t>(), s->ck_dit.as<int32_t>(),
                            anc.as<int32_t>(), anc2.as<int32_t>(), dep2.as<int32_t>(), s->d_err.as<int>(), st);
        HIPCHK(hipGetLastError());
        check_kernel_errors(s);  // synchronizes; a cycle fails here, leaving no hierarchy set
    }
    s->ck_hier = true;
    s->ck_weighted = weight && n > 0;
}

// WMC, NOC and DIT of every class into `out` (device or host memory)
void compute_ck_impl(mm_system *s, mm_class_ck *out, bool device_out) {
    if (!out && s->c > 0) fail(MM_EINVAL, "out is NULL");
    if (!s->structure_valid) {
        upload_structure(s);
        s->structure_valid = true;
    }
    if (!s->layout_valid) build_layout(s);  // class membership
    if (s->c == 0) return;
    hipStream_t st = s->stream;
    CkOut *dst = reinterpret_cast<CkOut *>(out);
    if (!device_out) {
        s->ck_out.reserve(s->ctx, &s->bytes, (size_t)s->c * sizeof(CkOut));
        dst = s->ck_out.as<CkOut>();
    }
    launch_ck_class(s->view(), s->ck_weighted ? s->ck_weight.as<int32_t>() : nullptr,
                    s->ck_hier ? s->ck_noc.as<int32_t>() : nullptr, s->ck_hier ? s->ck_dit.as<int32_t>() : nullptr,
                    dst, st);
    HIPCHK(hipGetLastError());
    if (!device_out) {
        HIPCHK(hipMemcpyAsync(out, dst, (size_t)s->c * sizeof(CkOut), hipMemcpyDeviceToHost, st));
        check_kernel_errors(s);  // synchronizes
    }
}

// ---------------------------------------------------------------------------
// Working memory of mm_move_affected_noalloc: one array per GPU, which each GPU
// the library runs on holds until the process ends. On the host the array's
// name only stands for the symbol; its address on each device comes from
// hipGetSymbolAddress (noalloc_setup, at context creation) and only that
// address is handed to kernels. Regions: class flags, per-class CBO changes,
// exclusive positions (int64, one more than the classes) and the prefix-sum
// work area.
constexpr size_t na_round(size_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t NA_CLASSES = MM_NOALLOC_MAX_CLASSES;
constexpr size_t NA_FLAG = 0;
constexpr size_t NA_VAL = NA_FLAG + na_round(4 * (size_t)NA_CLASSES);
constexpr size_t NA_POS = NA_VAL + na_round(4 * (size_t)NA_CLASSES);
constexpr size_t NA_SCAN = NA_POS + na_round(8 * ((size_t)NA_CLASSES + 1));
// scan_area_elems(n) = 3 + ceil(n / 2048) words of 8 bytes
constexpr size_t NA_SCAN_WORDS = 3 + ((size_t)NA_CLASSES + 2047) / 2048;
constexpr size_t NA_BYTES = NA_SCAN + na_round(8 * NA_SCAN_WORDS);
static_assert(NA_BYTES == MM_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header's");

static __device__ __align__(256) unsigned char noalloc_scratch[NA_BYTES];

std::mutex noalloc_mu;
std::vector<void *> noalloc_dev;          // per device: the array's address, NULL until set up
std::vector<std::string> noalloc_errors;  // per device: why the address is unknown

// Called with `device` current, once per device (later calls return at once).
void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if ((int)noalloc_dev.size() <= device) {
        noalloc_dev.resize((size_t)device + 1, nullptr);
        noalloc_errors.resize((size_t)device + 1);
    }
    if (noalloc_dev[device] || !noalloc_errors[device].empty()) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        noalloc_errors[device] = std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                 hipGetErrorString(e);
        return;
    }
    noalloc_dev[device] = p;
}

char *noalloc_base(int device) {
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (device < 0 || device >= (int)noalloc_dev.size() || !noalloc_dev[device])
        fail(MM_EHIP, device >= 0 && device < (int)noalloc_errors.size() && !noalloc_errors[device].empty()
                          ? noalloc_errors[device]
                          : "the scratch array of this device was not set up");
    return static_cast<char *>(noalloc_dev[device]);
}

// mm_move_affected's work with device outputs, on the scratch array: no device
// allocation and no wait for the device.
void affected_noalloc_impl(mm_system *s, int32_t m, int32_t T, int32_t *d_cls, int32_t *d_dcbo, int64_t cap,
                           int64_t *d_n) {
    if (!d_n) fail(MM_EINVAL, "d_n is NULL");
    if (cap < 0 || (cap > 0 && (!d_cls || !d_dcbo))) fail(MM_EINVAL, "bad output buffers");
    if (m < 0 || m >= s->n) fail(MM_EINVAL, "method out of range");
    if (T < 0 || T >= s->c) fail(MM_EINVAL, "class out of range");
    const int32_t S = s->owner[m];
    if (T == S) fail(MM_EINVAL, "destination is the method's own class");
    if (s->c > NA_CLASSES)
        fail(MM_EINVAL, "system has " + std::to_string(s->c) + " classes; the allocation-free call takes at most " +
                            std::to_string(NA_CLASSES));
    if (!s->structure_valid || !s->layout_valid || !s->metrics_valid)
        fail(MM_EINVAL, "the system's metrics are not current (call mm_compute_metrics first)");
    char *b = noalloc_base(s->ctx->device);
    int32_t *flag = reinterpret_cast<int32_t *>(b + NA_FLAG);
    int32_t *val = reinterpret_cast<int32_t *>(b + NA_VAL);
    int64_t *pos = reinterpret_cast<int64_t *>(b + NA_POS);
    hipStream_t st = s->stream;
    const int32_t c = s->c;
    fill_i32(flag, 0, c, st);  // the array keeps the previous call's flags
    ScorePlan p;
    memset(&p, 0, sizeof(p));
    p.in = map_view(s->in);
    p.w = map_view(s->w);
    launch_affected_mark(p, m, S, T, map_slots_host(s->in.host_hdr[m]), flag, val, st);
    ScanArea a;
    a.dev = reinterpret_cast<int64_t *>(b + NA_SCAN);
    a.cap_words = scan_area_elems(c);
    if (a.cap_words > (int64_t)NA_SCAN_WORDS) fail(MM_EINTERNAL, "prefix-sum area of the scratch array too small");
    a.need_clear = true;  // cleared by the scan itself: nothing carries over from another call
    a.scans = 0;
    a.err = s->d_err.as<int>();
    scan_i32(flag, pos, c, a, st);
    launch_affected_out(flag, val, pos, c, cap, d_cls, d_dcbo, d_n, st);
    HIPCHK(hipGetLastError());
}

void apply_edit_impl(mm_system *s, const mm_edit_desc *e) {
    if (!e) fail(MM_EINVAL, "edit is NULL");
    const int32_t k = e->k;
    if (k < 0) fail(MM_EINVAL, "negative edit size");
    if (k == 0) return;
    if (!e->method) fail(MM_EINVAL, "edit methods are NULL");
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = e->method[i];
        if (m < 0 || m >= s->n) fail(MM_EINVAL, "edited method out of range at " + std::to_string(i));
        if (e->new_class && (e->new_class[i] < 0 || e->new_class[i] >= s->c))
            fail(MM_EINVAL, "new class out of range at " + std::to_string(i));
    }
    // edited methods in ascending order (a repeat is an error)
    std::vector<int32_t> ord(k);
    for (int32_t i = 0; i < k; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return e->method[a] < e->method[b]; });
    for (int32_t j = 1; j < k; ++j)
        if (e->method[ord[j]] == e->method[ord[j - 1]])
            fail(MM_EINVAL, "method " + std::to_string(e->method[ord[j]]) + " edited twice");
    check_csr("edit acc", e->acc_off, e->acc_idx, k, s->na);
    check_csr("edit call", e->call_off, e->call_idx, k, s->n);
    if (s->part_cls.size() > 2) {
        // a batch: an edited method stays in its part, and so do its new rows
        for (int32_t i = 0; i < k; ++i) {
            const int32_t m = e->method[i];
            const int64_t pm = part_of(s->part_meth, m);
            if (e->new_class && part_of(s->part_cls, e->new_class[i]) != pm)
                fail(MM_EINVAL, "edit " + std::to_string(i) + " moves a method to another system of the batch");
            for (int64_t q = e->acc_off[i]; q < e->acc_off[i + 1]; ++q)
                if (part_of(s->part_attr, e->acc_idx[q]) != pm)
                    fail(MM_EINVAL, "edit " + std::to_string(i) + " accesses an attribute of another system of the batch");
            for (int64_t q = e->call_off[i]; q < e->call_off[i + 1]; ++q)
                if (part_of(s->part_meth, e->call_idx[q]) != pm)
                    fail(MM_EINVAL, "edit " + std::to_string(i) + " calls a method of another system of the batch");
        }
    }
    std::vector<int32_t> ao, ai, co, ci;
    canonical_rows(e->acc_off, e->acc_idx, k, ao, ai);
    canonical_rows(e->call_off, e->call_idx, k, co, ci);
    const int32_t n = s->n;
    int64_t nacc = (int64_t)s->acc_idx.size(), ncall = (int64_t)s->call_idx.size();
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = e->method[i];
        nacc += (ao[i + 1] - ao[i]) - (s->acc_off[m + 1] - s->acc_off[m]);
        ncall += (co[i + 1] - co[i]) - (s->call_off[m + 1] - s->call_off[m]);
    }
    if (nacc > INT32_MAX || ncall > INT32_MAX || nacc + ncall > INT32_MAX)
        fail(MM_EOVERFLOW, "edited system has more than 2^31-1 references");
    // incremental when every metric is current on this layout and the pools
    // hold what the edit adds: marks from the state before the edit
    const EditView view{e, ord, ao, ai, co, ci};
    EditPlan plan;
    const bool inc = s->layout_valid && s->structure_valid && s->incr_enabled && s->incr.base &&
                     edit_plan(s, view, plan);
    std::vector<int64_t> old_len;
    if (inc) {
        edit_mark(s, view);
        old_len.resize((size_t)k);
        for (int32_t i = 0; i < k; ++i) {
            const int32_t m = e->method[i];
            old_len[(size_t)i] = (s->call_off[m + 1] - s->call_off[m]) + (s->acc_off[m + 1] - s->acc_off[m]);
        }
    }
    // new offsets, then the rows: every unchanged span of methods is one copy
    // (its offsets shifted by the change so far)
    std::vector<int32_t> &nao = s->spare_acc_off, &nco = s->spare_call_off, &nai = s->spare_acc_idx,
                         &nci = s->spare_call_idx;
    nao.resize((size_t)n + 1);
    nco.resize((size_t)n + 1);
    nai.resize((size_t)nacc);
    nci.resize((size_t)ncall);
    nao[0] = nco[0] = 0;
    {
        int32_t da = 0, dc = 0, prev = 0;
        const int32_t *sao = s->acc_off.data(), *sco = s->call_off.data();
        int32_t *pao = nao.data(), *pco = nco.data();
        for (int32_t j = 0; j <= k; ++j) {
            const int32_t m = j < k ? e->method[ord[j]] : n;
            for (int32_t x = prev; x < m; ++x) {
                pao[x + 1] = sao[x + 1] + da;
                pco[x + 1] = sco[x + 1] + dc;
            }
            if (j < k) {
                const int32_t i = ord[j];
                pao[m + 1] = pao[m] + (ao[i + 1] - ao[i]);
                pco[m + 1] = pco[m] + (co[i + 1] - co[i]);
                da = pao[m + 1] - sao[m + 1];
                dc = pco[m + 1] - sco[m + 1];
            }
            prev = m + 1;
        }
    }
    // the copies of both row arrays: every unchanged span and every new row is
    // one copy, cut into pieces of at most 1 MiB and shared over a few host
    // threads on large systems
    struct Piece {
        int32_t *dst;
        const int32_t *src;
        int64_t len;
    };
    std::vector<Piece> pieces;
    auto add = [&](int32_t *dst, const int32_t *src, int64_t len) {
        const int64_t step = (int64_t)1 << 18;
        for (int64_t o = 0; o < len; o += step) pieces.push_back({dst + o, src + o, std::min(step, len - o)});
    };
    auto splice = [&](std::vector<int32_t> &dst, const std::vector<int32_t> &noff, const std::vector<int32_t> &src,
                      const std::vector<int32_t> &soff, const std::vector<int32_t> &eo,
                      const std::vector<int32_t> &ei) {
        int32_t prev = 0;
        for (int32_t j = 0; j <= k; ++j) {
            const int32_t m = j < k ? e->method[ord[j]] : n;
            add(dst.data() + noff[prev], src.data() + soff[prev], soff[m] - soff[prev]);
            if (j < k) {
                const int32_t i = ord[j];
                add(dst.data() + noff[m], ei.data() + eo[i], eo[i + 1] - eo[i]);
            }
            prev = m + 1;
        }
    };
    splice(nai, nao, s->acc_idx, s->acc_off, ao, ai);
    splice(nci, nco, s->call_idx, s->call_off, co, ci);
    {
        const int64_t total = nacc + ncall;
        const int threads = total >= ((int64_t)1 << 20) ? 4 : 1;
        std::atomic<size_t> next{0};
        auto work = [&] {
            for (size_t q; (q = next.fetch_add(1)) < pieces.size();)
                memcpy(pieces[q].dst, pieces[q].src, (size_t)pieces[q].len * sizeof(int32_t));
        };
        std::vector<std::future<void>> helpers;
        for (int h = 1; h < threads; ++h) helpers.push_back(std::async(std::launch::async, work));
        work();
        for (auto &f : helpers) f.get();
    }
    s->acc_off.swap(nao);
    s->acc_idx.swap(nai);
    s->call_off.swap(nco);
    s->call_idx.swap(nci);
    if (inc) {
        try {
            edit_apply(s, view, plan, old_len);  // owners, layout patches, device rows and callers
        } catch (...) {
            // the host mirror holds the whole edit (owners are set first); the
            // device copy is rebuilt from it by the next call that needs it
            for (int32_t i = 0; e->new_class && i < k; ++i) s->owner[e->method[i]] = e->new_class[i];
            s->incr.ops.clear();
            invalidate(s, true);
            s->structure_valid = false;
            throw;
        }
        invalidate(s, false);
        return;
    }
    if (e->new_class)
        for (int32_t i = 0; i < k; ++i) s->owner[e->method[i]] = e->new_class[i];
    // the host mirror holds the edit from here on; an upload that fails part
    // way is redone by the next call that needs the device copy
    invalidate(s, true);
    s->structure_valid = false;
    upload_structure(s);
    s->structure_valid = true;
}

// Ranked suggestions (Sec. III-A): score the kind's candidates with its rule
// (kept records only, origins filtered by the threshold), then order the kept
// records by the kind's key with a stable descending sort. The ranked records
// are left in s_kept; returns their number.
int64_t rank_suggestions(mm_system *s, int32_t kind, int32_t threshold) {
    if (kind < MM_SUGGEST_LCOM || kind > MM_SUGGEST_SIMILAR) fail(MM_EINVAL, "bad suggestion kind");
    if (threshold != MM_THRESH_NONE && threshold != MM_THRESH_AVERAGE) fail(MM_EINVAL, "bad suggestion threshold");
    ScoreArgs a{kind == MM_SUGGEST_SIMILAR ? MM_CAND_SIMILAR : MM_CAND_REFERENCED, nullptr, nullptr, 0,
                kind == MM_SUGGEST_CBO ? (uint32_t)MM_CBO : (uint32_t)MM_LCOM_PQ,
                kind == MM_SUGGEST_CBO ? MM_RULE_PAPER_CBO : MM_RULE_PAPER_LCOM, 1};
    a.origin = (kind == MM_SUGGEST_SIMILAR || threshold == MM_THRESH_NONE) ? 0 : (kind == MM_SUGGEST_LCOM ? 1 : 2);
    if (a.origin && s->part_cls.size() > 2) fail(MM_EINVAL, "the class average of a batch would mix systems");
    validate_score_args(s, a);
    score_run(s, a, nullptr, 0);
    const int64_t kept = s->cache.n_out;
    s->cache.valid = false;  // the kept list is consumed below
    if (kept == 0) return 0;
    if (kept > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 suggestions");
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    s->s_rank_rec.reserve(ctx, cb, (size_t)kept * sizeof(MoveRec));
    s->s_rank_key.reserve(ctx, cb, (size_t)kept * 4);
    s->s_rank_key2.reserve(ctx, cb, (size_t)kept * 4);
    s->s_rank_idx.reserve(ctx, cb, (size_t)kept * 4);
    s->s_rank_idx2.reserve(ctx, cb, (size_t)kept * 4);
    s->s_kept.reserve(ctx, cb, (size_t)kept * sizeof(MoveRec));
    launch_compact(compact_plan(s), s->s_rank_rec.as<MoveRec>(), st);
    const int key_kind = kind == MM_SUGGEST_LCOM ? 0 : kind == MM_SUGGEST_CBO ? 1 : 2;
    launch_rank_keys(s->s_rank_rec.as<MoveRec>(), kept, s->d_meth.as<MethodAgg>(), key_kind,
                     s->s_rank_key.as<uint32_t>(), s->s_rank_idx.as<int32_t>(), st);
    size_t tmp_bytes = 0;
    HIPCHK(rank_sort(nullptr, tmp_bytes, nullptr, nullptr, nullptr, nullptr, kept, st));
    s->s_rank_tmp.reserve(ctx, cb, std::max<size_t>(tmp_bytes, 1));
    HIPCHK(rank_sort(s->s_rank_tmp.p, tmp_bytes, s->s_rank_key.as<uint32_t>(), s->s_rank_key2.as<uint32_t>(),
                     s->s_rank_idx.as<int32_t>(), s->s_rank_idx2.as<int32_t>(), kept, st));
    launch_rank_gather(s->s_rank_rec.as<MoveRec>(), s->s_rank_idx2.as<int32_t>(), kept, s->s_kept.as<MoveRec>(), st);
    HIPCHK(hipGetLastError());
    return kept;
}

void suggest_impl(mm_system *s, int32_t kind, int32_t threshold, mm_move_score *out, int64_t cap, int64_t *n) {
    if (!n) fail(MM_EINVAL, "n is NULL");
    if (out && cap < 0) fail(MM_EINVAL, "negative capacity");
    const int64_t kept = rank_suggestions(s, kind, threshold);
    *n = kept;
    if (!out || kept == 0) return;
    if (cap < kept) fail(MM_ERANGE, "output capacity " + std::to_string(cap) + " < " + std::to_string(kept));
    HIPCHK(hipMemcpyAsync(out, s->s_kept.p, (size_t)kept * sizeof(MoveRec), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
}

// The ranked suggestions reduced, in rank order, to moves whose affected
// classes (origin, destination, owners of the method's callers) are disjoint.
void independent_impl(mm_system *s, int32_t kind, int32_t threshold, mm_move_score *out, int64_t cap, int64_t *n) {
    if (!n) fail(MM_EINVAL, "n is NULL");
    if (out && cap < 0) fail(MM_EINVAL, "negative capacity");
    if (s->c > IND_MAX_CLASSES) fail(MM_EOVERFLOW, "conflict-free sets support at most 2^19 classes");
    const int64_t kept = rank_suggestions(s, kind, threshold);
    int64_t taken = 0;
    if (kept > 0) {
        mm_context *ctx = s->ctx;
        s->s_rank_rec.reserve(ctx, &s->bytes, (size_t)kept * sizeof(MoveRec));
        s->s_counts.reserve(ctx, &s->bytes, 32);
        int64_t *d_count = (int64_t *)(s->s_counts.as<char>() + 24);
        launch_independent(s->s_kept.as<MoveRec>(), kept, map_view(s->in), s->c, s->s_rank_rec.as<MoveRec>(),
                           d_count, s->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&taken, d_count, 8, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    *n = taken;
    if (!out || taken == 0) return;
    if (cap < taken) fail(MM_ERANGE, "output capacity " + std::to_string(cap) + " < " + std::to_string(taken));
    HIPCHK(hipMemcpyAsync(out, s->s_rank_rec.p, (size_t)taken * sizeof(MoveRec), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
}

// Greedy plan: apply the best suggestion, rescore, repeat (at most max_moves);
// the applied moves are undone at the end unless keep_applied.
void plan_impl(mm_system *s, int32_t kind, int32_t threshold, int32_t max_moves, int32_t keep_applied,
               mm_move_score *out, int64_t *n) {
    if (!n || (!out && max_moves > 0)) fail(MM_EINVAL, "NULL output");
    if (max_moves < 0) fail(MM_EINVAL, "negative max_moves");
    if (keep_applied != 0 && keep_applied != 1) fail(MM_EINVAL, "keep_applied must be 0 or 1");
    *n = 0;
    int64_t done = 0;
    try {
        for (; done < max_moves; ++done) {
            const int64_t kept = rank_suggestions(s, kind, threshold);
            if (kept == 0) break;
            HIPCHK(hipMemcpyAsync(out + done, s->s_kept.p, sizeof(MoveRec), hipMemcpyDeviceToHost, s->stream));
            HIPCHK(hipStreamSynchronize(s->stream));
            apply_move_impl(s, out[done].method, out[done].dst);
        }
    } catch (...) {
        for (int64_t i = done; i-- > 0;) apply_move_impl(s, out[i].method, out[i].src);
        throw;
    }
    if (!keep_applied)
        for (int64_t i = done; i-- > 0;) apply_move_impl(s, out[i].method, out[i].src);
    *n = done;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *mm_last_error(void) { return g_last_error.c_str(); }

mm_status mm_context_create(int32_t device, void *hip_stream, uint64_t mem_budget_bytes, mm_context **out) {
    return guarded([&] {
        if (!out) fail(MM_EINVAL, "out is NULL");
        int count = 0;
        HIPCHK(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) fail(MM_EINVAL, "bad device " + std::to_string(device));
        HIPCHK(hipSetDevice(device));
        int ncu = 0;
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
        noalloc_setup(device);
        mm_context *ctx = new mm_context();
        ctx->device = device;
        ctx->n_cu = ncu > 0 ? ncu : 256;
        ctx->budget = mem_budget_bytes;
        if (hip_stream) {
            ctx->stream = (hipStream_t)hip_stream;
        } else {
            if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
                delete ctx;
                fail(MM_EHIP, "hipStreamCreate failed");
            }
            ctx->own_stream = true;
        }
        *out = ctx;
    });
}

mm_status mm_context_destroy(mm_context *ctx) {
    return guarded([&] {
        if (!ctx) fail(MM_EINVAL, "context is NULL");
        if (ctx->n_systems) fail(MM_EBUSY, "context still holds systems");
        set_device(ctx);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        for (auto &kv : ctx->aux) {
            for (auto x : kv.second.s) {
                (void)hipStreamSynchronize(x);
                (void)hipStreamDestroy(x);
            }
            for (auto e : kv.second.ev) (void)hipEventDestroy(e);
        }
        ctx->aux.clear();
        for (auto &e : ctx->pool) (void)hipFree(e.second);
        ctx->pool.clear();
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
    });
}

mm_status mm_context_memory(mm_context *ctx, uint64_t *used, uint64_t *budget) {
    return guarded([&] {
        if (!ctx) fail(MM_EINVAL, "context is NULL");
        if (used) *used = ctx->used;
        if (budget) *budget = ctx->budget;
    });
}

mm_status mm_context_set_timing(mm_context *ctx, const char *kernels) {
    return guarded([&] {
        if (!ctx) fail(MM_EINVAL, "context is NULL");
        set_device(ctx);
        ctx->timer.resolve();
        std::string k = kernels ? kernels : "";
        ctx->timer.pattern = (k.empty() || k == "*") ? k : "," + k + ",";
    });
}

mm_status mm_context_timing(mm_context *ctx, mm_kernel_time *out, int32_t cap, int32_t *n, int32_t reset) {
    return guarded([&] {
        if (!ctx || !n) fail(MM_EINVAL, "NULL argument");
        set_device(ctx);
        ctx->timer.resolve();
        int32_t i = 0;
        for (auto &kv : ctx->timer.stats) {
            if (out && i < cap) {
                out[i].name = kv.second.name;
                out[i].launches = kv.second.n;
                out[i].total_ms = kv.second.ms;
            }
            ++i;
        }
        *n = i;
        if (reset) ctx->timer.stats.clear();
    });
}

mm_status mm_context_set_tuning(mm_context *ctx, const mm_tuning *t) {
    return guarded([&] {
        if (!ctx) fail(MM_EINVAL, "context is NULL");
        if (!t) {
            ctx->tuning = mm_tuning{CALLER_LIGHT, HEAVY_CHUNK, 0, 0, 0, 0};
            return;
        }
        if (t->caller_light < 0 || t->heavy_chunk < 1 || t->delta_chunk < 0 || t->delta_grid < 0 ||
            (t->fill_chunk != 0 && (t->fill_chunk < 64 || t->fill_chunk > 2048)) || t->fill_group < 0)
            fail(MM_EINVAL, "bad tuning values");
        ctx->tuning = *t;
    });
}

mm_status mm_context_get_tuning(mm_context *ctx, mm_tuning *t) {
    return guarded([&] {
        if (!ctx || !t) fail(MM_EINVAL, "NULL argument");
        *t = ctx->tuning;
    });
}

mm_status mm_autotune(mm_system *sys, int32_t cand_mode, const int32_t *cand_method, const int32_t *cand_class,
                      int64_t n_cand, uint32_t metric_mask, int32_t rule, int32_t keep_only, int32_t repeats,
                      mm_tuning *best) {
    return guarded([&] {
        checked_sys(sys);
        ScoreArgs a{cand_mode, cand_method, cand_class, n_cand, metric_mask, rule, keep_only};
        autotune_impl(sys, a, repeats, best);
    });
}

mm_status mm_load_batch(mm_context *ctx, const mm_system_desc *descs, int32_t n_sys, mm_system **out) {
    return guarded([&] {
        if (ctx) set_device(ctx);
        load_batch_impl(ctx, descs, n_sys, out);
    });
}

mm_status mm_system_parts(mm_system *sys, int32_t *n_parts, int32_t *class_off, int32_t *method_off,
                          int32_t *attr_off) {
    return guarded([&] {
        checked_sys(sys);
        if (!n_parts) fail(MM_EINVAL, "n_parts is NULL");
        const bool batch = !sys->part_cls.empty();
        *n_parts = batch ? (int32_t)sys->part_cls.size() - 1 : 1;
        const int32_t np = *n_parts;
        for (int32_t i = 0; i <= np; ++i) {
            if (class_off) class_off[i] = batch ? sys->part_cls[i] : (i ? sys->c : 0);
            if (method_off) method_off[i] = batch ? sys->part_meth[i] : (i ? sys->n : 0);
            if (attr_off) attr_off[i] = batch ? sys->part_attr[i] : (i ? sys->na : 0);
        }
    });
}

mm_status mm_load_system(mm_context *ctx, const mm_system_desc *desc, mm_system **out) {
    return guarded([&] { load_impl(ctx, desc, out); });
}

mm_status mm_free_system(mm_system *sys) {
    return guarded([&] {
        if (!sys) fail(MM_EINVAL, "system is NULL");
        set_device(sys->ctx);
        (void)hipStreamSynchronize(sys->stream);
        mm_context *ctx = sys->ctx;
        delete sys;
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        ctx->n_systems--;
    });
}

mm_status mm_system_info_get(mm_system *sys, mm_system_info *out) {
    return guarded([&] {
        checked_sys(sys);
        if (!out) fail(MM_EINVAL, "out is NULL");
        out->n_classes = sys->c;
        out->n_methods = sys->n;
        out->n_attrs = sys->na;
        out->pad = 0;
        out->nnz_acc = (int64_t)sys->acc_idx.size();
        out->nnz_call = (int64_t)sys->call_idx.size();
        out->device_bytes = sys->bytes;
        out->version = sys->version;
    });
}

mm_status mm_compute_metrics(mm_system *sys, mm_class_metrics *out_cls, mm_method_metrics *out_m) {
    return guarded([&] {
        checked_sys(sys);
        ensure_metrics(sys);
        hipStream_t st = sys->stream;
        if (out_cls && sys->c)
            HIPCHK(hipMemcpyAsync(out_cls, sys->d_cls.p, (size_t)sys->c * sizeof(ClassAgg), hipMemcpyDeviceToHost, st));
        if (out_m && sys->n)
            HIPCHK(hipMemcpyAsync(out_m, sys->d_meth.p, (size_t)sys->n * sizeof(MethodAgg), hipMemcpyDeviceToHost, st));
        check_kernel_errors(sys);
    });
}

mm_status mm_compute_metrics_device(mm_system *sys, mm_class_metrics *d_cls, mm_method_metrics *d_m) {
    return guarded([&] {
        checked_sys(sys);
        sys->metrics_valid = false;  // an explicit call always recomputes
        sys->cache.valid = false;
        ensure_metrics(sys, (ClassAgg *)d_cls, (MethodAgg *)d_m);
    });
}

mm_status mm_score_moves(mm_system *sys, int32_t cand_mode, const int32_t *cand_method, const int32_t *cand_class,
                         int64_t n_cand, uint32_t metric_mask, int32_t rule, int32_t keep_only, mm_move_score *out,
                         int64_t out_capacity, int64_t *n_out) {
    return guarded([&] {
        checked_sys(sys);
        ScoreArgs a{cand_mode, cand_method, cand_class, n_cand, metric_mask, rule, keep_only};
        score_impl(sys, a, out, false, out_capacity, n_out);
    });
}

mm_status mm_score_moves_device(mm_system *sys, int32_t cand_mode, const int32_t *cand_method,
                                const int32_t *cand_class, int64_t n_cand, uint32_t metric_mask, int32_t rule,
                                int32_t keep_only, mm_move_score *d_out, int64_t out_capacity, int64_t *n_out) {
    return guarded([&] {
        checked_sys(sys);
        ScoreArgs a{cand_mode, cand_method, cand_class, n_cand, metric_mask, rule, keep_only};
        score_impl(sys, a, d_out, true, out_capacity, n_out);
    });
}

mm_status mm_suggest(mm_system *sys, int32_t kind, int32_t threshold, mm_move_score *out, int64_t capacity,
                     int64_t *n) {
    return guarded([&] {
        checked_sys(sys);
        suggest_impl(sys, kind, threshold, out, capacity, n);
    });
}

mm_status mm_suggest_independent(mm_system *sys, int32_t kind, int32_t threshold, mm_move_score *out,
                                 int64_t capacity, int64_t *n) {
    return guarded([&] {
        checked_sys(sys);
        independent_impl(sys, kind, threshold, out, capacity, n);
    });
}

mm_status mm_plan(mm_system *sys, int32_t kind, int32_t threshold, int32_t max_moves, int32_t keep_applied,
                  mm_move_score *out, int64_t *n) {
    return guarded([&] {
        checked_sys(sys);
        plan_impl(sys, kind, threshold, max_moves, keep_applied, out, n);
    });
}

mm_status mm_move_affected(mm_system *sys, int32_t method, int32_t dst_class, int32_t *cls, int32_t *d_cbo,
                           int64_t capacity, int64_t *n) {
    return guarded([&] {
        checked_sys(sys);
        affected_impl(sys, method, dst_class, cls, d_cbo, capacity, n);
    });
}

mm_status mm_set_hierarchy(mm_system *sys, const int32_t *parent, const int32_t *weight) {
    return guarded([&] {
        checked_sys(sys);
        set_hierarchy_impl(sys, parent, weight);
    });
}

mm_status mm_compute_ck(mm_system *sys, mm_class_ck *out) {
    return guarded([&] {
        checked_sys(sys);
        compute_ck_impl(sys, out, false);
    });
}

mm_status mm_compute_ck_device(mm_system *sys, mm_class_ck *d_out) {
    return guarded([&] {
        checked_sys(sys);
        compute_ck_impl(sys, d_out, true);
    });
}

mm_status mm_move_affected_noalloc(mm_system *sys, int32_t method, int32_t dst_class, int32_t *d_cls,
                                   int32_t *d_cbo, int64_t capacity, int64_t *d_n) {
    return guarded([&] {
        checked_sys(sys);
        affected_noalloc_impl(sys, method, dst_class, d_cls, d_cbo, capacity, d_n);
    });
}

mm_status mm_similarity(mm_system *sys, int32_t threshold, mm_sim_stats *out) {
    return guarded([&] {
        checked_sys(sys);
        if (!out) fail(MM_EINVAL, "out is NULL");
        check_threshold(threshold);
        sys->sim.stats_version = sys->sim.count_version = -1;  // an explicit call always recomputes,
        sys->cache.valid = false;                              // and so does the next SIMILAR scoring
        sim_count(sys, threshold);
        const int64_t n = sys->n;
        out->n_pairs = n >= 2 ? n * (n - 1) / 2 : 0;
        out->n_nonzero = (int64_t)sys->sim.nnz;
        out->n_high = sys->sim.n_kept;
        out->n_candidates = sys->sim.n_cands;
        out->threshold = threshold;
        out->max_union = sys->sim.umax;
        out->average = sys->sim.average;
    });
}

mm_status mm_similarity_pairs(mm_system *sys, int32_t threshold, mm_sim_pair *out, int64_t capacity,
                              int64_t *n) {
    return guarded([&] {
        checked_sys(sys);
        sim_pairs(sys, threshold, out, capacity, n);
    });
}

mm_status mm_set_similarity_threshold(mm_system *sys, int32_t threshold) {
    return guarded([&] {
        checked_sys(sys);
        check_threshold(threshold);
        sys->sim_threshold = threshold;
    });
}

mm_status mm_system_set_incremental(mm_system *sys, int32_t enabled) {
    return guarded([&] {
        checked_sys(sys);
        if (enabled != 0 && enabled != 1) fail(MM_EINVAL, "enabled must be 0 or 1");
        sys->incr_enabled = enabled != 0;
    });
}

mm_status mm_apply_move(mm_system *sys, int32_t method, int32_t dst_class) {
    return guarded([&] {
        checked_sys(sys);
        apply_move_impl(sys, method, dst_class);
    });
}

mm_status mm_apply_edit(mm_system *sys, const mm_edit_desc *edit) {
    return guarded([&] {
        checked_sys(sys);
        apply_edit_impl(sys, edit);
    });
}

}  // extern "C"

#include "mm_server_impl.h"

// k_metrics.hip -- gfx950 kernels computing the per-method and per-class
// metrics of Sec. II: fan-in / fan-out (Sec. II-A), CBO, both LCOM forms and RFC
// (Sec. II-B).
//
// Pipeline (two chains joined by events, see launch_compute_metrics):
//   k_entry_classes   once per change of the rows or the owners: the class of
//                     every call, access and caller entry, read beside the entry
//                     by the kernels below
//   k_method_basic    one lane per method: fan-in, fan-out, own-attribute uses and
//                     the bit mask of the own attributes it uses
//   k_map_tab_wc      W: per class, the classes it uses, with reference counts,
//                     grouped in an LDS hash table that is then copied out as
//                     the class's table (CBO = number of keys); CNT: per class,
//                     the methods its methods call, with the number of its
//                     methods calling each (RFC counts the keys owned by other
//                     classes). A wave per class builds both tables when they fit
//                     one LDS region (else one each); k_map_tab_sep does the same
//                     per segment for the recompute after moves.
//   k_map_tab_mid     the same for segments of MAP_CAP..MID_CAP references: a
//                     block of four waves per table of up to MID_HMAX slots
//   k_in_runs, k_map_tab_in    callers of each method grouped by their class
//   k_big_stage,      larger segments (W and CNT of more than MID_CAP
//   k_big_build       references, caller maps of more than MAP_CAP): fill items
//                     count their keys in LDS and stage the distinct pairs by
//                     table partition; a block per partition then builds it in
//                     LDS and copies it out whole (no global atomic on a table)
//   k_coaccess(_lds)  INT8 MFMA: G_C = B_C B_C^T over the class's own attributes;
//                     per method the number of other methods with G > 0 (ballot +
//                     popcount of the accumulator signs)
//   k_finalize        16 lanes (or a wave, for classes of more than FIN_SMALL
//                     members) per class: n, a, CBO, RFC, P, Q, LCOM_HS
#include <algorithm>

#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

// fan-in, fan-out, own-attribute uses and the own-attribute mask of method m;
// rnz (filled by the co-access kernels) is zeroed, or kept when keep_rnz
__device__ __forceinline__ void method_basic(const DevSys &d, int m, bool keep_rnz, MethodAgg *__restrict__ out,
                                             uint64_t *__restrict__ own_mask) {
    int S = d.owner[m];
    int u = 0;
    uint64_t bits = 0;
    for (int e = d.acc_off[m]; e < d.acc_off[m + 1]; ++e) {
        const int li = d.acc_rank[e];  // rank and class of the entry's attribute, read together
        if (d.acc_cls[e] == S) {
            ++u;
            if (li < 64) bits |= 1ull << li;
        }
    }
    MethodAgg r;
    r.fan_in = d.rc_off[m + 1] - d.rc_off[m];
    r.fan_out = d.call_off[m + 1] - d.call_off[m];
    r.u_own = u;
    r.rnz = keep_rnz ? out[m].rnz : 0;
    out[m] = r;
    own_mask[m] = bits;
}

__global__ __launch_bounds__(256) void k_method_basic(DevSys d, MethodAgg *__restrict__ out,
                                                     uint64_t *__restrict__ own_mask) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    method_basic(d, m, false, out, own_mask);
}

// The methods list[0 .. n): the first n_zero get rnz = 0 (their class's co-access
// is recomputed, or the class has no attributes), the others keep theirs.
__global__ __launch_bounds__(256) void k_method_basic_list(DevSys d, const int32_t *__restrict__ list, int n,
                                                          int n_zero, MethodAgg *__restrict__ out,
                                                          uint64_t *__restrict__ own_mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    method_basic(d, list[i], i >= n_zero, out, own_mask);
}

enum { KIND_W = 0, KIND_CNT = 1, KIND_IN = 2 };

// count one more `key` in an LDS table of H slots; true when this call stored the key
__device__ __forceinline__ bool lds_insert(int32_t *tk, int32_t *tv, int H, int32_t key, int *err) {
    uint32_t h = slot_hash(key) & (uint32_t)(H - 1);
    for (int probe = 0; probe < H; ++probe) {
        int32_t prev = atomicCAS(&tk[h], EMPTY_KEY, key);
        if (prev == EMPTY_KEY || prev == key) {
            atomicAdd(&tv[h], 1);
            return prev == EMPTY_KEY;
        }
        h = (h + 1) & (uint32_t)(H - 1);
    }
    atomicOr(err, ERR_MAP_OVERFLOW);
    return false;
}

// The grouping key of element e of a member batch (calls first, then
// accesses): the member whose row holds it, found by binary search over the
// batch's starts, then the callee (CNT, with its class in kcls, loaded beside
// it) or the class of its call or access entry (W, one load from the entry
// classes).
template <int KIND>
__device__ __forceinline__ int32_t batch_key(const DevSys &d, const int32_t *s_start, const int32_t *s_cb,
                                             const int32_t *s_ab, const int32_t *s_nc, int e, int32_t &kcls) {
    int lo = 0, hi = WAVE - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int pos = e - s_start[lo];
    if (KIND == KIND_CNT) {
        kcls = d.call_cls[s_cb[lo] + pos];
        return d.call_idx[s_cb[lo] + pos];
    }
    kcls = pos < s_nc[lo] ? d.call_cls[s_cb[lo] + pos] : d.acc_cls[s_ab[lo] + pos - s_nc[lo]];
    return kcls;
}

// The same key through the rows and the owner / attribute-class arrays: the
// fill items of the large segments read long runs of rows whose gathers stay
// in cache, where streaming the entry classes beside them costs more.
template <int KIND>
__device__ __forceinline__ int32_t batch_key_gather(const DevSys &d, const int32_t *s_start, const int32_t *s_cb,
                                                    const int32_t *s_ab, const int32_t *s_nc, int e) {
    int lo = 0, hi = WAVE - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int pos = e - s_start[lo];
    if (pos < s_nc[lo] || KIND == KIND_CNT) {
        const int32_t x = d.call_idx[s_cb[lo] + pos];
        return KIND == KIND_CNT ? x : d.owner[x];
    }
    return d.acls[d.acc_idx[s_ab[lo] + pos - s_nc[lo]]];
}

// The class of every call, access and caller entry (the gathers the map and
// scoring kernels would otherwise make per entry): one lane per entry.
__global__ __launch_bounds__(256) void k_entry_classes(DevSys d, int64_t ncall, int64_t nacc,
                                                       int32_t *__restrict__ call_cls, int32_t *__restrict__ acc_cls,
                                                       int32_t *__restrict__ rc_cls, int32_t *__restrict__ acc_rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncall) {
        const int32_t x = d.call_idx[i], y = d.rc_idx[i];
        call_cls[i] = d.owner[x];
        rc_cls[i] = d.owner[y];
    } else if (i - ncall < nacc) {
        const int32_t a = d.acc_idx[i - ncall];
        acc_cls[i - ncall] = d.acls[a];
        acc_rank[i - ncall] = d.alocal[a];
    }
}


// Orders the LDS accesses of one wave (a wave's LDS operations complete in
// issue order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A batch of up to 64 members of a class, staged by one wave: where each
// member's entries start in the batch, its call and access rows and its
// number of calls.
struct MapStage {
    int32_t start[WAVE], cb[WAVE], ab[WAVE], nc[WAVE];
};

// the segment lists of one k_map_tab_sep launch
struct MapTabWork {
    const int32_t *w_list, *c_list;
    int n_w, n_w_large, n_c, n_c_large;
};

// LDS of a two-wave block: a table region and a staging area per wave; a
// segment of more than MAP_HSMALL slots takes both regions.
struct MapTabLds {
    int32_t tk[2 * MAP_HSMALL];
    int32_t tv[2 * MAP_HSMALL];
    MapStage st[2];
};
static_assert(MAP_HMAX <= 2 * MAP_HSMALL, "a large table fits in the block's two regions");

// Group the keys of one segment (class C's member rows) in the calling wave's
// LDS table (tk, tv) of the segment's own size, then copy it out slot for slot.
// The segment's key count and, for CNT, the number of keys owned by other
// classes go to its header.
template <int KIND>
__device__ __forceinline__ void map_tab_wave(const DevSys &d, int seg, const MapOut &mo, int *err, int32_t *tk,
                                             int32_t *tv, int hmax, MapStage &st) {
    static_assert(KIND == KIND_W || KIND == KIND_CNT, "class maps only");
    const int lane = threadIdx.x & (WAVE - 1);
    const MapHdr g = mo.hdr[seg];
    const int H = g.cap;  // a power of two
    if (H > hmax) {       // the layout never builds one; refuse rather than overrun LDS
        if (lane == 0) atomicOr(err, ERR_MAP_OVERFLOW);
        return;
    }
    for (int s = lane; s < H; s += WAVE) {
        tk[s] = EMPTY_KEY;
        tv[s] = 0;
    }
    const int C = seg;
    const int mb = d.mem_off[C], me = d.mem_end[C];
    int foreign = 0;  // CNT: keys owned by another class
    for (int base = mb; base < me; base += WAVE) {
        const int y = base + lane < me ? d.mem_idx[base + lane] : -1;
        int nc = 0, len = 0, cb = 0, ab = 0;
        if (y >= 0) {
            cb = d.call_off[y];
            ab = d.acc_off[y];
            nc = d.call_off[y + 1] - cb;
            len = (KIND == KIND_CNT) ? nc : nc + d.acc_off[y + 1] - ab;
        }
        const int incl = wave_incl_scan(len);
        const int total = __shfl(incl, WAVE - 1, WAVE);
        st.start[lane] = incl - len;
        st.cb[lane] = cb;
        st.ab[lane] = ab;
        st.nc[lane] = nc;
        wave_lds_sync();
        for (int e0 = lane; e0 < total; e0 += 4 * WAVE) {  // four entries per lane in flight
            int32_t key[4], kc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * WAVE;
                key[u] = e < total ? batch_key<KIND>(d, st.start, st.cb, st.ab, st.nc, e, kc[u]) : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (key[u] < 0 || (KIND == KIND_W && key[u] == C)) continue;
                // CNT: a callee of another class counts once, when first stored
                if (lds_insert(tk, tv, H, key[u], err) && KIND == KIND_CNT && kc[u] != C) ++foreign;
            }
        }
        wave_lds_sync();  // the batch is read before the next one is staged
    }

    int32_t *keys = mo.keys + g.base;
    int32_t *vals = mo.vals + g.base;
    int K = 0;
    for (int s0 = lane; s0 < H; s0 += 4 * WAVE) {  // four slots per lane
        int32_t key[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * WAVE;
            key[u] = s < H ? tk[s] : EMPTY_KEY;
            v[u] = s < H ? tv[s] : 0;
            K += key[u] != EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * WAVE;
            if (s < H) {
                keys[s] = key[u];
                vals[s] = v[u];
            }
        }
    }
    K = wave_sum(K);
    if (KIND == KIND_CNT) foreign = wave_sum(foreign);
    if (lane == 0) {
        mo.hdr[seg].len = K;
        if (KIND != KIND_W) mo.foreign[seg] = foreign;
    }
}

// The W and CNT tables in one launch of two-wave blocks, each segment on its own
// (the recompute after moves, whose lists name W and CNT segments apart). Each list holds its
// segments of more than MAP_HSMALL slots first (n_*_large of them), then the
// others. Blocks, in order: one per large W segment, one per large CNT segment
// (wave 0 groups it in both LDS regions, wave 1 leaves at once), then the small
// W and the small CNT segments two to a block (a wave and a region each). The
// two maps do not depend on each other. Waves never wait for each other.
__global__ __launch_bounds__(128) void k_map_tab_sep(DevSys d, MapTabWork wk, MapOut w, MapOut cnt, int *err) {
    __shared__ MapTabLds L;
    const int wv = threadIdx.x >> 6;
    int b = blockIdx.x;
    if (b < wk.n_w_large + wk.n_c_large) {
        if (wv != 0) return;
        if (b < wk.n_w_large)
            map_tab_wave<KIND_W>(d, wk.w_list[b], w, err, L.tk, L.tv, 2 * MAP_HSMALL, L.st[0]);
        else
            map_tab_wave<KIND_CNT>(d, wk.c_list[b - wk.n_w_large], cnt, err, L.tk, L.tv, 2 * MAP_HSMALL, L.st[0]);
        return;
    }
    b -= wk.n_w_large + wk.n_c_large;
    int32_t *tk = L.tk + wv * MAP_HSMALL, *tv = L.tv + wv * MAP_HSMALL;
    const int qw = (wk.n_w - wk.n_w_large + 1) >> 1;
    if (b < qw) {
        const int i = wk.n_w_large + 2 * b + wv;
        if (i < wk.n_w) map_tab_wave<KIND_W>(d, wk.w_list[i], w, err, tk, tv, MAP_HSMALL, L.st[wv]);
        return;
    }
    b -= qw;
    const int i = wk.n_c_large + 2 * b + wv;
    if (i < wk.n_c) map_tab_wave<KIND_CNT>(d, wk.c_list[i], cnt, err, tk, tv, MAP_HSMALL, L.st[wv]);
}

// The W and CNT tables of one class in one wave: a batch of members is staged
// once; each call entry gives a W key (the callee's class) and a CNT key (the
// callee), each access a W key. The two tables sit side by side in the wave's
// LDS region (W, then CNT), each of its segment's own size, and are copied out
// slot for slot with their key counts (and, for CNT, the keys owned by other
// classes). A class whose W table groups in LDS has its CNT table there too:
// its calls are a part of its references.
__device__ __forceinline__ void map_tab_wave_wc(const DevSys &d, int C, const MapOut &w, const MapOut &cnt, int *err,
                                                int32_t *tk, int32_t *tv, int hmax, MapStage &st) {
    const int lane = threadIdx.x & (WAVE - 1);
    const MapHdr gw = w.hdr[C], gc = cnt.hdr[C];
    const int Hw = gw.cap;                               // a power of two
    const int Hc = gc.kind == MAP_TABLE ? gc.cap : 0;    // no calls: no CNT table
    if (Hw + Hc > hmax) {  // the layout never builds one; refuse rather than overrun LDS
        if (lane == 0) atomicOr(err, ERR_MAP_OVERFLOW);
        return;
    }
    for (int s = lane; s < Hw + Hc; s += WAVE) {
        tk[s] = EMPTY_KEY;
        tv[s] = 0;
    }
    int32_t *ctk = tk + Hw, *ctv = tv + Hw;
    const int mb = d.mem_off[C], me = d.mem_end[C];
    int foreign = 0;  // CNT keys owned by another class
    for (int base = mb; base < me; base += WAVE) {
        const int y = base + lane < me ? d.mem_idx[base + lane] : -1;
        int nc = 0, len = 0, cb = 0, ab = 0;
        if (y >= 0) {
            cb = d.call_off[y];
            ab = d.acc_off[y];
            nc = d.call_off[y + 1] - cb;
            len = nc + d.acc_off[y + 1] - ab;
        }
        const int incl = wave_incl_scan(len);
        const int total = __shfl(incl, WAVE - 1, WAVE);
        st.start[lane] = incl - len;
        st.cb[lane] = cb;
        st.ab[lane] = ab;
        st.nc[lane] = nc;
        wave_lds_sync();
        for (int e0 = lane; e0 < total; e0 += 4 * WAVE) {  // four entries per lane in flight
            int32_t wkey[4], ckey[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * WAVE;
                wkey[u] = ckey[u] = -1;
                if (e < total) {
                    int lo = 0, hi = WAVE - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (st.start[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    const int pos = e - st.start[lo];
                    if (pos < st.nc[lo]) {  // a call: callee and its class, read together
                        ckey[u] = d.call_idx[st.cb[lo] + pos];
                        wkey[u] = d.call_cls[st.cb[lo] + pos];
                    } else {
                        wkey[u] = d.acc_cls[st.ab[lo] + pos - st.nc[lo]];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (wkey[u] >= 0 && wkey[u] != C) lds_insert(tk, tv, Hw, wkey[u], err);
                // a callee of another class counts once, when first stored
                if (ckey[u] >= 0 && lds_insert(ctk, ctv, Hc, ckey[u], err) && wkey[u] != C) ++foreign;
            }
        }
        wave_lds_sync();  // the batch is read before the next one is staged
    }
    // W copy-out, then CNT
    int Kw = 0, Kc = 0;
    for (int s0 = lane; s0 < Hw; s0 += 4 * WAVE) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * WAVE;
            if (s < Hw) {
                const int32_t key = tk[s];
                Kw += key != EMPTY_KEY;
                w.keys[gw.base + s] = key;
                w.vals[gw.base + s] = tv[s];
            }
        }
    }
    for (int s0 = lane; s0 < Hc; s0 += 4 * WAVE) {  // four slots per lane
        int32_t key[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * WAVE;
            key[u] = s < Hc ? ctk[s] : EMPTY_KEY;
            v[u] = s < Hc ? ctv[s] : 0;
            Kc += key[u] != EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * WAVE;
            if (s < Hc) {
                cnt.keys[gc.base + s] = key[u];
                cnt.vals[gc.base + s] = v[u];
            }
        }
    }
    Kw = wave_sum(Kw);
    Kc = wave_sum(Kc);
    foreign = wave_sum(foreign);
    if (lane == 0) {
        w.hdr[C].len = Kw;
        if (Hc) {
            cnt.hdr[C].len = Kc;
            cnt.foreign[C] = foreign;
        }
    }
}

// The W and CNT tables of the full recompute in one launch of two-wave blocks
// (the layout of k_map_tab_sep: a region of MAP_HSMALL slots and a staging
// area per wave). Work items: a class's W and CNT tables together (when they
// fit MAP_HMAX slots), or one of them alone (item = class * 4 + what: 0 both,
// 1 W, 2 CNT). Items of more than MAP_HSMALL slots come first, one per block in
// both regions (the second wave leaves at once); the others two per block.
// Waves never wait for each other.
__global__ __launch_bounds__(128) void k_map_tab_wc(DevSys d, MapWcWork wk, MapOut w, MapOut cnt, int *err) {
    __shared__ MapTabLds L;
    const int wv = threadIdx.x >> 6;
    int b = blockIdx.x;
    int item;
    int32_t *tk, *tv;
    int hmax;
    if (b < wk.n_large) {
        if (wv != 0) return;
        item = wk.list[b];
        tk = L.tk;
        tv = L.tv;
        hmax = 2 * MAP_HSMALL;
    } else {
        const int i = 2 * (b - wk.n_large) + wv;
        if (i >= wk.n_small) return;  // a whole wave leaves together
        item = wk.list[wk.n_large + i];
        tk = L.tk + wv * MAP_HSMALL;
        tv = L.tv + wv * MAP_HSMALL;
        hmax = MAP_HSMALL;
    }
    const int C = item >> 2, what = item & 3;
    if (what == 0) map_tab_wave_wc(d, C, w, cnt, err, tk, tv, hmax, L.st[wv]);
    else if (what == 1) map_tab_wave<KIND_W>(d, C, w, err, tk, tv, hmax, L.st[wv]);
    else map_tab_wave<KIND_CNT>(d, C, cnt, err, tk, tv, hmax, L.st[wv]);
}

// Group the keys of one segment (class C's member rows) in a block's LDS table
// of the segment's own size (at most MID_HMAX slots), then copy it out slot for
// slot, with its key count and, for CNT, the keys owned by other classes in
// its header. Each of the four waves stages its own batches of 64 members; a
// wave's batch is read before it stages the next, and the table is complete
// after the block's barrier.
struct MapMidLds {
    int32_t tk[MID_HMAX];
    int32_t tv[MID_HMAX];
    MapStage st[4];
    int s_k, s_for;
};

template <int KIND>
__device__ __forceinline__ void map_tab_block(const DevSys &d, int seg, const MapOut &mo, int *err, MapMidLds &L) {
    static_assert(KIND == KIND_W || KIND == KIND_CNT, "class maps only");
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & (WAVE - 1), wv = tid >> 6;
    const MapHdr g = mo.hdr[seg];
    const int H = g.cap;  // a power of two
    if (H > MID_HMAX) {   // the layout never builds one; refuse rather than overrun LDS
        if (tid == 0) atomicOr(err, ERR_MAP_OVERFLOW);
        return;
    }
    for (int s = tid; s < H; s += nth) {
        L.tk[s] = EMPTY_KEY;
        L.tv[s] = 0;
    }
    if (tid == 0) {
        L.s_k = 0;
        L.s_for = 0;
    }
    __syncthreads();
    const int C = seg;
    const int mb = d.mem_off[C], me = d.mem_end[C];
    MapStage &st = L.st[wv];
    int foreign = 0;  // CNT: keys owned by another class
    for (int base = mb + wv * WAVE; base < me; base += 4 * WAVE) {  // the waves take batches in turn
        const int y = base + lane < me ? d.mem_idx[base + lane] : -1;
        int nc = 0, len = 0, cb = 0, ab = 0;
        if (y >= 0) {
            cb = d.call_off[y];
            ab = d.acc_off[y];
            nc = d.call_off[y + 1] - cb;
            len = (KIND == KIND_CNT) ? nc : nc + d.acc_off[y + 1] - ab;
        }
        const int incl = wave_incl_scan(len);
        const int total = __shfl(incl, WAVE - 1, WAVE);
        st.start[lane] = incl - len;
        st.cb[lane] = cb;
        st.ab[lane] = ab;
        st.nc[lane] = nc;
        wave_lds_sync();
        for (int e0 = lane; e0 < total; e0 += 4 * WAVE) {  // four entries per lane in flight
            int32_t key[4], kc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * WAVE;
                key[u] = e < total ? batch_key<KIND>(d, st.start, st.cb, st.ab, st.nc, e, kc[u]) : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (key[u] < 0 || (KIND == KIND_W && key[u] == C)) continue;
                // CNT: a callee of another class counts once, when first stored
                if (lds_insert(L.tk, L.tv, H, key[u], err) && KIND == KIND_CNT && kc[u] != C) ++foreign;
            }
        }
        wave_lds_sync();  // the batch is read before the wave stages its next one
    }
    __syncthreads();
    int32_t *keys = mo.keys + g.base;
    int32_t *vals = mo.vals + g.base;
    int K = 0;
    for (int s0 = tid; s0 < H; s0 += 4 * nth) {  // four slots per thread
        int32_t key[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * nth;
            key[u] = s < H ? L.tk[s] : EMPTY_KEY;
            v[u] = s < H ? L.tv[s] : 0;
            K += key[u] != EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * nth;
            if (s < H) {
                keys[s] = key[u];
                vals[s] = v[u];
            }
        }
    }
    K = wave_sum(K);
    if (KIND == KIND_CNT) foreign = wave_sum(foreign);
    if (lane == 0) {
        atomicAdd(&L.s_k, K);
        if (KIND == KIND_CNT) atomicAdd(&L.s_for, foreign);
    }
    __syncthreads();
    if (tid == 0) {
        mo.hdr[seg].len = L.s_k;
        if (KIND != KIND_W) mo.foreign[seg] = L.s_for;
    }
}

// The W and CNT tables of MAP_CAP..MID_CAP references in one launch: a block
// of four waves per table, W segments first.
__global__ __launch_bounds__(256) void k_map_tab_mid(DevSys d, const int32_t *__restrict__ w_list, int n_w,
                                                     const int32_t *__restrict__ c_list, int n_c, MapOut w,
                                                     MapOut cnt, int *err) {
    __shared__ MapMidLds L;
    const int b = blockIdx.x;
    if (b < n_w)
        map_tab_block<KIND_W>(d, w_list[b], w, err, L);
    else if (b - n_w < n_c)
        map_tab_block<KIND_CNT>(d, c_list[b - n_w], cnt, err, L);
}

// Caller tables of middle length (IN_SMALL < callers <= MAP_CAP): one block of
// four waves per method, sharing one LDS hash table of the callers' classes;
// the table is then copied out slot for slot with the loss flag of each class
// X (all of X's references to S are calls to this method: w_X(S) equals the
// count), four slots per thread with their lookups overlapped.
__global__ __launch_bounds__(256) void k_map_tab_in(DevSys d, const int32_t *__restrict__ list, MapOut mo,
                                                    MapView wv, int *err) {
    __shared__ int32_t tk[MAP_HMAX];
    __shared__ int32_t tv[MAP_HMAX];
    __shared__ int s_k, s_own;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int m = list[blockIdx.x];
    const MapHdr g = mo.hdr[m];
    const int H = g.cap;  // a power of two
    if (H > MAP_HMAX) {   // the layout never builds one; refuse rather than overrun LDS
        if (tid == 0) atomicOr(err, ERR_MAP_OVERFLOW);
        return;
    }
    for (int s = tid; s < H; s += nth) {
        tk[s] = EMPTY_KEY;
        tv[s] = 0;
    }
    if (tid == 0) {
        s_k = 0;
        s_own = 0;
    }
    __syncthreads();
    const int b = d.rc_off[m], e = d.rc_off[m + 1];
    for (int i0 = b + tid; i0 < e; i0 += 2 * nth) {  // two callers per thread in flight
        int32_t y[2], cy[2], key[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {  // caller and its class loaded together
            const bool in = i0 + u * nth < e;
            y[u] = in ? d.rc_idx[i0 + u * nth] : m;
            cy[u] = in ? d.rc_cls[i0 + u * nth] : -1;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) key[u] = y[u] != m ? cy[u] : -1;
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (key[u] >= 0) lds_insert(tk, tv, H, key[u], err);
    }
    __syncthreads();
    int32_t *keys = mo.keys + g.base;
    int32_t *vals = mo.vals + g.base;
    const int S = d.owner[m];
    int K = 0, own = 0;
    for (int s0 = tid; s0 < H; s0 += 4 * nth) {
        int32_t key[4], v[4];
        MapHdr h[4];
        uint32_t sl[4];
        int32_t k0[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * nth;
            key[u] = s < H ? tk[s] : EMPTY_KEY;
            v[u] = s < H ? tv[s] : 0;
            K += key[u] != EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) h[u] = key[u] != EMPTY_KEY ? wv.hdr[key[u]] : MapHdr{0, 0, MAP_EMPTY, 0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sl[u] = slot_hash(S) & ((uint32_t)h[u].cap - 1u);
            k0[u] = h[u].kind == MAP_TABLE ? wv.keys[h[u].base + sl[u]] : EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (key[u] == S) own = v[u];
            if (key[u] != EMPTY_KEY && tab_get_from(h[u], wv.keys, wv.vals, S, sl[u], k0[u]) == v[u])
                v[u] |= (int32_t)0x80000000;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * nth;
            if (s < H) {
                keys[s] = key[u];
                vals[s] = v[u];
            }
        }
    }
    K = wave_sum(K);
    own = wave_sum(own);  // one thread at most holds the own class
    if ((tid & (WAVE - 1)) == 0) {
        atomicAdd(&s_k, K);
        atomicAdd(&s_own, own);
    }
    __syncthreads();
    if (tid == 0) {
        mo.hdr[m].len = s_k;
        mo.foreign[m] = s_own;
    }
}

// Callers of a method grouped by class, for caller rows of 1..IN_SMALL entries.
// A segment of SEG lanes (SEG >= the row length) takes one method: each lane
// loads one caller and its class, a bitonic network of lane shuffles sorts the
// classes, and ballots over the sorted keys give the groups: a lane whose key
// differs from its left neighbour starts a group, its rank among the starts is
// the group's place in the sorted run, the next start bounds its count. Group
// leaders then set the loss flag: all of X's uses of S come from this method
// (w_X(S) equals the count). Self calls are not callers.
template <int SEG>
__device__ __forceinline__ void in_run_segment(const DevSys &d, const MapOut &mo, const MapView &wv,
                                               const int32_t *__restrict__ list, int n_list, int blk) {
    static_assert(SEG >= 2 && SEG <= WAVE && (SEG & (SEG - 1)) == 0, "segment of 2..64 lanes");
    const int lane = threadIdx.x & (WAVE - 1);
    const int j = threadIdx.x & (SEG - 1);
    const int seg = blk * (int)(blockDim.x / SEG) + (int)threadIdx.x / SEG;
    const bool act = seg < n_list;
    const int m = act ? list[seg] : -1;
    int b = 0, k = 0, S = -1, base = 0;
    if (act) {
        b = d.rc_off[m];
        k = d.rc_off[m + 1] - b;
        S = d.owner[m];
        base = mo.hdr[m].base;
    }
    int32_t key = INT32_MAX;  // empty lanes sort last
    if (j < k) {
        const int y = d.rc_idx[b + j];
        const int cy = d.rc_cls[b + j];
        if (y != m) key = cy;
    }
#pragma unroll
    for (int kk = 2; kk <= SEG; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const int32_t p = __shfl_xor(key, jj, WAVE);
            const bool take_min = ((j & jj) == 0) == ((j & kk) == 0);
            key = take_min ? min(key, p) : max(key, p);
        }
    }
    const int32_t left = __shfl_up(key, 1, WAVE);
    const bool valid = key != INT32_MAX;
    const bool start = valid && (j == 0 || left != key);
    const int sbase = lane & ~(SEG - 1);
    const uint64_t segmask = (SEG == WAVE ? ~0ull : ((1ull << SEG) - 1ull)) << sbase;
    const uint64_t st = __ballot(start) & segmask;
    const uint64_t vm = __ballot(valid) & segmask;
    const uint64_t above = st & ~((2ull << lane) - 1ull);  // starts right of this lane
    const int end = above ? __ffsll((long long)above) - 1 : sbase + __popcll(vm);
    const int cnt = end - lane;
    const uint64_t own_bits = __ballot(start && key == S) & segmask;
    const int own_src = own_bits ? __ffsll((long long)own_bits) - 1 : lane;
    const int own_cnt = __shfl(cnt, own_src, WAVE);
    if (start) {
        const int r = __popcll(st & ((1ull << lane) - 1ull));
        const MapHdr h = wv.hdr[key];
        const uint32_t sl = slot_hash(S) & ((uint32_t)h.cap - 1u);
        const int32_t k0 = h.kind == MAP_TABLE ? wv.keys[h.base + sl] : EMPTY_KEY;
        int32_t v = cnt;
        if (tab_get_from(h, wv.keys, wv.vals, S, sl, k0) == v) v |= (int32_t)0x80000000;
        mo.keys[base + r] = key;
        mo.vals[base + r] = v;
    }
    if (act && j == 0) {
        mo.hdr[m].len = __popcll(st);
        mo.foreign[m] = own_bits ? own_cnt : 0;
    }
}

static_assert(IN_SMALL == 32, "the longest short caller row fills a 32-lane segment");

// The four row-length groups of short caller rows, one block range each.
__global__ __launch_bounds__(256) void k_in_runs(DevSys d, MapOut mo, MapView wv, const int32_t *__restrict__ runs,
                                                 SegGrid g) {
    const int bx = blockIdx.x;
    if (bx < g.blk[1])
        in_run_segment<4>(d, mo, wv, runs + g.off[0], g.off[1] - g.off[0], bx);
    else if (bx < g.blk[2])
        in_run_segment<8>(d, mo, wv, runs + g.off[1], g.off[2] - g.off[1], bx - g.blk[1]);
    else if (bx < g.blk[3])
        in_run_segment<16>(d, mo, wv, runs + g.off[2], g.off[3] - g.off[2], bx - g.blk[2]);
    else
        in_run_segment<32>(d, mo, wv, runs + g.off[3], g.off[4] - g.off[3], bx - g.blk[3]);
}

// Hash-table segments (more references than the LDS tiers take) are built in
// two passes, neither with a global atomic on the tables:
//   k_big_stage, a block per fill item: the item's keys are counted in an LDS
//     table, and its distinct (key, count) pairs are written to the item's own
//     staging range, bucketed by the partition of each key's home slot; the
//     segment's partition table receives where each bucket starts;
//   k_big_build, a block per (segment, partition): the partition's buckets of
//     every item of the segment are added into an LDS table of the partition's
//     slots, which is copied out whole (empty slots too, so no reset is needed),
//     with the segment's key count (and, for CNT, its keys owned by another
//     class; for caller maps, the callers in the method's own class).
// Global updates are non-returning adds of a block's totals only: a
// device-scope atomic on a shared table costs a memory round trip, so a fill
// in place would be bound by rounds of them.

// tables built whole in LDS by the other builders are one partition each
static_assert(MID_HMAX <= PART_SLOTS && MAP_HMAX <= PART_SLOTS, "LDS-built tables fit one partition");
static_assert(PART_SLOTS % 256 == 0, "partitions copied out by whole blocks");

struct BigStageLds {  // a wave's member batch (row starts flattened over its lanes)
    int32_t s_start[4][WAVE];
    int32_t s_cb[4][WAVE];
    int32_t s_ab[4][WAVE];
    int32_t s_nc[4][WAVE];
    int32_t wsum[4];
};

// add n to key's count in an LDS table of hm + 1 slots that holds fewer keys
// than slots (an item's table: at least twice its entries)
__device__ __forceinline__ void stage_add(int32_t *tk, int32_t *tv, uint32_t hm, int32_t key, int32_t n, int *err) {
    uint32_t h = slot_hash(key) & hm;
    for (uint32_t probe = 0; probe <= hm; ++probe) {
        const int32_t prev = atomicCAS(&tk[h], EMPTY_KEY, key);
        if (prev == EMPTY_KEY || prev == key) {
            atomicAdd(&tv[h], n);
            return;
        }
        h = (h + 1u) & hm;
    }
    atomicOr(err, ERR_MAP_OVERFLOW);
}

// in-place exclusive prefix sum of a[0 .. n) by the block (256 threads), each
// thread summing a contiguous piece; returns the total
__device__ int block_excl_scan(int32_t *a, int n, int32_t *wsum) {
    const int tid = threadIdx.x, per = (n + 255) / 256, lo = min(n, tid * per), hi = min(n, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    const int incl = wave_incl_scan(s);
    if ((tid & (WAVE - 1)) == WAVE - 1) wsum[tid >> 6] = incl;
    __syncthreads();
    int before = incl - s;
    for (int w = 0; w < (tid >> 6); ++w) before += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    for (int i = lo; i < hi; ++i) {
        const int v = a[i];
        a[i] = before;
        before += v;
    }
    __syncthreads();
    return total;
}

// key of entry e of member y's row: its calls (CNT: the callee; W: the
// callee's class), then (W) its accesses' classes
template <int KIND>
__device__ __forceinline__ int32_t row_key(const DevSys &d, int y, int e) {
    const int cb = d.call_off[y], nc = d.call_off[y + 1] - cb;
    if (KIND == KIND_CNT) return d.call_idx[cb + e];
    return e < nc ? d.call_cls[cb + e] : d.acc_cls[d.acc_off[y] + e - nc];
}

template <int KIND>
__device__ __forceinline__ void big_stage_item(const DevSys &d, const BigItem &it, const BigMap &bm, int H,
                                               int32_t *tk, int32_t *tv, int32_t *pc, BigStageLds &L, int *err) {
    const int seg = it.seg, tid = threadIdx.x, nth = blockDim.x;
    const int32_t cap = bm.mo.hdr[seg].cap;
    const int np = cap > PART_SLOTS ? cap / PART_SLOTS : 1;
    const uint32_t hm = (uint32_t)H - 1u, cm = (uint32_t)cap - 1u;
    for (int s = tid; s < H; s += nth) {
        tk[s] = EMPTY_KEY;
        tv[s] = 0;
    }
    for (int s = tid; s <= np; s += nth) pc[s] = 0;
    if (it.j == 0 && tid == 0) {  // the build adds every partition's totals to these
        bm.mo.hdr[seg].len = 0;
        if (KIND == KIND_CNT) bm.mo.foreign[seg] = 0;
    }
    __syncthreads();
    if (KIND == KIND_IN) {
        // four callers per thread in flight; the loop runs alike in every lane
        // of a wave (lanes past the item hold no key), for the run detection
        const int lane = tid & (WAVE - 1);
        for (int w0 = it.a + (tid - lane); w0 < it.b; w0 += 4 * nth) {
            int32_t y[4], key[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = w0 + lane + u * nth;
                y[u] = i < it.b ? d.rc_idx[i] : seg;
            }
            // consecutive method ids: their owners are read almost in order
#pragma unroll
            for (int u = 0; u < 4; ++u) key[u] = y[u] != seg ? d.owner[y[u]] : -1;  // self calls are not callers
            // the lanes of a wave hold consecutive callers, and methods are
            // numbered class by class, so equal keys come in runs: the first lane
            // of each run adds the run's length
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t left = __shfl_up(key[u], 1, WAVE);
                const bool head = lane == 0 || key[u] != left;
                const uint64_t heads = __ballot(head);
                const uint64_t after = lane == WAVE - 1 ? 0ull : heads >> (lane + 1);
                const int len = after ? __ffsll((long long)after) : WAVE - lane;
                if (head && key[u] >= 0) stage_add(tk, tv, hm, key[u], len, err);
            }
        }
    } else if (it.y >= 0) {
        // a piece of one long row, four entries per thread in flight
        for (int e0 = it.a + tid; e0 < it.b; e0 += 4 * nth) {
            int32_t key[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nth;
                key[u] = e < it.b ? row_key<KIND>(d, it.y, e) : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (key[u] >= 0 && !(KIND == KIND_W && key[u] == seg)) stage_add(tk, tv, hm, key[u], 1, err);
        }
    } else {
        const int lane = tid & 63, wv = tid >> 6;
        // every wave runs the same number of batches, so the barriers match
        for (int base0 = it.a; base0 < it.b; base0 += 4 * WAVE) {
            const int j = base0 + wv * WAVE + lane;
            const int y = j < it.b ? d.mem_idx[j] : -1;
            int nc = 0, len = 0, cb = 0, ab = 0;
            if (y >= 0) {
                cb = d.call_off[y];
                ab = d.acc_off[y];
                nc = d.call_off[y + 1] - cb;
                len = (KIND == KIND_CNT) ? nc : nc + d.acc_off[y + 1] - ab;
            }
            const int incl = wave_incl_scan(len);
            const int total = __shfl(incl, WAVE - 1, WAVE);
            L.s_start[wv][lane] = incl - len;
            L.s_cb[wv][lane] = cb;
            L.s_ab[wv][lane] = ab;
            L.s_nc[wv][lane] = nc;
            __syncthreads();
            for (int e0 = lane; e0 < total; e0 += 4 * WAVE) {  // four entries per lane in flight
                int32_t key[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * WAVE;
                    key[u] = e < total ? batch_key_gather<KIND>(d, L.s_start[wv], L.s_cb[wv], L.s_ab[wv], L.s_nc[wv], e)
                                       : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (key[u] >= 0 && !(KIND == KIND_W && key[u] == seg)) stage_add(tk, tv, hm, key[u], 1, err);
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // bucket the distinct keys by the partition of their home slot: counts,
    // starts (written to the partition table), then each pair to its place
    for (int s = tid; s < H; s += nth)
        if (tk[s] != EMPTY_KEY) atomicAdd(&pc[(slot_hash(tk[s]) & cm) / PART_SLOTS], 1);
    __syncthreads();
    block_excl_scan(pc, np + 1, L.wsum);
    for (int p = tid; p <= np; p += nth) bm.bt[it.bt + (int64_t)p * it.nI + it.j] = pc[p];
    __syncthreads();
    int2 *out = bm.stage + it.stage;
    for (int s = tid; s < H; s += nth) {
        const int32_t key = tk[s];
        if (key == EMPTY_KEY) continue;
        const int q = atomicAdd(&pc[(slot_hash(key) & cm) / PART_SLOTS], 1);
        out[q] = make_int2(key, tv[s]);
    }
}

__global__ __launch_bounds__(256) void k_big_stage(DevSys d, BigWork b, int *err) {
    extern __shared__ int32_t big_dyn[];  // tk[H], tv[H], pc[np_max + 1]
    __shared__ BigStageLds L;
    const int H = b.lds_slots;
    int32_t *tk = big_dyn, *tv = big_dyn + H, *pc = big_dyn + 2 * H;
    int x = blockIdx.x;
    if (x < b.m[0].n_items) {
        big_stage_item<KIND_W>(d, b.m[0].items[x], b.m[0], H, tk, tv, pc, L, err);
        return;
    }
    x -= b.m[0].n_items;
    if (x < b.m[1].n_items) {
        big_stage_item<KIND_CNT>(d, b.m[1].items[x], b.m[1], H, tk, tv, pc, L, err);
        return;
    }
    big_stage_item<KIND_IN>(d, b.m[2].items[x - b.m[1].n_items], b.m[2], H, tk, tv, pc, L, err);
}

struct BigBuildLds {
    int32_t tk[PART_SLOTS];
    int32_t tv[PART_SLOTS];
    int32_t off[256];   // a group of 256 items: where each one's pairs start in the group's order
    int64_t src[256];   //   and where they are in the staging area
    int32_t wsum[4];
    int32_t red[2][4];
};

template <int KIND>
__device__ __forceinline__ void big_build_part(const DevSys &d, const BigPart &pt, const BigMap &bm, BigBuildLds &L,
                                               int *err) {
    const int seg = pt.seg, p = pt.p, nI = pt.nI, tid = threadIdx.x, nth = blockDim.x;
    const MapHdr g = bm.mo.hdr[seg];
    const uint32_t pm = part_mask(g.cap), cm = (uint32_t)g.cap - 1u;
    const int psz = (int)pm + 1;
    for (int s = tid; s < psz; s += nth) {
        L.tk[s] = EMPTY_KEY;
        L.tv[s] = 0;
    }
    // the partition's pairs of 256 items at a time, flattened over the block
    for (int j0 = 0; j0 < nI; j0 += nth) {
        const int j = j0 + tid;
        int cnt = 0;
        int64_t src = 0;
        if (j < nI) {
            const int32_t s0 = bm.bt[pt.bt + (int64_t)p * nI + j];
            cnt = bm.bt[pt.bt + (int64_t)(p + 1) * nI + j] - s0;
            src = bm.items[pt.i0 + j].stage + s0;
        }
        const int incl = wave_incl_scan(cnt);
        __syncthreads();  // the previous group's readers are done (and the clearing above)
        if ((tid & (WAVE - 1)) == WAVE - 1) L.wsum[tid >> 6] = incl;
        __syncthreads();
        int before = incl - cnt;
        for (int w = 0; w < (tid >> 6); ++w) before += L.wsum[w];
        const int total = L.wsum[0] + L.wsum[1] + L.wsum[2] + L.wsum[3];
        L.off[tid] = before;
        L.src[tid] = src;
        __syncthreads();
        for (int q = tid; q < total; q += nth) {
            int lo = 0, hi = nth - 1;  // the last item whose pairs start at or before q
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.off[mid] <= q) lo = mid; else hi = mid - 1;
            }
            const int2 pr = bm.stage[L.src[lo] + (q - L.off[lo])];
            uint32_t h = slot_hash(pr.x) & pm;
            bool done = false;
            for (int probe = 0; probe < psz && !done; ++probe) {
                const int32_t prev = atomicCAS(&L.tk[h], EMPTY_KEY, pr.x);
                if (prev == EMPTY_KEY || prev == pr.x) {
                    atomicAdd(&L.tv[h], pr.y);
                    done = true;
                }
                h = (h + 1u) & pm;
            }
            if (!done) atomicOr(err, ERR_MAP_OVERFLOW);
        }
    }
    __syncthreads();
    // copy the partition out whole; count its keys (and CNT's foreign keys)
    int32_t *keys = bm.mo.keys + g.base + (int64_t)p * psz;
    int32_t *vals = bm.mo.vals + g.base + (int64_t)p * psz;
    int K = 0, F = 0;
    for (int s = tid; s < psz; s += nth) {
        const int32_t k = L.tk[s];
        keys[s] = k;
        vals[s] = L.tv[s];
        K += k != EMPTY_KEY;
        if (KIND == KIND_CNT && k != EMPTY_KEY) F += d.owner[k] != seg;
    }
    K = wave_sum(K);
    if (KIND == KIND_CNT) F = wave_sum(F);
    if ((tid & (WAVE - 1)) == 0) {
        L.red[0][tid >> 6] = K;
        L.red[1][tid >> 6] = F;
    }
    __syncthreads();
    if (tid == 0) {
        K = L.red[0][0] + L.red[0][1] + L.red[0][2] + L.red[0][3];
        if (K) atomicAdd(&bm.mo.hdr[seg].len, K);
        if (KIND == KIND_CNT) {
            F = L.red[1][0] + L.red[1][1] + L.red[1][2] + L.red[1][3];
            if (F) atomicAdd(&bm.mo.foreign[seg], F);
        }
        if (KIND == KIND_IN) {
            // callers of the method in its own class: stored by the partition
            // holding that class's home slot
            const int32_t S = d.owner[seg];
            const uint32_t home = slot_hash(S) & cm;
            if ((int)(home / PART_SLOTS) == p || g.cap <= PART_SLOTS) {
                uint32_t h = home & pm;
                int32_t v = 0;
                for (int probe = 0; probe < psz; ++probe) {
                    const int32_t k = L.tk[h];
                    if (k == S) { v = L.tv[h]; break; }
                    if (k == EMPTY_KEY) break;
                    h = (h + 1u) & pm;
                }
                bm.mo.foreign[seg] = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_big_build(DevSys d, BigWork b, int *err) {
    __shared__ BigBuildLds L;
    int x = blockIdx.x;
    if (x < b.m[0].n_parts) {
        big_build_part<KIND_W>(d, b.m[0].parts[x], b.m[0], L, err);
        return;
    }
    x -= b.m[0].n_parts;
    if (x < b.m[1].n_parts) {
        big_build_part<KIND_CNT>(d, b.m[1].parts[x], b.m[1], L, err);
        return;
    }
    big_build_part<KIND_IN>(d, b.m[2].parts[x - b.m[1].n_parts], b.m[2], L, err);
}

// Loss flags of the large caller maps: item {segment, first slot, end slot}.
__global__ __launch_bounds__(256) void k_big_in_flags(DevSys d, const int4 *__restrict__ items, MapOut mo,
                                                     MapView wv) {
    const int4 it = items[blockIdx.x];
    const int m = it.x;
    const MapHdr g = mo.hdr[m];
    const int S = d.owner[m];
    const uint32_t hS = slot_hash(S);
    for (int i0 = it.y + threadIdx.x; i0 < it.z; i0 += 4 * blockDim.x) {  // four slots per thread, loads together
        int32_t key[4], v[4], k0[4];
        MapHdr h[4];
        uint32_t sl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * blockDim.x;
            key[u] = i < it.z ? mo.keys[g.base + i] : EMPTY_KEY;
            v[u] = i < it.z ? mo.vals[g.base + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) h[u] = key[u] != EMPTY_KEY ? wv.hdr[key[u]] : MapHdr{0, 0, MAP_EMPTY, 0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sl[u] = hS & ((uint32_t)h[u].cap - 1u);
            k0[u] = h[u].kind == MAP_TABLE ? wv.keys[h[u].base + sl[u]] : EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (key[u] == EMPTY_KEY) continue;
            // W tables are tables or empty: w_X(S) from the first probe on
            if (tab_get_from(h[u], wv.keys, wv.vals, S, sl[u], k0[u]) == v[u])
                mo.vals[g.base + i0 + u * blockDim.x] = v[u] | (int32_t)0x80000000;
        }
    }
}

// One wave per (class, row tile of 16 methods): full rows of G_C = B_C B_C^T on
// v_mfma_i32_16x16x64_i8, counting for each of the tile's methods the other
// methods of C with which it shares an own attribute.
__global__ __launch_bounds__(256) void k_coaccess(DevSys d, const int2 *__restrict__ items, int nitems,
                                                 const uint64_t *__restrict__ own_mask, MethodAgg *__restrict__ out) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nitems) return;
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int2 it = items[w];
    const int C = it.x, ti = it.y;
    const int mb = d.mem_off[C];
    const int n = d.mem_end[C] - mb;
    const int a = d.acnt[C];
    const int nt = (n + 15) >> 4, nkb = (a + 63) >> 6;
    const int ri = ti * 16 + r;
    const int mi = ri < n ? d.mem_idx[mb + ri] : -1;
    int rowcnt = 0;
    if (nkb > 0) {
        const v4i A0 = mask_operand(mi >= 0 ? own_mask[mi] : 0ull, grp);
        for (int tj = 0; tj < nt; ++tj) {
            const int cj = tj * 16 + r;
            const int mj = cj < n ? d.mem_idx[mb + cj] : -1;
            v4i acc = {0, 0, 0, 0};
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A0, mask_operand(mj >= 0 ? own_mask[mj] : 0ull, grp), acc,
                                                        0, 0, 0);
            for (int kb = 1; kb < nkb; ++kb)
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(attr_operand(d, mi, C, kb, grp),
                                                            attr_operand(d, mj, C, kb, grp), acc, 0, 0, 0);
            // acc[q] = G[4*grp + q][r]: row in tile ti, column in tile tj
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * grp + q;
                bool pos = (ti * 16 + row < n) && (cj < n) && !(ti == tj && row == r) && acc[q] > 0;
                unsigned long long bal = __ballot(pos);
                if (lane < 16 && (lane & 3) == q)
                    rowcnt += __popcll((bal >> (16 * (lane >> 2))) & 0xFFFFull);
            }
        }
    }
    if (lane < 16) {
        const int row = ti * 16 + lane;
        if (row < n) out[d.mem_idx[mb + row]].rnz = rowcnt;
    }
}

// Row totals of one 16-row tile from per-lane counts: lane (grp, r) holds in
// cq[q] the positive co-access entries of row 4 grp + q in its columns; the
// 16 lanes of a group are summed, the diagonal entry (a member shares its own
// attributes with itself whenever it has any) is taken off, and lane l < 16
// stores row l. row_mask / row_m: lane l holds the mask / method of the
// tile's row l (lanes 16 ti + l for the one-wave form, l for the LDS form).
__device__ __forceinline__ void co_row_totals(int (&cq)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int dd = 1; dd < 16; dd <<= 1) cq[q] += __shfl_xor(cq[q], dd, WAVE);
}

__device__ __forceinline__ int co_row_of_lane(const int (&cq)[4], int lane) {
    // row l = 4 (l >> 2) + (l & 3) is held by lane 16 (l >> 2) in cq[l & 3]
    const int src = 16 * ((lane & 15) >> 2);
    const int v0 = __shfl(cq[0], src, WAVE), v1 = __shfl(cq[1], src, WAVE);
    const int v2 = __shfl(cq[2], src, WAVE), v3 = __shfl(cq[3], src, WAVE);
    const int q = lane & 3;
    return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}

// one-wave form: lane 16 ti + l holds row l's member and mask
__device__ __forceinline__ void co_row_counts(int (&cq)[4], int ti, int n, uint64_t my_mask, int my_m,
                                              MethodAgg *__restrict__ out) {
    const int lane = threadIdx.x & (WAVE - 1);
    co_row_totals(cq);
    const int total = co_row_of_lane(cq, lane);
    const int src = ti * 16 + (lane & 15);
    const uint64_t mask = __shfl(my_mask, src, WAVE);
    const int m = __shfl(my_m, src, WAVE);
    if (lane < 16 && src < n) out[m].rnz = total - (mask != 0ull ? 1 : 0);
}

// Co-access counts for classes of at most 64 methods with at most 64 own
// attributes: one wave per class, lane l holding member l's own-attribute mask
// (one load per lane); the operands of each 16x16 tile pair come from lane
// shuffles, one INT8 MFMA per pair (co_tile: k extent 32 when the class has at
// most 32 own attributes, else 64), the positive entries off the diagonal
// counted by ballots.
__global__ __launch_bounds__(256) void k_coaccess_small(DevSys d, const int32_t *__restrict__ classes, int ncls,
                                                       const uint64_t *__restrict__ own_mask,
                                                       MethodAgg *__restrict__ out) {
    const int w = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= ncls) return;  // a whole wave leaves together
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int C = classes[w];
    const int mb = d.mem_off[C];
    const int n = d.mem_end[C] - mb;  // 1..64
    const int my_m = lane < n ? d.mem_idx[mb + lane] : -1;
    const uint64_t my_mask = my_m >= 0 ? own_mask[my_m] : 0ull;
    const int nt = (n + 15) >> 4;
    const bool k32 = d.acnt[C] <= 32;  // every own-attribute rank below 32
    for (int ti = 0; ti < nt; ++ti) {
        const uint64_t ra = __shfl(my_mask, ti * 16 + r, WAVE);
        // lane (grp, r) counts the positive entries of rows 16 ti + 4 grp + q in
        // columns 16 tj + r; members past n have no attributes and count nothing
        int cq[4] = {0, 0, 0, 0};
        for (int tj = 0; tj < nt; ++tj) {
            const v4i acc = co_tile(ra, __shfl(my_mask, tj * 16 + r, WAVE), grp, k32);
#pragma unroll
            for (int q = 0; q < 4; ++q) cq[q] += acc[q] > 0 ? 1 : 0;
        }
        co_row_counts(cq, ti, n, my_mask, my_m, out);
    }
}

// Co-access counts for classes of more than 64 methods with at most 64 own
// attributes (one k-block): a block takes four row tiles of one class (one per
// wave) and stages the own-attribute masks of the class's members in LDS,
// CO_LDS at a time; every
// wave then runs its row tile against each column tile from LDS: one INT8 MFMA
// per 16x16 tile (co_tile), the positive entries off the diagonal counted by
// ballots.
constexpr int CO_LDS = 4096;

__global__ __launch_bounds__(256) void k_coaccess_lds(DevSys d, const int2 *__restrict__ groups,
                                                     const uint64_t *__restrict__ own_mask,
                                                     MethodAgg *__restrict__ out) {
    __shared__ uint64_t sm[CO_LDS];
    const int2 it = groups[blockIdx.x];
    const int C = it.x;
    const int mb = d.mem_off[C];
    const int n = d.mem_end[C] - mb;
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int ti = it.y + (int)(threadIdx.x >> 6);
    const bool row_ok = ti * 16 < n;
    const int ri = ti * 16 + r;
    const int mi = row_ok && ri < n ? d.mem_idx[mb + ri] : -1;
    const uint64_t amask = mi >= 0 ? own_mask[mi] : 0ull;
    const bool k32 = d.acnt[C] <= 32;  // every own-attribute rank below 32
    // lane (grp, r) counts the positive entries of rows 16 ti + 4 grp + q in
    // columns c0 + 16 tj + r; members past n have no attributes and count nothing
    int cq[4] = {0, 0, 0, 0};
    for (int c0 = 0; c0 < n; c0 += CO_LDS) {  // same trip count in every wave: the barriers are reached by all
        const int cn = min(CO_LDS, n - c0);
        const int ntc = (cn + 15) >> 4;
        __syncthreads();
        // staged up to a whole tile: the columns past the class are empty masks
        for (int j = threadIdx.x; j < ntc * 16; j += blockDim.x)
            sm[j] = j < cn ? own_mask[d.mem_idx[mb + c0 + j]] : 0ull;
        __syncthreads();
        if (row_ok) {
            uint64_t next = sm[r];  // column tile 0, then each next one read before the current product
            for (int tj = 0; tj < ntc; ++tj) {
                const uint64_t cur = next;
                if (tj + 1 < ntc) next = sm[(tj + 1) * 16 + r];
                const v4i acc = co_tile(amask, cur, grp, k32);
#pragma unroll
                for (int q = 0; q < 4; ++q) cq[q] += acc[q] > 0 ? 1 : 0;
            }
        }
    }
    if (row_ok) {
        co_row_totals(cq);
        const int total = co_row_of_lane(cq, lane);
        // lane l < 16 holds row l's member (mi) and mask (amask) already
        if (lane < 16 && ri < n) out[mi].rnz = total - (amask != 0ull ? 1 : 0);
    }
}

// One segment of SEG lanes (a power of two up to a wave, aligned in it) per
// class: n, a, CBO, RFC, P, Q, LCOM_HS. C < 0: the segment has no class (its
// lanes still take part in the segment's shuffles).
template <int SEG>
__device__ __forceinline__ void finalize_class(const DevSys &d, int C, const MethodAgg *__restrict__ meth,
                                               const MapHdr *__restrict__ whdr, const int32_t *__restrict__ foreign,
                                               ClassAgg *__restrict__ out, ClassAgg *__restrict__ cls_copy,
                                               MethodAgg *__restrict__ meth_copy) {
    const int lane = threadIdx.x & (SEG - 1);
    const int mb = C >= 0 ? d.mem_off[C] : 0, me = C >= 0 ? d.mem_end[C] : 0;
    long long rs = 0, us = 0;
    for (int i0 = mb + lane; i0 < me; i0 += 4 * SEG) {  // four members per lane, their loads issued together
        int y[4];
        MethodAgg x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = i0 + u * SEG < me ? d.mem_idx[i0 + u * SEG] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = y[u] >= 0 ? meth[y[u]] : MethodAgg{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rs += x[u].rnz;
            us += x[u].u_own;
            if (meth_copy && y[u] >= 0) meth_copy[y[u]] = x[u];  // every method is a member of exactly one class
        }
    }
#pragma unroll
    for (int o = SEG / 2; o > 0; o >>= 1) {
        rs += __shfl_xor(rs, o, WAVE);
        us += __shfl_xor(us, o, WAVE);
    }
    if (lane == 0 && C >= 0) {
        const int64_t n = me - mb, a = d.acnt[C];
        ClassAgg o;
        o.n = (int32_t)n;
        o.a = (int32_t)a;
        o.cbo = whdr[C].len;
        o.rfc = (int32_t)n + foreign[C];
        o.q = rs / 2;
        o.p = n * (n - 1) / 2 - o.q;
        if (n * a == 0) {
            o.hs_num = 0;
            o.hs_den = 1;
        } else {
            o.hs_den = n * a;
            o.hs_num = n * a - us;
        }
        out[C] = o;
        if (cls_copy) cls_copy[C] = o;
    }
}

// Every class, from a list of the classes of at most FIN_SMALL members (16
// lanes each, 16 to a block) followed by the larger ones (a wave each, 4 to a
// block): most classes have a few members, so a wave each would leave most of
// its lanes idle.

__global__ __launch_bounds__(256) void k_finalize(DevSys d, const int32_t *__restrict__ list, int n_small,
                                                 int n_large, const MethodAgg *__restrict__ meth,
                                                 const MapHdr *__restrict__ whdr, const int32_t *__restrict__ foreign,
                                                 ClassAgg *__restrict__ out, ClassAgg *__restrict__ cls_copy,
                                                 MethodAgg *__restrict__ meth_copy) {
    const int nb_small = (n_small + 15) / 16;
    if ((int)blockIdx.x < nb_small) {
        const int i = blockIdx.x * 16 + (threadIdx.x >> 4);
        finalize_class<16>(d, i < n_small ? list[i] : -1, meth, whdr, foreign, out, cls_copy, meth_copy);
        return;
    }
    const int i = (blockIdx.x - nb_small) * 4 + (threadIdx.x >> 6);
    if (i >= n_large) return;  // a whole wave leaves together
    finalize_class<WAVE>(d, list[n_small + i], meth, whdr, foreign, out, cls_copy, meth_copy);
}

// the classes list[0 .. n)
__global__ __launch_bounds__(256) void k_finalize_list(DevSys d, const int32_t *__restrict__ list, int n,
                                                      const MethodAgg *__restrict__ meth,
                                                      const MapHdr *__restrict__ whdr,
                                                      const int32_t *__restrict__ foreign, ClassAgg *__restrict__ out) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    finalize_class<WAVE>(d, list[i], meth, whdr, foreign, out, nullptr, nullptr);
}

// Patches of the resident structure after a move: op {target array, index, value}.
__global__ __launch_bounds__(256) void k_scatter(const int4 *__restrict__ ops, int n, PatchTargets t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 op = ops[i];
    t.t[op.x][op.y] = op.z;
}

// flag[X] = 1 for every class X owning a caller of one of the listed methods
// (the method itself excluded); a block per listed method
__global__ __launch_bounds__(256) void k_caller_classes(DevSys d, const int32_t *__restrict__ methods,
                                                       int32_t *__restrict__ flag) {
    const int m = methods[blockIdx.x];
    for (int i = d.rc_off[m] + threadIdx.x; i < d.rc_off[m + 1]; i += blockDim.x) {
        const int y = d.rc_idx[i];
        if (y != m) flag[d.owner[y]] = 1;
    }
}

// slot of method m among the edited methods (ascending), -1 if not edited
__device__ __forceinline__ int edit_slot(const EditRows &e, int m) {
    int lo = 0, hi = e.k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (e.meth[mid] < m) lo = mid + 1; else hi = mid;
    }
    return (lo < e.k && e.meth[lo] == m) ? lo : -1;
}

__global__ __launch_bounds__(256) void k_edit_len(EditRows e) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= e.n) return;
    const int j = edit_slot(e, m);
    e.len_acc[m] = j >= 0 ? e.e_acc_off[j + 1] - e.e_acc_off[j] : e.acc_off[m + 1] - e.acc_off[m];
    e.len_call[m] = j >= 0 ? e.e_call_off[j + 1] - e.e_call_off[j] : e.call_off[m + 1] - e.call_off[m];
}

// one thread per method: its offsets and its two rows at their new places
__global__ __launch_bounds__(256) void k_edit_copy(EditRows e, const int64_t *__restrict__ pa,
                                                  const int64_t *__restrict__ pc, int32_t *__restrict__ nao,
                                                  int32_t *__restrict__ nai, int32_t *__restrict__ nco,
                                                  int32_t *__restrict__ nci) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > e.n) return;
    nao[m] = (int32_t)pa[m];
    nco[m] = (int32_t)pc[m];
    if (m == e.n) return;
    const int j = edit_slot(e, m);
    const int32_t *sa = j >= 0 ? e.e_acc_idx + e.e_acc_off[j] : e.acc_idx + e.acc_off[m];
    const int32_t *sc = j >= 0 ? e.e_call_idx + e.e_call_off[j] : e.call_idx + e.call_off[m];
    const int la = (int)(pa[m + 1] - pa[m]), lc = (int)(pc[m + 1] - pc[m]);
    for (int i = 0; i < la; ++i) nai[pa[m] + i] = sa[i];
    for (int i = 0; i < lc; ++i) nci[pc[m] + i] = sc[i];
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Callers of every method (reverse call rows): count per callee, then, from
// the prefix sum, the offsets and an atomic fill (order inside a list arbitrary).
// Callers of every method (the reverse call rows): the edges, tagged with their
// caller, are sorted by callee with a stable radix sort (so each list holds its
// callers in ascending order) and the row offsets are read off the sorted keys.
__global__ __launch_bounds__(256) void k_edge_rows(DevSys d, int32_t *__restrict__ rows) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= d.n) return;
    for (int e = d.call_off[y]; e < d.call_off[y + 1]; ++e) rows[e] = y;
}

// rc_off[t] = the first sorted edge whose callee is >= t (rc_off[n] = nnz):
// edge e writes the methods after its left neighbour's callee up to its own
__global__ __launch_bounds__(256) void k_rc_bounds(const int32_t *__restrict__ callee, int64_t nnz, int n,
                                                   int32_t *__restrict__ rc_off) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > nnz) return;
    const int lo = e == 0 ? 0 : callee[e - 1] + 1;
    const int hi = e == nnz ? n : callee[e];
    for (int t = lo; t <= hi; ++t) rc_off[t] = (int32_t)e;
}

// one block per moved method m: its callers y (entry m of y's call row) and its
// callees x (entry m of x's caller row), each found by binary search in the
// sorted row, take m's current class
__global__ __launch_bounds__(256) void k_entry_moves(DevSys d, EntryMoves mv, int32_t *__restrict__ call_cls,
                                                     int32_t *__restrict__ rc_cls) {
    const int m = mv.m[blockIdx.x];
    const int32_t T = d.owner[m];
    for (int i = d.rc_off[m] + threadIdx.x; i < d.rc_off[m + 1]; i += blockDim.x) {
        const int y = d.rc_idx[i];
        const int b = d.call_off[y];
        call_cls[b + lower_bound_i32(d.call_idx + b, d.call_off[y + 1] - b, m)] = T;
    }
    for (int e = d.call_off[m] + threadIdx.x; e < d.call_off[m + 1]; e += blockDim.x) {
        const int x = d.call_idx[e];
        const int b = d.rc_off[x];
        rc_cls[b + lower_bound_i32(d.rc_idx + b, d.rc_off[x + 1] - b, m)] = T;
    }
}

void launch_entry_moves(const DevSys &d, const EntryMoves &mv, int32_t *call_cls, int32_t *rc_cls, hipStream_t st) {
    if (mv.n > 0) k_entry_moves<<<mv.n, 256, 0, st>>>(d, mv, call_cls, rc_cls);
}

void launch_entry_classes(const DevSys &d, int64_t ncall, int64_t nacc, int32_t *call_cls, int32_t *acc_cls,
                          int32_t *rc_cls, int32_t *acc_rank, hipStream_t st) {
    if (ncall + nacc > 0)
        k_entry_classes<<<blocks_for(ncall + nacc, 256), 256, 0, st>>>(d, ncall, nacc, call_cls, acc_cls, rc_cls,
                                                                      acc_rank);
}

void launch_edge_rows(const DevSys &d, int32_t *rows, hipStream_t st) {
    if (d.n > 0) k_edge_rows<<<blocks_for(d.n, 256), 256, 0, st>>>(d, rows);
}

void launch_rc_bounds(const int32_t *callee_sorted, int64_t nnz, int n, int32_t *rc_off, hipStream_t st) {
    k_rc_bounds<<<blocks_for(nnz + 1, 256), 256, 0, st>>>(callee_sorted, nnz, n, rc_off);
}

// the two passes over the hash-table segments of the three maps
static void big_passes(const DevSys &d, const BigWork &b, hipStream_t st, KTimer *t, int *err) {
    const int n_items = b.m[0].n_items + b.m[1].n_items + b.m[2].n_items;
    const int n_parts = b.m[0].n_parts + b.m[1].n_parts + b.m[2].n_parts;
    if (n_items == 0 || n_parts == 0) return;
    MM_TIMED(t, "k_big_stage", st, k_big_stage<<<n_items, 256, big_stage_lds(b), st>>>(d, b, err));
    MM_TIMED(t, "k_big_build", st, k_big_build<<<n_parts, 256, 0, st>>>(d, b, err));
}

void launch_compute_metrics(const DevSys &d, const MetricsPlan &p, hipStream_t st, const AuxStreams *ax) {
    KTimer *t = p.timer;
    // Two chains (same stream = in order), joined by events:
    //   main: W and CNT tables grouped in LDS by waves, per-method counts and
    //         co-access, then (after chain A's tables) the caller tables grouped
    //         in LDS and the caller classes of short caller lists; the class
    //         aggregates once the other chain has joined
    //   A:    the hash-table segments of all three maps (staged by fill item,
    //         then built by partition), the W and CNT tables grouped in LDS by
    //         blocks, then (after the wave tables) the loss flags of the large
    //         caller maps
    // The host issues launches one at a time, so each chain's first kernels go first.
    // ev[5] marks every W and CNT table complete (a scoring pass that needs only
    // those maps may wait for it instead of the whole recompute).
    hipStream_t sA = ax ? ax->s[0] : st;
    if (ax) {
        (void)hipEventRecord(ax->ev[0], st);  // fork
        (void)hipStreamWaitEvent(sA, ax->ev[0], 0);
    }
    if (p.wc.n_large + p.wc.n_small > 0) {
        const int blocks = p.wc.n_large + (p.wc.n_small + 1) / 2;
        MM_TIMED(t, "k_map_tab_wc", st, k_map_tab_wc<<<blocks, 128, 0, st>>>(d, p.wc, p.w, p.cnt, p.err));
    }
    if (ax) (void)hipEventRecord(ax->ev[2], st);  // wave tables done
    big_passes(d, p.big, sA, t, p.err);
    if (p.n_w_mid + p.n_cnt_mid > 0)
        MM_TIMED(t, "k_map_tab_mid", sA,
                 k_map_tab_mid<<<p.n_w_mid + p.n_cnt_mid, 256, 0, sA>>>(d, p.w_mid, p.n_w_mid, p.cnt_mid, p.n_cnt_mid,
                                                                        p.w, p.cnt, p.err));
    if (ax) {
        (void)hipEventRecord(ax->ev[3], sA);  // hash-table segments and block tables done
        (void)hipStreamWaitEvent(sA, ax->ev[2], 0);
        (void)hipEventRecord(ax->ev[5], sA);  // every W and CNT table done: scoring may start its first pass
    }
    MapView wv{p.w.hdr, p.w.keys, p.w.vals};
    if (p.n_in_flag > 0)
        MM_TIMED(t, "k_big_in_flags", sA,
                 k_big_in_flags<<<p.n_in_flag, 256, 0, sA>>>(d, p.in_flag_items, p.in, wv));
    if (ax) (void)hipEventRecord(ax->ev[4], sA);  // chain A done
    if (d.n > 0)
        MM_TIMED(t, "k_method_basic", st, k_method_basic<<<blocks_for(d.n, 256), 256, 0, st>>>(d, p.meth, p.own_mask));
    if (p.n_co_small > 0)
        MM_TIMED(t, "k_coaccess_small", st,
                 k_coaccess_small<<<blocks_for(p.n_co_small, 4), 256, 0, st>>>(d, p.co_small, p.n_co_small,
                                                                              p.own_mask, p.meth));
    if (p.n_co_groups > 0)
        MM_TIMED(t, "k_coaccess_big", st,
                 k_coaccess_lds<<<p.n_co_groups, 256, 0, st>>>(d, p.co_groups, p.own_mask, p.meth));
    if (p.n_co_items > 0)
        MM_TIMED(t, "k_coaccess", st,
                 k_coaccess<<<blocks_for(p.n_co_items, 4), 256, 0, st>>>(d, p.co_items, p.n_co_items, p.own_mask,
                                                                        p.meth));
    if (ax) (void)hipStreamWaitEvent(st, ax->ev[3], 0);
    if (p.n_in_wave > 0)
        MM_TIMED(t, "k_map_tab_in", st, k_map_tab_in<<<p.n_in_wave, 256, 0, st>>>(d, p.in_wave, p.in, wv, p.err));
    SegGrid rg;
    rg.blk[0] = 0;
    for (int q = 0; q < 5; ++q) rg.off[q] = p.in_run_off[q];
    for (int q = 0; q < 4; ++q) {
        const int per_block = 256 / (4 << q);  // segments of 4, 8, 16, 32 lanes
        rg.blk[q + 1] = rg.blk[q] + (rg.off[q + 1] - rg.off[q] + per_block - 1) / per_block;
    }
    if (rg.blk[4] > 0)
        MM_TIMED(t, "k_in_runs", st, k_in_runs<<<rg.blk[4], 256, 0, st>>>(d, p.in, wv, p.in_runs, rg));
    if (ax) (void)hipStreamWaitEvent(st, ax->ev[4], 0);  // join
    if (p.n_fin_small + p.n_fin_large > 0)
        MM_TIMED(t, "k_finalize", st,
                 k_finalize<<<(p.n_fin_small + 15) / 16 + (p.n_fin_large + 3) / 4, 256, 0, st>>>(
                     d, p.fin_list, p.n_fin_small, p.n_fin_large, p.meth, p.w.hdr, p.cnt.foreign, p.cls, p.cls_out,
                     p.meth_out));
}

void launch_caller_classes(const DevSys &d, const int32_t *methods, int k, int32_t *flag, hipStream_t st) {
    if (k > 0) k_caller_classes<<<k, 256, 0, st>>>(d, methods, flag);
}

void launch_edit_lengths(const EditRows &e, hipStream_t st) {
    if (e.n > 0) k_edit_len<<<blocks_for(e.n, 256), 256, 0, st>>>(e);
}

void launch_edit_copy(const EditRows &e, const int64_t *pa, const int64_t *pc, int32_t *acc_off, int32_t *acc_idx,
                      int32_t *call_off, int32_t *call_idx, hipStream_t st) {
    k_edit_copy<<<blocks_for((int64_t)e.n + 1, 256), 256, 0, st>>>(e, pa, pc, acc_off, acc_idx, call_off, call_idx);
}

void launch_patch(const int4 *ops, int n, const PatchTargets &t, hipStream_t st) {
    if (n > 0) k_scatter<<<blocks_for(n, 256), 256, 0, st>>>(ops, n, t);
}

void launch_dirty_metrics(const DevSys &d, const DirtyPlan &p, hipStream_t st) {
    KTimer *t = p.timer;
    if (p.n_w + p.n_c > 0) {
        const MapTabWork wk{p.w_list, p.c_list, p.n_w, p.n_w_large, p.n_c, p.n_c_large};
        const int blocks = wk.n_w_large + wk.n_c_large + (wk.n_w - wk.n_w_large + 1) / 2 +
                           (wk.n_c - wk.n_c_large + 1) / 2;
        MM_TIMED(t, "k_map_tab_sep", st, k_map_tab_sep<<<blocks, 128, 0, st>>>(d, wk, p.w, p.cnt, p.err));
    }
    if (p.n_w_mid + p.n_c_mid > 0)
        MM_TIMED(t, "k_map_tab_mid", st,
                 k_map_tab_mid<<<p.n_w_mid + p.n_c_mid, 256, 0, st>>>(d, p.w_mid, p.n_w_mid, p.c_mid, p.n_c_mid, p.w,
                                                                      p.cnt, p.err));
    big_passes(d, p.big, st, t, p.err);
    if (p.n_basic > 0)
        MM_TIMED(t, "k_method_basic", st,
                 k_method_basic_list<<<blocks_for(p.n_basic, 256), 256, 0, st>>>(d, p.basic, p.n_basic,
                                                                                p.n_basic_zero, p.meth, p.own_mask));
    if (p.n_co_small > 0)
        MM_TIMED(t, "k_coaccess_small", st,
                 k_coaccess_small<<<blocks_for(p.n_co_small, 4), 256, 0, st>>>(d, p.co_small, p.n_co_small,
                                                                              p.own_mask, p.meth));
    if (p.n_co_groups > 0)
        MM_TIMED(t, "k_coaccess_big", st,
                 k_coaccess_lds<<<p.n_co_groups, 256, 0, st>>>(d, p.co_groups, p.own_mask, p.meth));
    if (p.n_co_items > 0)
        MM_TIMED(t, "k_coaccess", st,
                 k_coaccess<<<blocks_for(p.n_co_items, 4), 256, 0, st>>>(d, p.co_items, p.n_co_items, p.own_mask,
                                                                        p.meth));
    // caller maps: their loss flags read the W tables, complete from here on
    MapView wv{p.w.hdr, p.w.keys, p.w.vals};
    if (p.n_in_wave > 0)
        MM_TIMED(t, "k_map_tab_in", st, k_map_tab_in<<<p.n_in_wave, 256, 0, st>>>(d, p.in_wave, p.in, wv, p.err));
    SegGrid rg;
    rg.blk[0] = 0;
    for (int q = 0; q < 5; ++q) rg.off[q] = p.in_run_off[q];
    for (int q = 0; q < 4; ++q) {
        const int per_block = 256 / (4 << q);  // segments of 4, 8, 16, 32 lanes
        rg.blk[q + 1] = rg.blk[q] + (rg.off[q + 1] - rg.off[q] + per_block - 1) / per_block;
    }
    if (rg.blk[4] > 0)
        MM_TIMED(t, "k_in_runs", st, k_in_runs<<<rg.blk[4], 256, 0, st>>>(d, p.in, wv, p.in_runs, rg));
    if (p.n_in_flag > 0)
        MM_TIMED(t, "k_big_in_flags", st, k_big_in_flags<<<p.n_in_flag, 256, 0, st>>>(d, p.in_flag, p.in, wv));
    if (p.n_fin > 0)
        MM_TIMED(t, "k_finalize", st,
                 k_finalize_list<<<blocks_for(p.n_fin, 4), 256, 0, st>>>(d, p.fin, p.n_fin, p.meth, p.w.hdr,
                                                                        p.cnt.foreign, p.cls));
}

}  // namespace mm

// mm_dev.h -- device-side data views and helpers shared by the gfx950 kernels.
//
// Data kept resident per system (int32 ids, int32 offsets):
//   owner[n]        class of every method (changes with moves)
//   acls[na]        class of every attribute; alocal[na] its rank inside the class
//   acnt[c]         attributes per class
//   acc / call      method -> attribute and method -> method rows, sorted, no repeats
//   rc              callers of every method (reverse of call)
//   mem             methods of every class: rows mem_idx[mem_off[C] .. mem_end[C])
//                   of a pool in which a row may be moved to the end to grow
//
// Grouped counts ("maps") are stored per segment (a class or a method), either
//   as an open-addressing hash table (kind TABLE): cap (a power of two) slots at
//   keys/vals[base ..], empty slots hold key -1, len = number of keys; or as a
//   sorted run (kind RUN): keys[base .. base + len) ascending (short caller
//   lists, grouped by one lane). Every segment is built in LDS and copied out
//   whole. A key's home slot is slot_hash(key) & (cap - 1), and a probe moves
//   to the next slot inside the key's partition: tables of more than PART_SLOTS
//   slots are cut into partitions of PART_SLOTS slots (the home slot's high
//   bits choose one), so that one block can build each partition alone; a
//   smaller table is one partition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

constexpr int WAVE = 64;
constexpr int MAP_CAP = 512;        // segments of at most this many references group in LDS by a wave (caller maps: a block)
constexpr int MAP_HMAX = 1024;      // LDS table slots of the map builder (2 * MAP_CAP)
constexpr int MID_CAP = 2048;       // W/CNT segments of MAP_CAP..MID_CAP references group in LDS by a block (large systems)
constexpr int MID_HMAX = 4096;      // LDS table slots of a block grouping a segment of up to MID_CAP references
constexpr int MAP_HSMALL = 512;     // LDS slots of one wave's region in the W/CNT builders (an item needing more takes two)
constexpr int IN_SMALL = 32;        // caller rows up to this length are grouped by a lane segment
constexpr int CALLER_LIGHT = 32;    // caller classes handled inline by the delta kernel
constexpr int BIG_CHUNK = 1024;     // most entries per fill item of a hash-table segment
constexpr int BIG_CHUNK_MIN = 256;  //   and fewest (systems with few such references get more, smaller items)
constexpr int BIG_ITEMS_TARGET = 2048;  // fill items aimed at over all large segments
constexpr int PART_SLOTS = 4096;    // slots of a table partition (larger tables probe inside theirs)
constexpr int PART_MAX = 4096;      // most partitions of one table (tables of at most 2^24 slots)
constexpr int HEAVY_CHUNK = 256;    // caller-class slots per heavy work item (one per lane)
constexpr int FIN_SMALL = 64;       // classes of at most this many members are aggregated by 16 lanes, others by a wave
constexpr int PREP_SIDE_MIN = 1 << 17;  // methods from which scoring's first pass runs beside the metric recompute
constexpr int MID_TIER_MIN = 1 << 17;   // methods from which W/CNT tables of MAP_CAP..MID_CAP references take a block
constexpr int32_t EMPTY_KEY = -1;

enum { MAP_EMPTY = 0, MAP_TABLE = 1, MAP_RUN = 2 };

// error bits reported by kernels
constexpr int ERR_MAP_OVERFLOW = 1;
constexpr int ERR_HEAVY_OVERFLOW = 2;
constexpr int ERR_SCAN = 4;  // a prefix-sum tile found no published predecessor
constexpr int ERR_CYCLE = 8;  // a class hierarchy with a cycle

struct MapHdr {          // 16 bytes
    int32_t base;        // first slot
    int32_t len;         // keys present (written by the builder)
    int32_t kind;        // MAP_EMPTY / MAP_TABLE / MAP_RUN
    int32_t cap;         // table slots (a power of two) or run capacity
};

struct DevSys {
    int32_t c, n, na, pad;
    const int32_t *owner, *acls, *alocal, *acnt;
    const int32_t *acc_off, *acc_idx, *call_off, *call_idx, *rc_off, *rc_idx;
    const int32_t *mem_off, *mem_end, *mem_idx;  // class C's methods: mem_idx[mem_off[C] .. mem_end[C])
    // the class of every row entry, gathered once per change of the structure or
    // the owners (k_entry_classes): call_cls[e] = owner[call_idx[e]], acc_cls[e] =
    // acls[acc_idx[e]], rc_cls[e] = owner[rc_idx[e]], and acc_rank[e] =
    // alocal[acc_idx[e]]. Valid for the metric and scoring kernels (the metric
    // recompute builds them first when stale).
    const int32_t *call_cls, *acc_cls, *rc_cls, *acc_rank;
};

struct MapView {
    const MapHdr *hdr;
    const int32_t *keys;
    const int32_t *vals;
};

struct ClassAgg {        // same layout as mm_class_metrics (48 bytes)
    int32_t n, a, cbo, rfc;
    int64_t p, q, hs_num, hs_den;
};

struct MethodAgg {       // same layout as mm_method_metrics (16 bytes)
    int32_t fan_in, fan_out, u_own, rnz;
};

struct MoveRec {         // same layout as mm_move_score (96 bytes)
    int32_t method, src, dst;
    int32_t d_cbo_src, d_cbo_dst, d_rfc_src, d_rfc_dst;
    int32_t n_caller_cls, n_caller_worse, n_caller_better;
    int32_t keep, pad;
    int64_t d_lcom_src, d_lcom_dst;
    int64_t hs_num_src, hs_den_src, hs_num_dst, hs_den_dst;
};

struct CkOut {            // same layout as mm_class_ck (16 bytes)
    int64_t wmc;
    int32_t noc, dit;
};

// per-method terms of the move deltas that do not depend on the destination
struct MethodPrep {      // 32 bytes
    int32_t S;           // current class
    int32_t nout;        // distinct classes referenced (calls + accesses, self-call excluded)
    int32_t s_entry;     // index of S in the out run, -1 if absent
    int32_t lose_src;    // classes S stops using when m leaves (INT32_MIN: left to the candidates that need it)
    int32_t d_rfc_src;   // RFC delta of S (independent of the destination)
    int32_t in_src;      // callers of m inside S (m excluded)
    int32_t nin;         // distinct classes owning a caller of m (m excluded)
    int32_t ncand;       // REFERENCED candidates of m
};

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// slot hash of the LDS and global open-addressing tables
__device__ __forceinline__ uint32_t slot_hash(int32_t key) {
    return fmix32((uint32_t)key ^ 0x9e3779b9u);
}

// lower_bound over a sorted int32 run
__device__ __forceinline__ int lower_bound_i32(const int32_t *k, int len, int32_t key) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (k[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// mask of the slots of one partition of a table of `cap` slots
__host__ __device__ __forceinline__ uint32_t part_mask(int32_t cap) {
    return (uint32_t)(cap < PART_SLOTS ? cap : PART_SLOTS) - 1u;
}

// the slot a probe visits after `slot`: the next one, wrapping inside the
// partition (pm = part_mask(cap))
__device__ __forceinline__ uint32_t probe_next(uint32_t slot, uint32_t pm) {
    return (slot & ~pm) | ((slot + 1u) & pm);
}

// count stored for `key` in a segment whose header is loaded, 0 if absent (for
// caller maps the value carries a flag in bit 31: mask it with 0x7fffffff)
__device__ __forceinline__ int32_t map_get_h(const MapHdr &h, const int32_t *keys, const int32_t *vals,
                                             int32_t key) {
    if (h.kind == MAP_RUN) {
        const int i = lower_bound_i32(keys + h.base, h.len, key);
        return (i < h.len && keys[h.base + i] == key) ? vals[h.base + i] : 0;
    }
    if (h.kind != MAP_TABLE) return 0;
    const uint32_t pm = part_mask(h.cap);
    uint32_t slot = slot_hash(key) & ((uint32_t)h.cap - 1u);
    for (uint32_t probe = 0; probe <= pm; ++probe) {
        const int32_t k = keys[h.base + slot];
        if (k == key) return vals[h.base + slot];
        if (k == EMPTY_KEY) return 0;
        slot = probe_next(slot, pm);
    }
    return 0;
}

// Slot of `key` in a segment whose header is loaded, or -1 when absent. For a
// table, `slot`/`k0` are the first probe (k0 read already, EMPTY_KEY for a
// segment that is not a table); a run is scanned eight keys at a time, the
// loads of each batch issued together. Splitting the lookup this way lets a
// caller issue the first probes of several lookups, then their value loads,
// together.
__device__ __forceinline__ int map_find_from(const MapHdr &h, const int32_t *keys, int32_t key, uint32_t slot,
                                             int32_t k0) {
    if (h.kind == MAP_RUN) {
        for (int i0 = 0; i0 < h.len; i0 += 8) {
            int32_t k[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) k[u] = i0 + u < h.len ? keys[h.base + i0 + u] : INT32_MAX;
            int hit = -1;
#pragma unroll
            for (int u = 0; u < 8; ++u) hit = (hit < 0 && k[u] == key) ? i0 + u : hit;
            if (hit >= 0) return hit;
            if (k[7] > key) return -1;  // sorted run: every later key is larger
        }
        return -1;
    }
    if (h.kind != MAP_TABLE) return -1;
    const uint32_t pm = part_mask(h.cap);
    int32_t k = k0;
    for (uint32_t probe = 0; probe <= pm; ++probe) {
        if (k == key) return (int)slot;
        if (k == EMPTY_KEY) return -1;
        slot = probe_next(slot, pm);
        k = keys[h.base + slot];
    }
    return -1;
}

// first probe of a table lookup: its slot, and the key stored there
__device__ __forceinline__ int32_t map_probe_first(const MapHdr &h, const int32_t *keys, int32_t key,
                                                   uint32_t &slot) {
    slot = slot_hash(key) & ((uint32_t)h.cap - 1u);
    return h.kind == MAP_TABLE ? keys[h.base + slot] : EMPTY_KEY;
}

// count stored for `key` in segment `s`
__device__ __forceinline__ int32_t map_get(const MapView &mv, int32_t s, int32_t key) {
    return map_get_h(mv.hdr[s], mv.keys, mv.vals, key);
}

// presence of `key` in a table segment whose header is already loaded (kinds
// EMPTY / TABLE), continuing a probe from `slot` whose key `k0` was read already
__device__ __forceinline__ bool tab_has_from(const MapHdr &h, const int32_t *keys, int32_t key, uint32_t slot,
                                             int32_t k0) {
    if (k0 == key) return true;
    if (k0 == EMPTY_KEY) return false;
    const uint32_t pm = part_mask(h.cap);
    for (uint32_t probe = 1; probe <= pm; ++probe) {
        slot = probe_next(slot, pm);
        const int32_t k = keys[h.base + slot];
        if (k == key) return true;
        if (k == EMPTY_KEY) return false;
    }
    return false;
}

// count stored for `key` in a table segment whose header is loaded, continuing a
// probe from `slot` whose key `k0` was read already; 0 if absent
__device__ __forceinline__ int32_t tab_get_from(const MapHdr &h, const int32_t *keys, const int32_t *vals,
                                                int32_t key, uint32_t slot, int32_t k0) {
    if (k0 == EMPTY_KEY) return 0;
    const uint32_t pm = part_mask(h.cap);
    int32_t k = k0;
    for (uint32_t probe = 0; probe <= pm; ++probe) {
        if (k == key) return vals[h.base + slot];
        if (k == EMPTY_KEY) return 0;
        slot = probe_next(slot, pm);
        k = keys[h.base + slot];
    }
    return 0;
}

// Counts of four keys (use[u] false: 0) in one table segment, first probes
// issued together.
__device__ __forceinline__ void tab_get4(const MapHdr &h, const int32_t *keys, const int32_t *vals,
                                         const int32_t (&key)[4], const bool (&use)[4], int32_t (&out)[4]) {
    uint32_t sl[4];
    int32_t k0[4];
    const uint32_t m = (uint32_t)h.cap - 1u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        sl[u] = slot_hash(key[u]) & m;
        k0[u] = (use[u] && h.kind == MAP_TABLE) ? keys[h.base + sl[u]] : EMPTY_KEY;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) out[u] = tab_get_from(h, keys, vals, key[u], sl[u], k0[u]);
}

// Presence of four keys (use[u] false: ignored) in one table segment, with the
// four first probes issued together; returns how many used keys are absent.
__device__ __forceinline__ int tab_absent4(const MapHdr &h, const int32_t *keys, const int32_t (&key)[4],
                                          const bool (&use)[4]) {
    if (h.kind != MAP_TABLE) return (int)use[0] + (int)use[1] + (int)use[2] + (int)use[3];
    const uint32_t m = (uint32_t)h.cap - 1u;
    uint32_t sl[4];
    int32_t k0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        sl[u] = slot_hash(key[u]) & m;
        k0[u] = use[u] ? keys[h.base + sl[u]] : EMPTY_KEY;
    }
    int absent = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (use[u]) absent += !tab_has_from(h, keys, key[u], sl[u], k0[u]);
    return absent;
}

// number of slots to visit when iterating a segment's entries
__device__ __forceinline__ int map_slots(const MapHdr &h) {
    return h.kind == MAP_TABLE ? h.cap : (h.kind == MAP_RUN ? h.len : 0);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// inclusive prefix sum across the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int v) {
    int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

typedef int v4i __attribute__((ext_vector_type(4)));

// Bits of acc(m) restricted to the attributes of class C whose rank inside C is
// in [64 kb, 64 kb + 64). m < 0 gives 0 (a padding row of an MFMA tile).
__device__ __forceinline__ uint64_t attr_bits(const DevSys &d, int m, int C, int kb) {
    if (m < 0) return 0;
    uint64_t bits = 0;
    const int lo = kb * 64;
    for (int e = d.acc_off[m]; e < d.acc_off[m + 1]; ++e) {
        const int li = d.acc_rank[e] - lo;  // read beside the class, not through the attribute
        if (d.acc_cls[e] == C && (unsigned)li < 64u) bits |= 1ull << li;
    }
    return bits;
}

// 16 bits -> 16 bytes of 0/1: one lane's slice of an int8 MFMA operand. A
// nibble x times 0x204081 holds x at bit offsets 0, 7, 14 and 21, so bit k of x
// lands on bit 8k; the mask keeps exactly those four bits.
__device__ __forceinline__ v4i expand16(uint32_t b) {
    v4i r;
#pragma unroll
    for (int w = 0; w < 4; ++w) r[w] = (int)((((b >> (4 * w)) & 0xFu) * 0x204081u) & 0x01010101u);
    return r;
}

// Operand slice of lane group `grp` (lanes 16 grp .. 16 grp + 15) for method m:
// byte b of the slice stands for the attribute of rank 64 kb + 16 grp + b. The
// A and B operands of v_mfma_i32_16x16x64_i8 are built the same way, so each
// product term pairs the same attribute on both sides whatever order the
// instruction assigns to the 64 k-slots.
__device__ __forceinline__ v4i attr_operand(const DevSys &d, int m, int C, int kb, int grp) {
    return expand16((uint32_t)(attr_bits(d, m, C, kb) >> (16 * grp)) & 0xFFFFu);
}

__device__ __forceinline__ v4i mask_operand(uint64_t bits, int grp) {
    return expand16((uint32_t)(bits >> (16 * grp)) & 0xFFFFu);
}

// 8 bits -> 8 bytes of 0/1 (byte k stands for bit k), as expand16 does for 16
__device__ __forceinline__ long expand8(uint32_t b) {
    const uint32_t lo = ((b & 0xFu) * 0x204081u) & 0x01010101u;
    const uint32_t hi = (((b >> 4) & 0xFu) * 0x204081u) & 0x01010101u;
    return (long)(((uint64_t)hi << 32) | lo);
}

// One 16x16 tile of a co-access product: entry (i, j) counts the attributes
// that row i's mask (lane group grp's rows come from `ra`) shares with column
// j's (`cb`), each lane passing its own row's and column's masks. When every
// attribute rank is below 32 (k32, uniform over the wave) it is one
// v_mfma_i32_16x16x32_i8 on 8-byte slices (lane group grp: ranks 8 grp ..
// 8 grp + 7), half the k extent of v_mfma_i32_16x16x64_i8, which takes the
// other masks (ranks below 64). A and B slices are built alike in either form,
// so each product term pairs one attribute with itself. acc[q] holds entry
// (4 grp + q, r) of the tile, r = lane mod 16.
__device__ __forceinline__ v4i co_tile(uint64_t ra, uint64_t cb, int grp, bool k32) {
    v4i acc = {0, 0, 0, 0};
    if (k32)
        return __builtin_amdgcn_mfma_i32_16x16x32_i8(expand8((uint32_t)(ra >> (8 * grp)) & 0xFFu),
                                                     expand8((uint32_t)(cb >> (8 * grp)) & 0xFFu), acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(mask_operand(ra, grp), mask_operand(cb, grp), acc, 0, 0, 0);
}

// LCOM (original form) of a class with n methods and Q sharing pairs: P - Q
__device__ __forceinline__ int64_t lcom_pq(int64_t n, int64_t q) {
    return n * (n - 1) / 2 - 2 * q;
}

}  // namespace mm

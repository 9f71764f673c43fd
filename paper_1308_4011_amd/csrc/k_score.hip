// k_score.hip -- gfx950 kernels scoring Move Method candidates (m -> T) by their
// exact metric deltas on every affected class (Sec. III-A; Sec. IV-C re-runs the
// metric functions on the changed membership, which these deltas equal).
//
// Notation: S = class of m, out_m(D) = references of m (calls and accesses, the
// self-call excluded) to members of D, in_m(X) = callers of m in class X (m
// excluded), w_C(D) = references from C's methods to D's members (the CBO map),
// cnt_C(x) = methods of C calling x (the RFC map), U_C = own-attribute uses.
//
//   CBO   S keeps D != T iff w_S(D) > out_m(D); S uses T afterwards iff
//         w_S(T) - out_m(T) + in_m(S) > 0. T gains D not in {S, T} iff
//         w_T(D) = 0; T uses S afterwards iff w_T(S) + out_m(S) - in_m(T) > 0.
//         A caller class X gains T iff w_X(T) = 0 and loses S iff
//         w_X(S) = in_m(X).
//   RFC   S loses m iff no other method of S calls m, and loses each callee x
//         of m outside S that no other method of S calls; T gains m iff no
//         method of T calls m, and gains each callee x outside T that none of
//         T's methods calls.
//   LCOM  Q_S' = Q_S - rnz(m); Q_T' = Q_T + h_T(m), h_T(m) = methods of T that
//         share an attribute of T with m (INT8 MFMA, candidates grouped by T).
//   HS    U_S' = U_S - |acc(m) in A_S|, U_T' = U_T + |acc(m) in A_T|.
//
// Phases: k_prep (per method: its out run, sorted by class, and the
// destination-independent terms; a keep_only pass leaves the origin's map terms
// to the candidates that need them; on large systems it runs beside the metric
// recompute, and k_prep_in adds the caller terms after it), k_ref_fill
// (REFERENCED list), k_a9_* (the candidates whose method accesses an attribute
// of T, grouped by T; h_T(m) on MFMA), k_delta (one lane per candidate, in
// candidate order: every delta, the caller classes of short caller lists, the
// keep rule; the keep_only form takes the later stages of the few candidates
// left after stage A by the whole wave), k_heavy (long caller lists),
// compaction of the kept records.
#include <algorithm>

#include <stdexcept>

#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

constexpr int PREP_LDS = 32;
constexpr int32_t SRC_LAZY = INT32_MIN;  // origin-class term not computed by k_prep

// RFC change of S when m leaves, from m's call row (k_prep's eager form): -1 if no other method of S calls m, and -1 per
// callee outside S that no other method of S calls (cnt_S(x) == 1)
__device__ __forceinline__ int src_rfc(const DevSys &d, const ScorePlan &p, int m, int S) {
    const MapHdr hcS = p.cnt.hdr[S];
    const int cb = d.call_off[m], ce = d.call_off[m + 1];
    const int sp = lower_bound_i32(d.call_idx + cb, ce - cb, m);
    const int self = (sp < ce - cb && d.call_idx[cb + sp] == m) ? 1 : 0;
    int drs = (map_get_h(hcS, p.cnt.keys, p.cnt.vals, m) - self == 0) ? -1 : 0;
    for (int e0 = cb; e0 < ce; e0 += 4) {
        int32_t x[4], cx[4], got[4];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // callee and its class loaded together
            x[u] = e0 + u < ce ? d.call_idx[e0 + u] : -2;
            cx[u] = e0 + u < ce ? d.call_cls[e0 + u] : S;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) use[u] = x[u] >= 0 && x[u] != m && cx[u] != S;
        tab_get4(hcS, p.cnt.keys, p.cnt.vals, x, use, got);
#pragma unroll
        for (int u = 0; u < 4; ++u) drs -= (use[u] && got[u] == 1) ? 1 : 0;
    }
    return drs;
}

__global__ __launch_bounds__(128) void k_prep_long(DevSys d, ScorePlan p, int32_t *__restrict__ ref_count,
                                                   const int32_t *__restrict__ list, int n_list) {
    __shared__ int32_t buf[128 * PREP_LDS];
    __shared__ int32_t cbuf[128 * PREP_LDS];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_list) return;
    const int m = list[i];
    const int S = d.owner[m];
    const int cb = d.call_off[m], ce = d.call_off[m + 1];
    const int ab = d.acc_off[m], ae = d.acc_off[m + 1];
    const int nc = ce - cb;
    const int64_t off = (int64_t)ab + cb;
    const int R = nc + (ae - ab);
    // lookups that depend only on m and S, issued first
    const bool eager = !p.lazy_src;
    const MapHdr hwS = eager ? p.w.hdr[S] : MapHdr{0, 0, MAP_EMPTY, 0};
    const MapHdr hcS = eager ? p.cnt.hdr[S] : MapHdr{0, 0, MAP_EMPTY, 0};
    const int32_t cSm = eager ? map_get_h(hcS, p.cnt.keys, p.cnt.vals, m) : 0;
    int32_t *ok = p.outk + off;
    int32_t *oc = p.outc + off;
    int32_t *oa = p.outa + off;
    // private sort area: column-major LDS slice (element j at j * 128 + lane,
    // conflict-free), or the method's own out region for long rows
    const bool in_lds = R <= PREP_LDS;
    int32_t *kb = in_lds ? buf + threadIdx.x : ok;
    const int ks = in_lds ? 128 : 1;
    // referenced classes, tagged call (0) / access (1), insertion-sorted; the
    // row entries and their classes are loaded four at a time
    int k = 0, self = 0;
    for (int e0 = 0; e0 < R; e0 += 4) {
        int32_t x[4], cx[4], key[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // entry and its class loaded together
            const int e = e0 + u;
            x[u] = e < R ? (e < nc ? d.call_idx[cb + e] : d.acc_idx[ab + e - nc]) : -1;
            cx[u] = e < R ? (e < nc ? d.call_cls[cb + e] : d.acc_cls[ab + e - nc]) : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u;
            key[u] = e >= R ? -1 : (e < nc ? (x[u] == m ? -1 : cx[u] * 2) : cx[u] * 2 + 1);
            self += (e < nc && x[u] == m) ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (key[u] < 0) continue;
            int j = k++;
            while (j > 0 && kb[(j - 1) * ks] > key[u]) {
                kb[j * ks] = kb[(j - 1) * ks];
                --j;
            }
            kb[j * ks] = key[u];
        }
    }
    // group by class: the out run (class, references, accesses); class and
    // count also kept in the private slice for the lookups below
    int32_t *cnb = in_lds ? cbuf + threadIdx.x : oc;
    int K = 0, s_entry = -1;
    for (int i = 0; i < k;) {
        const int32_t D = kb[i * ks] >> 1;
        int j = i, na = 0;
        while (j < k && (kb[j * ks] >> 1) == D) na += kb[(j++) * ks] & 1;
        if (D == S) s_entry = K;
        ok[K] = D;
        oc[K] = j - i;
        oa[K] = na;
        // REFERENCED: the candidate (m, D) needs h_D(m) when m accesses D's attributes
        if (p.grouped && na > 0 && D != S) atomicAdd(&p.gcnt[D], 1);  // counted; the slot is taken at the fill
        kb[K * ks] = D;
        cnb[K * ks] = j - i;
        ++K;
        i = j;
    }
    // classes S stops using: w_S(D) == out_m(D) (lazy form: left to the
    // candidates that reach the CBO stage)
    int lose = eager ? 0 : SRC_LAZY;
    for (int q0 = 0; eager && q0 < K; q0 += 4) {
        int32_t key[4], got[4];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u;
            key[u] = q < K ? kb[q * ks] : -2;
            use[u] = q < K && q != s_entry;
        }
        tab_get4(hwS, p.w.keys, p.w.vals, key, use, got);
#pragma unroll
        for (int u = 0; u < 4; ++u) lose += (use[u] && got[u] == cnb[(q0 + u) * ks]) ? 1 : 0;
    }
    if (p.lazy_src) {  // the RFC term of S is left to the candidates that need it
        MethodPrep r;
        r.S = S;
        r.nout = K;
        r.s_entry = s_entry;
        r.lose_src = lose;
        r.d_rfc_src = SRC_LAZY;
        r.in_src = p.prep_in_late ? 0 : p.in_own[m];  // else k_prep_in fills them
        r.nin = p.prep_in_late ? 0 : p.in.hdr[m].len;
        r.ncand = K - (s_entry >= 0 ? 1 : 0);
        p.prep[m] = r;
        if (ref_count) ref_count[m] = r.ncand;
        return;
    }
    // RFC of S: callees x of m outside S with cnt_S(x) == 1
    int drs = (cSm - self == 0) ? -1 : 0;
    for (int e0 = cb; e0 < ce; e0 += 4) {
        int32_t x[4], cx[4], got[4];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // callee and its class loaded together
            x[u] = e0 + u < ce ? d.call_idx[e0 + u] : -2;
            cx[u] = e0 + u < ce ? d.call_cls[e0 + u] : S;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) use[u] = x[u] >= 0 && x[u] != m && cx[u] != S;
        tab_get4(hcS, p.cnt.keys, p.cnt.vals, x, use, got);
#pragma unroll
        for (int u = 0; u < 4; ++u) drs -= (use[u] && got[u] == 1) ? 1 : 0;
    }
    MethodPrep r;
    r.S = S;
    r.nout = K;
    r.s_entry = s_entry;
    r.lose_src = lose;
    r.d_rfc_src = drs;
    r.in_src = p.prep_in_late ? 0 : p.in_own[m];  // else k_prep_in fills them
    r.nin = p.prep_in_late ? 0 : p.in.hdr[m].len;
    r.ncand = K - (s_entry >= 0 ? 1 : 0);
    p.prep[m] = r;
    if (ref_count) ref_count[m] = r.ncand;
}

// The same per-method preparation for rows of up to 64 entries: a segment of
// SEG lanes (SEG >= the row length) takes one method, one lane per call or
// access. The referenced classes, tagged call / access, are sorted by a
// bitonic network of lane shuffles; ballots over the sorted keys give the out
// run (a lane whose class differs from its left neighbour starts an entry; its
// rank among the starts is the entry's index, the next start bounds its
// references, and the access tags inside that range count its accesses). The
// lookups that depend only on the lane's own element (the W entry of S for the
// class, the call count of S for the callee) go out in parallel.
template <int SEG>
__device__ __forceinline__ void prep_segment(const DevSys &d, const ScorePlan &p, int32_t *__restrict__ ref_count,
                                             const int32_t *__restrict__ list, int n_list, int blk) {
    static_assert(SEG >= 2 && SEG <= WAVE && (SEG & (SEG - 1)) == 0, "segment of 2..64 lanes");
    const int lane = threadIdx.x & (WAVE - 1);
    const int j = threadIdx.x & (SEG - 1);
    const int seg = blk * (int)(blockDim.x / SEG) + (int)threadIdx.x / SEG;
    const bool act = seg < n_list;
    const int m = act ? list[seg] : -1;
    int S = -1, cb = 0, nc = 0, ab = 0, R = 0;
    if (act) {
        S = d.owner[m];
        cb = d.call_off[m];
        nc = d.call_off[m + 1] - cb;
        ab = d.acc_off[m];
        R = nc + (d.acc_off[m + 1] - ab);
    }
    const int64_t off = (int64_t)ab + cb;
    const bool eager = !p.lazy_src;
    const MapHdr empty{0, 0, MAP_EMPTY, 0};
    const MapHdr hwS = act && eager ? p.w.hdr[S] : empty;
    const MapHdr hcS = act && eager ? p.cnt.hdr[S] : empty;
    // this lane's element: class * 2 for a call (self calls excluded), class * 2 + 1 for an access
    int32_t x = -1, key = INT32_MAX;
    bool self = false, foreign_call = false;
    if (j < R) {
        if (j < nc) {
            x = d.call_idx[cb + j];
            const int32_t ox = d.call_cls[cb + j];  // loaded beside x
            self = x == m;
            foreign_call = !self && ox != S;
            if (!self) key = ox * 2;
        } else {
            key = d.acc_cls[ab + j - nc] * 2 + 1;
        }
    }
    // RFC of S (eager form): callees outside S that only this method of S calls
    bool rfc_hit = false;
    int32_t cSm = 0;
    if (eager) {
        if (foreign_call && hcS.kind == MAP_TABLE) {
            const uint32_t sl = slot_hash(x) & ((uint32_t)hcS.cap - 1u);
            rfc_hit = tab_get_from(hcS, p.cnt.keys, p.cnt.vals, x, sl, p.cnt.keys[hcS.base + sl]) == 1;
        }
        if (act && j == 0) cSm = map_get_h(hcS, p.cnt.keys, p.cnt.vals, m);
    }
#pragma unroll
    for (int kk = 2; kk <= SEG; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const int32_t q = __shfl_xor(key, jj, WAVE);
            const bool take_min = ((j & jj) == 0) == ((j & kk) == 0);
            key = take_min ? min(key, q) : max(key, q);
        }
    }
    const int32_t left = __shfl_up(key, 1, WAVE);
    const bool valid = key != INT32_MAX;
    const int32_t D = key >> 1;
    const bool start = valid && (j == 0 || (left >> 1) != D);
    const int sbase = lane & ~(SEG - 1);
    const uint64_t segmask = (SEG == WAVE ? ~0ull : ((1ull << SEG) - 1ull)) << sbase;
    const uint64_t st = __ballot(start) & segmask;
    const uint64_t vm = __ballot(valid) & segmask;
    const uint64_t am = __ballot(valid && (key & 1)) & segmask;
    const uint64_t below = (1ull << lane) - 1ull;
    const uint64_t above = st & ~((2ull << lane) - 1ull);
    const int end = above ? __ffsll((long long)above) - 1 : sbase + __popcll(vm);
    const uint64_t before_end = end >= WAVE ? ~0ull : ((1ull << end) - 1ull);
    const int cnt = end - lane;
    const int na = __popcll(am & before_end & ~below);
    const uint64_t s_bits = __ballot(start && D == S) & segmask;
    bool lose_bit = false;
    if (start) {
        const int r = __popcll(st & below);
        p.outk[off + r] = D;
        p.outc[off + r] = cnt;
        p.outa[off + r] = na;
        // REFERENCED: the candidate (m, D) needs h_D(m) when m accesses D's attributes
        if (p.grouped && na > 0 && D != S) atomicAdd(&p.gcnt[D], 1);  // counted; the slot is taken at the fill
        // S stops using D: w_S(D) equals m's references to D (eager form)
        if (D != S && hwS.kind == MAP_TABLE) {
            const uint32_t sl = slot_hash(D) & ((uint32_t)hwS.cap - 1u);
            lose_bit = tab_get_from(hwS, p.w.keys, p.w.vals, D, sl, p.w.keys[hwS.base + sl]) == cnt;
        }
    }
    const int lose = eager ? __popcll(__ballot(lose_bit) & segmask) : SRC_LAZY;
    const int selfc = __popcll(__ballot(self) & segmask);
    const int rfc = __popcll(__ballot(rfc_hit) & segmask);
    if (act && j == 0) {
        const int K = __popcll(st);
        const int s_entry = s_bits ? __popcll(st & ((1ull << (__ffsll((long long)s_bits) - 1)) - 1ull)) : -1;
        MethodPrep r;
        r.S = S;
        r.nout = K;
        r.s_entry = s_entry;
        r.lose_src = lose;
        r.d_rfc_src = eager ? ((cSm - selfc == 0) ? -1 : 0) - rfc : SRC_LAZY;
        r.in_src = p.prep_in_late ? 0 : p.in_own[m];  // else k_prep_in fills them
        r.nin = p.prep_in_late ? 0 : p.in.hdr[m].len;
        r.ncand = K - (s_entry >= 0 ? 1 : 0);
        p.prep[m] = r;
        if (ref_count) ref_count[m] = r.ncand;
    }
}

// Row-length groups of up to 8, 16, 32 and 64 entries, one block range each.
__global__ __launch_bounds__(256) void k_prep(DevSys d, ScorePlan p, int32_t *__restrict__ ref_count, SegGrid g) {
    const int bx = blockIdx.x;
    const int32_t *L = p.prep_runs;
    if (bx < g.blk[1])
        prep_segment<8>(d, p, ref_count, L + g.off[0], g.off[1] - g.off[0], bx);
    else if (bx < g.blk[2])
        prep_segment<16>(d, p, ref_count, L + g.off[1], g.off[2] - g.off[1], bx - g.blk[1]);
    else if (bx < g.blk[3])
        prep_segment<32>(d, p, ref_count, L + g.off[2], g.off[3] - g.off[2], bx - g.blk[2]);
    else
        prep_segment<64>(d, p, ref_count, L + g.off[3], g.off[4] - g.off[3], bx - g.blk[3]);
}

// REFERENCED candidate arrays and the destination groups: one lane per out
// entry, a segment of SEG lanes per method (SEG >= its row length >= its
// entries); the entry's candidate index skips the method's own class.
template <int SEG>
__device__ __forceinline__ void ref_fill_segment(const DevSys &d, const ScorePlan &p, const int32_t *__restrict__ list,
                                                 int n_list, int blk) {
    const int j = threadIdx.x & (SEG - 1);
    const int seg = blk * (int)(blockDim.x / SEG) + (int)threadIdx.x / SEG;
    if (seg >= n_list) return;
    const int m = list[seg];
    const MethodPrep r = p.prep[m];
    if (j >= r.nout) return;
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    const int32_t D = p.outk[off + j];
    if (D == r.S) return;
    const int64_t pos = p.cand_off[m] + j - ((r.s_entry >= 0 && r.s_entry < j) ? 1 : 0);
    p.cm[pos] = m;
    p.ct[pos] = D;
    p.ce[pos] = (int32_t)(off + j);  // the entry's place in the out arrays (references < 2^31)
    // the destination groups of the co-access step: after the prefix sum the
    // counts are taken down again, one slot per candidate (their order within
    // a group is free)
    if (p.grouped && p.outa[off + j] > 0) p.glist[p.goff[D] + atomicSub(&p.gcnt[D], 1) - 1] = (int32_t)pos;
}

__global__ __launch_bounds__(256) void k_ref_fill(DevSys d, ScorePlan p, SegGrid g) {
    const int bx = blockIdx.x;
    const int32_t *L = p.prep_runs;
    if (bx < g.blk[1])
        ref_fill_segment<8>(d, p, L + g.off[0], g.off[1] - g.off[0], bx);
    else if (bx < g.blk[2])
        ref_fill_segment<16>(d, p, L + g.off[1], g.off[2] - g.off[1], bx - g.blk[1]);
    else if (bx < g.blk[3])
        ref_fill_segment<32>(d, p, L + g.off[2], g.off[3] - g.off[2], bx - g.blk[2]);
    else
        ref_fill_segment<64>(d, p, L + g.off[3], g.off[4] - g.off[3], bx - g.blk[3]);
}

// rows of more than 64 entries: one lane per method
__global__ __launch_bounds__(256) void k_ref_fill_long(DevSys d, ScorePlan p, const int32_t *__restrict__ list,
                                                       int n_list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_list) return;
    const int m = list[i];
    const MethodPrep r = p.prep[m];
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    int64_t pos = p.cand_off[m];
    for (int q = 0; q < r.nout; ++q) {
        const int32_t D = p.outk[off + q];
        if (D == r.S) continue;
        p.cm[pos] = m;
        p.ct[pos] = D;
        p.ce[pos] = (int32_t)(off + q);
        if (p.grouped && p.outa[off + q] > 0) p.glist[p.goff[D] + atomicSub(&p.gcnt[D], 1) - 1] = (int32_t)pos;
        ++pos;
    }
}

// candidate index of out entry q (class D) of method m, for ALL / REFERENCED
__device__ __forceinline__ int64_t cand_of(const ScorePlan &p, int m, const MethodPrep &r, int q, int32_t D) {
    if (p.mode == 1) return (int64_t)m * p.cm1 + (D < r.S ? D : D - 1);
    return p.cand_off[m] + q - ((r.s_entry >= 0 && r.s_entry < q) ? 1 : 0);
}

// Candidates whose method accesses an attribute of the destination: count per
// destination (pass 0) and scatter into the per-destination lists (pass 1).
__global__ __launch_bounds__(256) void k_a9_group(DevSys d, ScorePlan p, int pass) {
    if (p.mode == 0) {
        const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (k >= p.n_cand) return;
        const int m = p.cm[k], T = p.ct[k];
        const MethodPrep r = p.prep[m];
        const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
        const int e = lower_bound_i32(p.outk + off, r.nout, T);
        if (!(e < r.nout && p.outk[off + e] == T && p.outa[off + e] > 0)) return;
        if (pass == 0) p.gslot[k] = atomicAdd(&p.gcnt[T], 1);
        else p.glist[p.goff[T] + p.gslot[k]] = (int32_t)k;
        return;
    }
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    const MethodPrep r = p.prep[m];
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    for (int q = 0; q < r.nout; ++q) {
        const int32_t D = p.outk[off + q];
        if (D == r.S || p.outa[off + q] == 0) continue;
        const int64_t k = cand_of(p, m, r, q, D);
        if (pass == 0) p.gslot[k] = atomicAdd(&p.gcnt[D], 1);
        else p.glist[p.goff[D] + p.gslot[k]] = (int32_t)k;
    }
}

__device__ __forceinline__ int cand_method(const ScorePlan &p, int64_t k) {
    return p.mode == 1 ? (int)(k / p.cm1) : p.cm[k];
}

// One wave per destination class T: h_T(m) for its listed candidates, as column
// counts of B_T X^T on INT8 MFMA tiles (co_tile; rows: methods of T, columns: 16
// candidates). The own-attribute masks of T's methods are staged in the wave's
// own LDS region (A9_WAVE_LDS at a time; a wave's LDS accesses complete in
// issue order, so it reads its region without a barrier); rows past the class
// have zero masks and count nothing. Classes with more than 64 own attributes
// take their further k-blocks from the access rows.
constexpr int A9_WAVE_LDS = 512;

__global__ __launch_bounds__(256) void k_a9(DevSys d, ScorePlan p) {
    __shared__ uint64_t s_mask[4][A9_WAVE_LDS];
    const int wv = threadIdx.x >> 6;
    const int T = blockIdx.x * 4 + wv;
    if (T >= d.c) return;
    const int64_t gb = p.goff[T];
    const int cnt = (int)(p.goff[T + 1] - gb);
    if (cnt == 0) return;
    uint64_t *sm = s_mask[wv];
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int mb = d.mem_off[T];
    const int n = d.mem_end[T] - mb;
    const int nkb = (d.acnt[T] + 63) >> 6;
    const bool k32 = d.acnt[T] <= 32;  // every own-attribute rank below 32
    for (int c0 = 0; c0 < max(n, 1); c0 += A9_WAVE_LDS) {  // once at least: an empty class writes h = 0
        const int cn = min(A9_WAVE_LDS, n - c0);
        const int ntc = (cn + 15) >> 4;
        for (int j = lane; j < ntc * 16; j += WAVE) sm[j] = j < cn ? p.own_mask[d.mem_idx[mb + c0 + j]] : 0ull;
        __builtin_amdgcn_wave_barrier();
        for (int g0 = 0; g0 < cnt; g0 += 16) {
            const int kc = g0 + r < cnt ? p.glist[gb + g0 + r] : -1;
            const int mc = kc >= 0 ? cand_method(p, kc) : -1;
            const uint64_t b0 = attr_bits(d, mc, T, 0);
            int h = 0;
            for (int ti = 0; ti < ntc; ++ti) {
                v4i acc = co_tile(sm[ti * 16 + r], b0, grp, k32);
                if (nkb > 1) {
                    const int ri = c0 + ti * 16 + r;
                    const int mi = ri < n ? d.mem_idx[mb + ri] : -1;
                    for (int kb = 1; kb < nkb; ++kb)
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(attr_operand(d, mi, T, kb, grp),
                                                                    attr_operand(d, mc, T, kb, grp), acc, 0, 0, 0);
                }
                // acc[q] = G[4*grp + q][r]: row = method of T, column = candidate r
#pragma unroll
                for (int q = 0; q < 4; ++q) h += acc[q] > 0 ? 1 : 0;
            }
            h += __shfl_xor(h, 16, WAVE);
            h += __shfl_xor(h, 32, WAVE);
            if (grp == 0 && kc >= 0) p.hval[kc] = (c0 == 0 ? 0 : p.hval[kc]) + h;
        }
        __builtin_amdgcn_wave_barrier();  // every read of this chunk before the next one is staged
    }
}

__device__ __forceinline__ void hs_after(int64_t n, int64_t a, int64_t U, int64_t &num, int64_t &den) {
    if (n * a == 0) {
        num = 0;
        den = 1;
    } else {
        den = n * a;
        num = den - U;
    }
}

__device__ __forceinline__ int64_t own_uses(const ClassAgg &c) {
    return ((int64_t)c.n * c.a == 0) ? 0 : c.hs_den - c.hs_num;
}

// sign of num1/den1 - num0/den0 (denominators > 0)
__device__ __forceinline__ int frac_cmp(int64_t num0, int64_t den0, int64_t num1, int64_t den1) {
    __int128 l = (__int128)num1 * den0, r = (__int128)num0 * den1;
    return (l > r) - (l < r);
}

__device__ __forceinline__ int eval_keep(const MoveRec &r, const ClassAgg &cS, const ClassAgg &cT, uint32_t mask,
                                         int rule) {
    const int hsS = frac_cmp(cS.hs_num, cS.hs_den, r.hs_num_src, r.hs_den_src);
    const int hsT = frac_cmp(cT.hs_num, cT.hs_den, r.hs_num_dst, r.hs_den_dst);
    if (rule == 1) {  // PAPER_LCOM
        int keep = 1;
        if (mask & 2u) keep &= (r.d_lcom_src < 0) & (r.d_lcom_dst < 0);
        if (mask & 4u) keep &= (hsS < 0) & (hsT < 0);
        return keep;
    }
    if (rule == 2) return (r.d_cbo_src < 0) & (r.d_cbo_dst <= 0) & (r.n_caller_worse == 0);  // PAPER_CBO
    int up = 0, down = 0;  // PARETO
    if (mask & 1u) {
        up |= (r.d_cbo_src > 0) | (r.d_cbo_dst > 0) | (r.n_caller_worse > 0);
        down |= (r.d_cbo_src < 0) | (r.d_cbo_dst < 0) | (r.n_caller_better > 0);
    }
    if (mask & 2u) {
        up |= (r.d_lcom_src > 0) | (r.d_lcom_dst > 0);
        down |= (r.d_lcom_src < 0) | (r.d_lcom_dst < 0);
    }
    if (mask & 4u) {
        up |= (hsS > 0) | (hsT > 0);
        down |= (hsS < 0) | (hsT < 0);
    }
    if (mask & 8u) {
        up |= (r.d_rfc_src > 0) | (r.d_rfc_dst > 0);
        down |= (r.d_rfc_src < 0) | (r.d_rfc_dst < 0);
    }
    return !up && down;
}

// RFC deltas of S and T: T starts to respond with m if no method of T calls
// it, and with each callee outside T that none of T's methods calls
__device__ __forceinline__ void rfc_terms(const DevSys &d, const ScorePlan &p, int m, int S, int T, int drs_prep,
                                          MoveRec &rec) {
    rec.d_rfc_src = drs_prep != SRC_LAZY ? drs_prep : src_rfc(d, p, m, S);
    const MapHdr hcT = p.cnt.hdr[T];
    int drt = map_get_h(hcT, p.cnt.keys, p.cnt.vals, m) == 0 ? 1 : 0;
    const int cb = d.call_off[m], ce = d.call_off[m + 1];
    for (int q0 = cb; q0 < ce; q0 += 4) {
        int32_t key[4];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u;
            key[u] = q < ce ? d.call_idx[q] : -2;
            use[u] = q < ce && key[u] != m;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) use[u] = use[u] && d.owner[key[u]] != T;
        drt += tab_absent4(hcT, p.cnt.keys, key, use);
    }
    rec.d_rfc_dst = drt;
}

// Rule outcome known from part of the deltas (lower is better for every metric):
// a keep_only pass drops a candidate as soon as its outcome is settled, so most
// candidates never reach the table probes of the later stages.
//   stage A  LCOM pair count and LCOM_HS of S and T (no probes)
//   stage B  CBO of S and T
//   stage C  RFC of S and T
//   stage D  CBO of the caller classes
// PARETO rejects on any masked delta > 0; PAPER_LCOM is decided by stage A;
// PAPER_CBO by stages B and D.
__device__ __forceinline__ bool reject_lcom(const MoveRec &r, int hsS, int hsT, uint32_t mask, int rule) {
    if (rule == 1) {
        bool keep = true;
        if (mask & 2u) keep = keep && r.d_lcom_src < 0 && r.d_lcom_dst < 0;
        if (mask & 4u) keep = keep && hsS < 0 && hsT < 0;
        return !keep;
    }
    if (rule == 2) return false;
    return ((mask & 2u) && (r.d_lcom_src > 0 || r.d_lcom_dst > 0)) || ((mask & 4u) && (hsS > 0 || hsT > 0));
}

__device__ __forceinline__ bool reject_cbo(const MoveRec &r, uint32_t mask, int rule) {
    if (rule == 1) return false;
    if (rule == 2) return r.d_cbo_src >= 0 || r.d_cbo_dst > 0;
    return (mask & 1u) && (r.d_cbo_src > 0 || r.d_cbo_dst > 0);
}

__device__ __forceinline__ bool reject_rfc(const MoveRec &r, uint32_t mask, int rule) {
    return rule == 0 && (mask & 8u) && (r.d_rfc_src > 0 || r.d_rfc_dst > 0);
}

// origin threshold of ranked suggestions: the origin's LCOM (P - Q) or CBO is
// above the average over the c classes, tested exactly as value * c > sum
__device__ __forceinline__ bool origin_ok(const ScorePlan &p, const ClassAgg &cS, int c) {
    if (!p.origin) return true;
    const long long v = p.origin == 1 ? (long long)(cS.p - cS.q) : (long long)cS.cbo;
    return (__int128)v * c > (__int128)*p.origin_sum;
}

// whether a worse caller class settles a rejection
__device__ __forceinline__ bool callers_decide(uint32_t mask, int rule) {
    return rule == 2 || (rule == 0 && (mask & 1u));
}

// a kept candidate joins the short kept list (its order is restored later);
// once the list is full only the overflow mark is set, so a pass that keeps
// many candidates makes at most kept_cap atomic updates of the counter
__device__ __forceinline__ void kept_append(const ScorePlan &p, int64_t k) {
    if (!p.kept_idx) return;
    if (__hip_atomic_load(p.kept_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= p.kept_cap) {
        *p.kept_over = 1;
        return;
    }
    const int slot = atomicAdd(p.kept_count, 1);
    if (slot < p.kept_cap)
        p.kept_idx[slot] = (int32_t)k;
    else
        *p.kept_over = 1;
}

// Score candidate k for a full-record pass: every delta, inline caller classes
// for short caller lists, the keep rule; long caller lists are queued for
// k_heavy. (A keep_only pass uses score_keep_wave.)
__device__ __forceinline__ void score_one(const DevSys &d, const ScorePlan &p, int64_t k) {
    // pe: place of (m, T)'s out entry in the out arrays (REFERENCED: from the
    // fill, so that its counts load beside the method's record), -1 if m does
    // not reference T, -2 while to be found
    int m, T;
    int64_t pe = -2;
    if (p.mode == 1) {  // ALL
        m = (int)(k / p.cm1);
        const int t = (int)(k - (int64_t)m * p.cm1);
        const int S0 = d.owner[m];
        T = t < S0 ? t : t + 1;
    } else {
        m = p.cm[k];
        T = p.ct[k];
        if (p.mode == 2) pe = p.ce[k];
    }
    const int hv = p.hval[k];  // h_T(m) where k_a9 wrote it (read now, used only then)
    const MethodPrep P = p.prep[m];
    const int S = P.S;
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    if (pe == -2) {
        const int e = lower_bound_i32(p.outk + off, P.nout, T);
        pe = (e < P.nout && p.outk[off + e] == T) ? off + e : -1;
    }
    const int outT = pe >= 0 ? p.outc[pe] : 0;
    const int accT = pe >= 0 ? p.outa[pe] : 0;
    const ClassAgg cS = p.cls[S], cT = p.cls[T];
    const MethodAgg ma = p.meth[m];
    const int h = accT > 0 ? hv : 0;

    MoveRec rec;
    rec.method = m;
    rec.src = S;
    rec.dst = T;
    rec.keep = 0;
    rec.pad = 0;

    const bool origin_pass = origin_ok(p, cS, d.c);

    // stage A: LCOM and LCOM_HS of S and T
    rec.d_lcom_src = lcom_pq(cS.n - 1, cS.q - ma.rnz) - lcom_pq(cS.n, cS.q);
    rec.d_lcom_dst = lcom_pq(cT.n + 1, cT.q + h) - lcom_pq(cT.n, cT.q);
    hs_after(cS.n - 1, cS.a, own_uses(cS) - ma.u_own, rec.hs_num_src, rec.hs_den_src);
    hs_after(cT.n + 1, cT.a, own_uses(cT) + accT, rec.hs_num_dst, rec.hs_den_dst);

    // stage B: CBO of S and T. The three lookups w_S(T), w_T(S) and m's
    // callers in T go in step: their headers, then their first probes, then
    // their counts are each loaded together.
    const int outS = P.s_entry >= 0 ? p.outc[off + P.s_entry] : 0;
    const MapHdr hwS = p.w.hdr[S];
    const MapHdr hwT = p.w.hdr[T];
    const MapHdr hin = p.in.hdr[m];
    uint32_t slST, slTS, slIn;
    const int32_t kST = map_probe_first(hwS, p.w.keys, T, slST);
    const int32_t kTS = map_probe_first(hwT, p.w.keys, S, slTS);
    const int32_t kIn = map_probe_first(hin, p.in.keys, T, slIn);
    const int iST = map_find_from(hwS, p.w.keys, T, slST, kST);
    const int iTS = map_find_from(hwT, p.w.keys, S, slTS, kTS);
    const int iIn = map_find_from(hin, p.in.keys, T, slIn, kIn);
    const int wST = iST >= 0 ? p.w.vals[hwS.base + iST] : 0;
    const int wTS = iTS >= 0 ? p.w.vals[hwT.base + iTS] : 0;
    const int inT = iIn >= 0 ? p.in.vals[hin.base + iIn] & 0x7fffffff : 0;
    const int inS = P.in_src;
    // classes T starts to use: m's referenced classes other than S and T absent from w_T
    int dct = 0;
    for (int q0 = 0; q0 < P.nout; q0 += 4) {
        int32_t key[4];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u;
            key[u] = q < P.nout ? p.outk[off + q] : -2;
            use[u] = q < P.nout && key[u] != S && key[u] != T;
        }
        dct += tab_absent4(hwT, p.w.keys, key, use);
    }
    dct += (wTS + outS - inT > 0 ? 1 : 0) - (wTS > 0 ? 1 : 0);
    rec.d_cbo_src = -P.lose_src + ((outT > 0 && wST == outT) ? 1 : 0) +  // k_prep's eager form here
                    ((wST - outT + inS > 0 ? 1 : 0) - (wST > 0 ? 1 : 0));
    rec.d_cbo_dst = dct;
    rec.n_caller_cls = P.nin - (inS > 0 ? 1 : 0) - (inT > 0 ? 1 : 0);

    // stage C: RFC of S and T
    rfc_terms(d, p, m, S, T, P.d_rfc_src, rec);

    // stage D: caller classes X not in {S, T}: X gains T iff T is absent from
    // w_X, loses S iff the loss flag is set; headers of four caller classes are
    // read together
    int worse = 0, better = 0;
    const bool heavy = P.nin > p.caller_light;
    const MapHdr hi = hin;
    if (heavy) {
        const int nch = (map_slots(hi) + p.heavy_chunk - 1) / p.heavy_chunk;
        const int base = atomicAdd(p.heavy_count, nch);
        for (int q = 0; q < nch; ++q) {
            if ((int64_t)base + q < p.heavy_cap) p.heavy[base + q] = make_int2((int)k, q);
            else atomicOr(p.err, ERR_HEAVY_OVERFLOW);
        }
        const int hc = atomicAdd(p.hcand_count, 1);
        if (hc < p.hcand_cap) p.hcand[hc] = (int)k;
        else atomicOr(p.err, ERR_HEAVY_OVERFLOW);
        rec.n_caller_worse = 0;
        rec.n_caller_better = 0;
        p.rec[k] = rec;  // k_heavy adds the caller classes and decides
        return;
    }
    const int ns = map_slots(hi);
    for (int j0 = 0; j0 < ns; j0 += 4) {
        int32_t X[4], v[4];
        MapHdr hx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            X[u] = j0 + u < ns ? p.in.keys[hi.base + j0 + u] : EMPTY_KEY;
            v[u] = j0 + u < ns ? p.in.vals[hi.base + j0 + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (X[u] == S || X[u] == T) X[u] = EMPTY_KEY;
            hx[u] = X[u] != EMPTY_KEY ? p.w.hdr[X[u]] : MapHdr{0, 0, MAP_EMPTY, 0};
        }
        int32_t k0[4];
        uint32_t sl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sl[u] = slot_hash(T) & ((uint32_t)hx[u].cap - 1u);
            k0[u] = hx[u].kind == MAP_TABLE ? p.w.keys[hx[u].base + sl[u]] : EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (X[u] == EMPTY_KEY) continue;
            const int gain = (hx[u].kind == MAP_TABLE && tab_has_from(hx[u], p.w.keys, T, sl[u], k0[u])) ? 0 : 1;
            const int loss = (int)((uint32_t)v[u] >> 31);
            worse += gain > loss;
            better += gain < loss;
        }
    }
    rec.n_caller_worse = worse;
    rec.n_caller_better = better;
    rec.keep = eval_keep(rec, cS, cT, p.mask, p.rule) && origin_pass;
    p.rec[k] = rec;
}

// value of lane `src` (wave-uniform) in every lane
__device__ __forceinline__ int lane_val(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ int64_t lane_val64(int64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ MapHdr lane_hdr(const MapHdr &h, int src) {
    return MapHdr{lane_val(h.base, src), lane_val(h.len, src), lane_val(h.kind, src), lane_val(h.cap, src)};
}

// The keep_only form of score_one, called by every lane of a wave (valid false
// past the candidates), with the same results. Stage A runs per lane and leaves
// about one candidate in a hundred; the loops over table entries of the later
// stages (the classes S stops using, those T starts to use, the caller classes)
// then take one surviving candidate at a time with the wave's lanes over its
// entries, instead of a few lanes looping while the rest of the wave waits.
__device__ __forceinline__ void score_keep_wave(const DevSys &d, const ScorePlan &p, int64_t k, bool valid) {
    const int lane = lane_id();
    int m = 0, T = 0, S = 0, outT = 0, accT = 0, h = 0;
    int64_t off = 0;
    MethodPrep P{};
    ClassAgg cS{}, cT{};
    MethodAgg ma{};
    MoveRec rec{};
    bool alive = valid;
    if (alive) {
        int64_t pe = -2;
        if (p.mode == 1) {  // ALL
            m = (int)(k / p.cm1);
            const int t = (int)(k - (int64_t)m * p.cm1);
            const int S0 = d.owner[m];
            T = t < S0 ? t : t + 1;
        } else {
            m = p.cm[k];
            T = p.ct[k];
            if (p.mode == 2) pe = p.ce[k];
        }
        const int hv = p.hval[k];
        P = p.prep[m];
        S = P.S;
        off = (int64_t)d.acc_off[m] + d.call_off[m];
        if (pe == -2) {
            const int e = lower_bound_i32(p.outk + off, P.nout, T);
            pe = (e < P.nout && p.outk[off + e] == T) ? off + e : -1;
        }
        outT = pe >= 0 ? p.outc[pe] : 0;
        accT = pe >= 0 ? p.outa[pe] : 0;
        cS = p.cls[S];
        cT = p.cls[T];
        ma = p.meth[m];
        h = accT > 0 ? hv : 0;
        rec.method = m;
        rec.src = S;
        rec.dst = T;
        // stage A: LCOM and LCOM_HS of S and T
        rec.d_lcom_src = lcom_pq(cS.n - 1, cS.q - ma.rnz) - lcom_pq(cS.n, cS.q);
        rec.d_lcom_dst = lcom_pq(cT.n + 1, cT.q + h) - lcom_pq(cT.n, cT.q);
        hs_after(cS.n - 1, cS.a, own_uses(cS) - ma.u_own, rec.hs_num_src, rec.hs_den_src);
        hs_after(cT.n + 1, cT.a, own_uses(cT) + accT, rec.hs_num_dst, rec.hs_den_dst);
        const int hsS = frac_cmp(cS.hs_num, cS.hs_den, rec.hs_num_src, rec.hs_den_src);
        const int hsT = frac_cmp(cT.hs_num, cT.hs_den, rec.hs_num_dst, rec.hs_den_dst);
        if (!origin_ok(p, cS, d.c) || reject_lcom(rec, hsS, hsT, p.mask, p.rule)) {
            p.flags[k] = 0;
            alive = false;
        }
    }

    // stage B: CBO of S and T; the candidate's own lookups per lane
    MapHdr hwS{0, 0, MAP_EMPTY, 0}, hwT{0, 0, MAP_EMPTY, 0}, hin{0, 0, MAP_EMPTY, 0};
    int wST = 0, wTS = 0, inT = 0, outS = 0;
    if (alive) {
        outS = P.s_entry >= 0 ? p.outc[off + P.s_entry] : 0;
        hwS = p.w.hdr[S];
        hwT = p.w.hdr[T];
        hin = p.in.hdr[m];
        uint32_t slST, slTS, slIn;
        const int32_t kST = map_probe_first(hwS, p.w.keys, T, slST);
        const int32_t kTS = map_probe_first(hwT, p.w.keys, S, slTS);
        const int32_t kIn = map_probe_first(hin, p.in.keys, T, slIn);
        const int iST = map_find_from(hwS, p.w.keys, T, slST, kST);
        const int iTS = map_find_from(hwT, p.w.keys, S, slTS, kTS);
        const int iIn = map_find_from(hin, p.in.keys, T, slIn, kIn);
        wST = iST >= 0 ? p.w.vals[hwS.base + iST] : 0;
        wTS = iTS >= 0 ? p.w.vals[hwT.base + iTS] : 0;
        inT = iIn >= 0 ? p.in.vals[hin.base + iIn] & 0x7fffffff : 0;
    }
    // over each survivor's out entries, a lane per entry: the classes S stops
    // using (w_S(D) equals m's references to D; when k_prep left it) and the
    // classes other than S and T absent from w_T
    int lose = P.lose_src, dct = 0;
    for (uint64_t todo = __ballot(alive); todo; todo &= todo - 1) {
        const int src = __ffsll((long long)todo) - 1;
        const int sS = lane_val(S, src), sT = lane_val(T, src), nout = lane_val(P.nout, src);
        const int s_entry = lane_val(P.s_entry, src);
        const bool need_lose = lane_val(P.lose_src, src) == SRC_LAZY;
        const int64_t soff = lane_val64(off, src);
        const MapHdr sw = lane_hdr(hwS, src), tw = lane_hdr(hwT, src);
        int nl = 0, na = 0;
        for (int j0 = 0; j0 < nout; j0 += WAVE) {
            const int j = j0 + lane;
            const bool in = j < nout;
            const int32_t key = in ? p.outk[soff + j] : -2;
            const int32_t cnt = in ? p.outc[soff + j] : 0;
            const bool useL = need_lose && in && j != s_entry && sw.kind == MAP_TABLE;
            const bool useD = in && key != sS && key != sT;
            uint32_t slS = 0, slT = 0;
            const int32_t kS = useL ? map_probe_first(sw, p.w.keys, key, slS) : EMPTY_KEY;
            const int32_t kT = useD && tw.kind == MAP_TABLE ? map_probe_first(tw, p.w.keys, key, slT) : EMPTY_KEY;
            const bool lost = useL && tab_get_from(sw, p.w.keys, p.w.vals, key, slS, kS) == cnt;
            const bool absent = useD && !(tw.kind == MAP_TABLE && tab_has_from(tw, p.w.keys, key, slT, kT));
            nl += __popcll(__ballot(lost));
            na += __popcll(__ballot(absent));
        }
        if (lane == src) {
            if (need_lose) lose = nl;
            dct = na;
        }
    }
    if (alive) {
        dct += (wTS + outS - inT > 0 ? 1 : 0) - (wTS > 0 ? 1 : 0);
        rec.d_cbo_src = -lose + ((outT > 0 && wST == outT) ? 1 : 0) + ((wST - outT + P.in_src > 0 ? 1 : 0) - (wST > 0 ? 1 : 0));
        rec.d_cbo_dst = dct;
        rec.n_caller_cls = P.nin - (P.in_src > 0 ? 1 : 0) - (inT > 0 ? 1 : 0);
        if (reject_cbo(rec, p.mask, p.rule)) {
            p.flags[k] = 0;
            alive = false;
        }
    }

    // stage C: RFC of S and T, per lane (read only when RFC plays a part in the
    // rule; otherwise filled for the written records)
    const bool rfc_now = (p.mask & 8u) != 0;
    if (alive && rfc_now) {
        rfc_terms(d, p, m, S, T, P.d_rfc_src, rec);
        if (reject_rfc(rec, p.mask, p.rule)) {
            p.flags[k] = 0;
            alive = false;
        }
    }

    // stage D: caller classes X not in {S, T}; long caller lists go to k_heavy
    if (alive && P.nin > p.caller_light) {
        const int nch = (map_slots(hin) + p.heavy_chunk - 1) / p.heavy_chunk;
        const int base = atomicAdd(p.heavy_count, nch);
        for (int q = 0; q < nch; ++q) {
            if ((int64_t)base + q < p.heavy_cap) p.heavy[base + q] = make_int2((int)k, q);
            else atomicOr(p.err, ERR_HEAVY_OVERFLOW);
        }
        const int hc = atomicAdd(p.hcand_count, 1);
        if (hc < p.hcand_cap) p.hcand[hc] = (int)k;
        else atomicOr(p.err, ERR_HEAVY_OVERFLOW);
        rec.n_caller_worse = 0;
        rec.n_caller_better = 0;
        if (!rfc_now) rfc_terms(d, p, m, S, T, P.d_rfc_src, rec);  // the record goes to k_heavy
        p.rec[k] = rec;
        p.flags[k] = 0;
        alive = false;
    }
    // over each survivor's caller-map slots, a lane per slot: X gains T iff T is
    // absent from w_X, loses S iff the slot's loss flag is set
    const bool stop_on_worse = callers_decide(p.mask, p.rule);
    int worse = 0, better = 0;
    for (uint64_t todo = __ballot(alive); todo; todo &= todo - 1) {
        const int src = __ffsll((long long)todo) - 1;
        const int sS = lane_val(S, src), sT = lane_val(T, src);
        const MapHdr hi = lane_hdr(hin, src);
        const int ns = map_slots(hi);
        int nw = 0, nb = 0;
        for (int j0 = 0; j0 < ns; j0 += WAVE) {
            const int j = j0 + lane;
            int32_t X = j < ns ? p.in.keys[hi.base + j] : EMPTY_KEY;
            const int32_t v = j < ns ? p.in.vals[hi.base + j] : 0;
            if (X == sS || X == sT) X = EMPTY_KEY;
            const MapHdr hx = X != EMPTY_KEY ? p.w.hdr[X] : MapHdr{0, 0, MAP_EMPTY, 0};
            uint32_t sl = 0;
            const int32_t k0 = hx.kind == MAP_TABLE ? map_probe_first(hx, p.w.keys, sT, sl) : EMPTY_KEY;
            const int gain = (hx.kind == MAP_TABLE && tab_has_from(hx, p.w.keys, sT, sl, k0)) ? 0 : 1;
            const int loss = (int)((uint32_t)v >> 31);
            nw += __popcll(__ballot(X != EMPTY_KEY && gain > loss));
            nb += __popcll(__ballot(X != EMPTY_KEY && gain < loss));
            if (stop_on_worse && nw > 0) break;  // settled (nw is the same in every lane)
        }
        if (lane == src) {
            worse = nw;
            better = nb;
        }
    }
    if (!alive) return;
    if (stop_on_worse && worse > 0) {
        p.flags[k] = 0;
        return;
    }
    rec.n_caller_worse = worse;
    rec.n_caller_better = better;
    cS = p.cls[S];  // read again rather than held through the wave loops (few candidates get here)
    cT = p.cls[T];
    if (!rfc_now) {  // the decision does not read RFC; fill it for the record if kept
        rec.d_rfc_src = rec.d_rfc_dst = 0;
        rec.keep = eval_keep(rec, cS, cT, p.mask, p.rule);
        if (rec.keep) rfc_terms(d, p, m, S, T, P.d_rfc_src, rec);
    } else {
        rec.keep = eval_keep(rec, cS, cT, p.mask, p.rule);
    }
    if (rec.keep) p.rec[k] = rec;
    p.flags[k] = rec.keep;
    if (rec.keep) kept_append(p, k);
}

// One lane per candidate, in candidate order (consecutive lanes share methods).
// KEEP: the keep_only form (a kernel of its own, so that each form has its own
// register budget).
template <bool KEEP>
__global__ __launch_bounds__(256) void k_delta(DevSys d, ScorePlan p) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (KEEP) score_keep_wave(d, p, k, k < p.n_cand);  // every lane of the wave takes part
    else if (k < p.n_cand) score_one(d, p, k);
}

// Persistent form: a fixed grid; each wave fetches chunks of delta_chunk
// candidates from a counter until none are left (every wave exits once the
// counter passes n_cand).
template <bool KEEP>
__global__ __launch_bounds__(256) void k_delta_persistent(DevSys d, ScorePlan p) {
    const int lane = threadIdx.x & 63;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)p.delta_next, (unsigned long long)p.delta_chunk);
        base = __shfl(base, 0, WAVE);
        if (base >= p.n_cand) break;
        const int64_t end = min(base + (int64_t)p.delta_chunk, p.n_cand);
        if (KEEP) {
            for (int64_t k0 = base; k0 < end; k0 += WAVE) score_keep_wave(d, p, k0 + lane, k0 + lane < end);
        } else {
            for (int64_t k = base + lane; k < end; k += WAVE) score_one(d, p, k);
        }
    }
}

// One wave per (candidate, chunk of its method's caller-class slots).
__global__ __launch_bounds__(256) void k_heavy(ScorePlan p) {
    const int lane = threadIdx.x & 63;
    int64_t count = *p.heavy_count;
    if (count > p.heavy_cap) count = p.heavy_cap;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < count; i += nw) {
        const int2 it = p.heavy[i];
        const int k = it.x, q = it.y;
        const int m = p.rec[k].method, S = p.rec[k].src, T = p.rec[k].dst;
        const MapHdr hi = p.in.hdr[m];
        const int lo = q * p.heavy_chunk;
        const int hi_ = min(map_slots(hi), lo + p.heavy_chunk);
        int worse = 0, better = 0;
        for (int j = lo + lane; j < hi_; j += WAVE) {
            const int32_t X = p.in.keys[hi.base + j];
            if (X == EMPTY_KEY || X == S || X == T) continue;
            const int gain = map_get(p.w, X, T) == 0 ? 1 : 0;
            const int loss = (int)((uint32_t)p.in.vals[hi.base + j] >> 31);
            worse += gain > loss;
            better += gain < loss;
        }
        worse = wave_sum(worse);
        better = wave_sum(better);
        if (lane == 0 && (worse | better)) {
            atomicAdd(&p.rec[k].n_caller_worse, worse);
            atomicAdd(&p.rec[k].n_caller_better, better);
        }
    }
}

__global__ __launch_bounds__(256) void k_heavy_keep(ScorePlan p) {
    int64_t count = *p.hcand_count;
    if (count > p.hcand_cap) count = p.hcand_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = p.hcand[i];
        MoveRec &r = p.rec[k];
        const ClassAgg cS = p.cls[r.src];
        const int keep = eval_keep(r, cS, p.cls[r.dst], p.mask, p.rule) && origin_ok(p, cS, p.cm1 + 1);
        r.keep = keep;
        if (p.keep_only) {
            p.flags[k] = keep;
            if (keep) kept_append(p, k);
        }
    }
}

// The short kept list in candidate order: each kept candidate's place is the
// number of kept candidates before it (indices are distinct), so one block
// writes the records in order without a scan over every candidate.
__global__ __launch_bounds__(1024) void k_kept_order(ScorePlan p, MoveRec *__restrict__ out) {
    __shared__ int32_t s_idx[KEPT_FAST_MAX];
    // an overflowed list reports a count above its capacity: the host then lays
    // the records out by the scan of the keep flags, which also gives the count
    const int64_t count = *p.kept_over ? p.kept_cap + 1 : (int64_t)*p.kept_count;
    if (threadIdx.x == 0) {
        if (p.kept_out) *p.kept_out = count;
        if (p.status_dev) {  // the last kernel of the pass: the host reads these once the stream is done
            __hip_atomic_store(p.status_dev, *p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(reinterpret_cast<long long *>(p.status_dev + 2), (long long)count, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __threadfence_system();
        }
    }
    if (count > p.kept_cap || count > p.compact_cap) return;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s_idx[i] = p.kept_idx[i];
    __syncthreads();
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const int32_t k = s_idx[i];
        int r = 0;
        for (int64_t j = 0; j < count; ++j) r += s_idx[j] < k ? 1 : 0;
        out[r] = p.rec[k];
    }
}

__global__ __launch_bounds__(256) void k_compact(ScorePlan p, MoveRec *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 && p.kept_out) *p.kept_out = p.kpos[p.n_cand];
    if (k >= p.n_cand || p.kpos[p.n_cand] > p.compact_cap) return;  // too many for the buffer: write nothing
    if (p.flags[k]) out[p.kpos[k]] = p.rec[k];
}

// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Caller classes of one move (m -> T), X not in {S, T}: X gains T iff T is
// absent from w_X, loses S iff all of X's references to S are calls to m (flag
// bit 31 of the caller map). One lane per slot of m's caller segment; marks
// flag[X] = 1 and dval[X] = the CBO change of X.
__global__ __launch_bounds__(256) void k_affected_mark(MapView in, MapView w, int m, int S, int T,
                                                       int32_t *__restrict__ flag, int32_t *__restrict__ dval) {
    const MapHdr hi = in.hdr[m];
    const int ns = map_slots(hi);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        const int32_t X = in.keys[hi.base + j];
        if (X == EMPTY_KEY || X == S || X == T) continue;
        const int32_t v = in.vals[hi.base + j];
        const int gain = map_get(w, X, T) == 0 ? 1 : 0;
        const int loss = (int)((uint32_t)v >> 31);
        flag[X] = 1;
        dval[X] = gain - loss;
    }
}

// marked classes in ascending order: class X goes to position pos[X] when that
// is below cap; n_out (if not NULL) receives the number of marked classes
__global__ __launch_bounds__(256) void k_affected_out(const int32_t *__restrict__ flag,
                                                      const int32_t *__restrict__ dval,
                                                      const int64_t *__restrict__ pos, int c, int64_t cap,
                                                      int32_t *__restrict__ cls, int32_t *__restrict__ dcbo,
                                                      int64_t *__restrict__ n_out) {
    const int X = blockIdx.x * blockDim.x + threadIdx.x;
    if (X == 0 && n_out) *n_out = pos[c];
    if (X >= c || !flag[X]) return;
    const int64_t at = pos[X];
    if (at >= cap) return;
    cls[at] = X;
    dcbo[at] = dval[X];
}

void launch_affected_mark(const ScorePlan &p, int m, int S, int T, int n_slots, int32_t *flag, int32_t *dval,
                          hipStream_t st) {
    if (n_slots <= 0) return;
    const unsigned g = std::min<unsigned>(nblk(n_slots, 256), 1024u);
    k_affected_mark<<<g, 256, 0, st>>>(p.in, p.w, m, S, T, flag, dval);
}

void launch_affected_out(const int32_t *flag, const int32_t *dval, const int64_t *pos, int c, int64_t cap,
                         int32_t *cls, int32_t *dcbo, int64_t *n_out, hipStream_t st) {
    if (c > 0) k_affected_out<<<nblk(c, 256), 256, 0, st>>>(flag, dval, pos, c, cap, cls, dcbo, n_out);
}

// the row-length groups of the method list, as block ranges of 8-, 16-, 32- and 64-lane segments
static SegGrid prep_grid(const ScorePlan &p) {
    SegGrid g;
    g.blk[0] = 0;
    for (int q = 0; q < 6; ++q) g.off[q] = p.prep_run_off[q];
    for (int q = 0; q < 4; ++q) {
        const int per_block = 256 / (8 << q);
        g.blk[q + 1] = g.blk[q] + (g.off[q + 1] - g.off[q] + per_block - 1) / per_block;
    }
    g.blk[5] = g.blk[4];
    return g;
}

void launch_prep(const DevSys &d, const ScorePlan &p, int32_t *ref_count, hipStream_t st) {
    const SegGrid g = prep_grid(p);
    if (g.blk[4] > 0) MM_TIMED(p.timer, "k_prep", st, k_prep<<<g.blk[4], 256, 0, st>>>(d, p, ref_count, g));
    const int n_long = g.off[5] - g.off[4];
    if (n_long > 0)
        MM_TIMED(p.timer, "k_prep_long", st,
                 k_prep_long<<<nblk(n_long, 128), 128, 0, st>>>(d, p, ref_count, p.prep_runs + g.off[4], n_long));
}

// The caller terms of every method's record (callers inside its class, classes
// owning a caller), from the caller maps, when k_prep left them (prep_in_late):
// then k_prep needs only the W and CNT maps and may run beside the caller-map
// phase of the metric recompute; this pass follows both.
__global__ __launch_bounds__(256) void k_prep_in(int n, MethodPrep *__restrict__ prep,
                                                 const int32_t *__restrict__ in_own,
                                                 const MapHdr *__restrict__ in_hdr) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    prep[m].in_src = in_own[m];
    prep[m].nin = in_hdr[m].len;
}

void launch_prep_in(const DevSys &d, const ScorePlan &p, hipStream_t st) {
    if (d.n > 0)
        MM_TIMED(p.timer, "k_prep_in", st, k_prep_in<<<nblk(d.n, 256), 256, 0, st>>>(d.n, p.prep, p.in_own, p.in.hdr));
}

void launch_ref_fill(const DevSys &d, const ScorePlan &p, hipStream_t st) {
    const SegGrid g = prep_grid(p);
    if (g.blk[4] > 0) MM_TIMED(p.timer, "k_ref_fill", st, k_ref_fill<<<g.blk[4], 256, 0, st>>>(d, p, g));
    const int n_long = g.off[5] - g.off[4];
    if (n_long > 0)
        MM_TIMED(p.timer, "k_ref_fill_long", st,
                 k_ref_fill_long<<<nblk(n_long, 256), 256, 0, st>>>(d, p, p.prep_runs + g.off[4], n_long));
}

void launch_score(const DevSys &d, const ScorePlan &p, ScanArea &scan, hipStream_t st) {
    KTimer *t = p.timer;
    // the work-list counters sit at gcnt[c + 2] and gcnt[c + 3]: the fill of the
    // destination counts (here, or before k_prep when grouped) clears them too
    if (p.heavy_count != p.gcnt + d.c + 2 || p.hcand_count != p.heavy_count + 1 ||
        (p.kept_count && (p.kept_count != p.gcnt + d.c + 4 || p.kept_over != p.gcnt + d.c + 5)))
        throw std::logic_error("work-list counters are not placed after the destination counts");
    if (!p.grouped) fill_i32(p.gcnt, 0, (int64_t)d.c + GCNT_TAIL, st);
    if (p.n_cand == 0) return;
    if (!p.grouped) {
        const unsigned gb = p.mode == 0 ? nblk(p.n_cand, 256) : nblk(d.n, 256);
        MM_TIMED(t, "k_a9_group", st, k_a9_group<<<gb, 256, 0, st>>>(d, p, 0));
        scan_i32(p.gcnt, p.goff, d.c, scan, st, t);
        MM_TIMED(t, "k_a9_group", st, k_a9_group<<<gb, 256, 0, st>>>(d, p, 1));
    }
    if (d.c > 0) MM_TIMED(t, "k_a9", st, k_a9<<<nblk(d.c, 4), 256, 0, st>>>(d, p));
    if (p.delta_chunk > 0) {
        fill_i32(p.delta_next, 0, 2, st);
        if (p.keep_only)
            MM_TIMED(t, "k_delta", st, k_delta_persistent<true><<<(unsigned)p.delta_grid, 256, 0, st>>>(d, p));
        else
            MM_TIMED(t, "k_delta", st, k_delta_persistent<false><<<(unsigned)p.delta_grid, 256, 0, st>>>(d, p));
    } else if (p.keep_only) {
        MM_TIMED(t, "k_delta", st, k_delta<true><<<nblk(p.n_cand, 256), 256, 0, st>>>(d, p));
    } else {
        MM_TIMED(t, "k_delta", st, k_delta<false><<<nblk(p.n_cand, 256), 256, 0, st>>>(d, p));
    }
    if (p.heavy_cap > 0) {
        int64_t blocks = std::min<int64_t>((p.heavy_cap + 3) / 4, 2048);
        MM_TIMED(t, "k_heavy", st, k_heavy<<<(unsigned)blocks, 256, 0, st>>>(p));
        blocks = std::min<int64_t>((p.hcand_cap + 255) / 256, 1024);
        MM_TIMED(t, "k_heavy_keep", st, k_heavy_keep<<<(unsigned)blocks, 256, 0, st>>>(p));
    }
}

void launch_kept_order(const ScorePlan &p, MoveRec *out, hipStream_t st) {
    if (p.kept_cap > KEPT_FAST_MAX) throw std::logic_error("kept list longer than the ordering block holds");
    MM_TIMED(p.timer, "k_kept_order", st, k_kept_order<<<1, 1024, 0, st>>>(p, out));
}

void launch_compact(const ScorePlan &p, MoveRec *out, hipStream_t st) {
    if (p.n_cand > 0) MM_TIMED(p.timer, "k_compact", st, k_compact<<<nblk(p.n_cand, 256), 256, 0, st>>>(p, out));
}

}  // namespace mm

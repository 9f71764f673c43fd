// k_metrics.hip -- gfx950 kernels computing the per-method and per-class
// metrics of Sec. II: fan-in / fan-out (Sec. II-A), CBO, both LCOM forms and RFC
// (Sec. II-B).
//
// Pipeline (all on the system's stream):
//   k_method_basic   one lane per method: fan-in, fan-out, own-attribute uses
//   k_map_build<W>   one wave per (class, partition): classes used by the class,
//                    with reference counts (CBO = number of keys)
//   k_map_build<CNT> one wave per (class, partition): methods called by the class,
//                    with the number of its methods calling each (RFC counts the
//                    keys owned by other classes)
//   k_in_small / k_map_build<IN>  callers of each method grouped by their class
//   k_coaccess       INT8 MFMA: G_C = B_C B_C^T over the class's own attributes;
//                    per method the number of other methods with G > 0 (ballot +
//                    popcount of the accumulator signs)
//   k_finalize       one wave per class: n, a, CBO, RFC, P, Q, LCOM_HS
#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

__global__ __launch_bounds__(256) void k_method_basic(DevSys d, MethodAgg *__restrict__ out) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    int S = d.owner[m];
    int u = 0;
    for (int e = d.acc_off[m]; e < d.acc_off[m + 1]; ++e) u += d.acls[d.acc_idx[e]] == S;
    MethodAgg r;
    r.fan_in = d.rc_off[m + 1] - d.rc_off[m];
    r.fan_out = d.call_off[m + 1] - d.call_off[m];
    r.u_own = u;
    r.rnz = 0;
    out[m] = r;
}

enum { KIND_W = 0, KIND_CNT = 1, KIND_IN = 2 };

// element `pos` of the combined row of method y: calls first, then accesses
template <int KIND>
__device__ __forceinline__ int32_t elem_key(const DevSys &d, int y, int pos, int ncall) {
    if (KIND == KIND_CNT) return d.call_idx[d.call_off[y] + pos];
    if (pos < ncall) return d.owner[d.call_idx[d.call_off[y] + pos]];
    return d.acls[d.acc_idx[d.acc_off[y] + pos - ncall]];
}

__device__ __forceinline__ void lds_insert(int32_t *tk, int32_t *tv, int H, int32_t key, int *err) {
    uint32_t h = slot_hash(key) & (uint32_t)(H - 1);
    for (int probe = 0; probe < H; ++probe) {
        int32_t prev = atomicCAS(&tk[h], EMPTY_KEY, key);
        if (prev == EMPTY_KEY || prev == key) {
            atomicAdd(&tv[h], 1);
            return;
        }
        h = (h + 1) & (uint32_t)(H - 1);
    }
    atomicOr(err, ERR_MAP_OVERFLOW);
}

// Group the keys of one (segment, partition) in an LDS hash table, then write
// them sorted with their counts. One wave (the whole workgroup) per item.
template <int KIND>
__global__ __launch_bounds__(64) void k_map_build(DevSys d, const int2 *__restrict__ items,
                                                  const int32_t *__restrict__ list, MapOut mo,
                                                  MapView wv, int *err) {
    __shared__ int32_t tk[MAP_HMAX];
    __shared__ int32_t tv[MAP_HMAX];
    __shared__ int32_t s_start[WAVE];
    __shared__ int32_t s_y[WAVE];
    __shared__ int32_t s_nc[WAVE];
    const int lane = threadIdx.x;
    const int it = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int2 sp = items[it];
    const int seg = sp.x, part = sp.y;
    const MapSeg g = mo.seg[seg];
    int H = 64;
    while (H < 2 * g.rcap && H < MAP_HMAX) H <<= 1;
    for (int s = lane; s < H; s += WAVE) {
        tk[s] = EMPTY_KEY;
        tv[s] = 0;
    }
    __syncthreads();

    if (KIND == KIND_IN) {
        const int m = seg;
        const int b = d.rc_off[m], e = d.rc_off[m + 1];
        for (int i = b + lane; i < e; i += WAVE) {
            int y = d.rc_idx[i];
            if (y == m) continue;
            int32_t key = d.owner[y];
            if (part_of(key, g.nparts) != part) continue;
            lds_insert(tk, tv, H, key, err);
        }
    } else {
        const int C = seg;
        const int mb = d.mem_off[C], me = d.mem_off[C + 1];
        for (int base = mb; base < me; base += WAVE) {
            int y = base + lane < me ? d.mem_idx[base + lane] : -1;
            int nc = 0, len = 0;
            if (y >= 0) {
                nc = d.call_off[y + 1] - d.call_off[y];
                len = (KIND == KIND_CNT) ? nc : nc + d.acc_off[y + 1] - d.acc_off[y];
            }
            int incl = wave_incl_scan(len);
            int total = __shfl(incl, WAVE - 1, WAVE);
            s_start[lane] = incl - len;
            s_y[lane] = y;
            s_nc[lane] = nc;
            __syncthreads();
            for (int e = lane; e < total; e += WAVE) {
                // member j: the last one whose row starts at or before e
                int lo = 0, hi = WAVE - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
                }
                // (members with empty rows never satisfy this for an element they lack)
                int j = lo;
                int key = elem_key<KIND>(d, s_y[j], e - s_start[j], s_nc[j]);
                if (KIND == KIND_W && key == C) continue;
                if (part_of(key, g.nparts) != part) continue;
                lds_insert(tk, tv, H, key, err);
            }
            __syncthreads();
        }
    }
    __syncthreads();

    // compact the occupied slots to the front (order-preserving, in place)
    int K = 0;
    for (int base = 0; base < H; base += WAVE) {
        int32_t k = tk[base + lane], v = tv[base + lane];
        bool valid = k != EMPTY_KEY;
        unsigned long long bal = __ballot(valid);
        int pos = K + __popcll(bal & ((1ull << lane) - 1ull));
        __syncthreads();
        if (valid) {
            tk[pos] = k;
            tv[pos] = v;
        }
        K += __popcll(bal);
        __syncthreads();
    }
    if (K > g.rcap) {
        if (lane == 0) atomicOr(err, ERR_MAP_OVERFLOW);
        K = g.rcap;
    }
    int Kp = 1;
    while (Kp < K) Kp <<= 1;
    for (int s = K + lane; s < Kp; s += WAVE) tk[s] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of (tk, tv) over Kp entries
    for (int k2 = 2; k2 <= Kp; k2 <<= 1) {
        for (int j = k2 >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < Kp; i += WAVE) {
                int ixj = i ^ j;
                if (ixj > i) {
                    int32_t a = tk[i], b = tk[ixj];
                    bool up = (i & k2) == 0;
                    if ((a > b) == up) {
                        tk[i] = b;
                        tk[ixj] = a;
                        int32_t t = tv[i];
                        tv[i] = tv[ixj];
                        tv[ixj] = t;
                    }
                }
            }
            __syncthreads();
        }
    }

    const int64_t off = (int64_t)g.base + (int64_t)part * g.rcap;
    int foreign = 0;
    const int S = (KIND == KIND_IN) ? d.owner[seg] : 0;
    for (int i = lane; i < K; i += WAVE) {
        int32_t key = tk[i], v = tv[i];
        if (KIND == KIND_CNT) foreign += d.owner[key] != seg;
        if (KIND == KIND_IN) {
            // the caller class X stops using S after the move iff all of its
            // references to S are calls to this method
            if (map_get(wv, key, S) == v) v |= (int32_t)0x80000000;
        }
        mo.keys[off + i] = key;
        mo.vals[off + i] = v;
    }
    if (KIND == KIND_CNT) foreign = wave_sum(foreign);
    if (lane == 0) {
        mo.plen[it] = K;
        if (KIND == KIND_CNT) mo.pforeign[it] = foreign;
    }
}

// Callers of a method grouped by class, for short caller rows: one lane per
// method, insertion sort inside the method's own output run.
__global__ __launch_bounds__(256) void k_in_small(DevSys d, MapOut mo, MapView wv) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    int b = d.rc_off[m], e = d.rc_off[m + 1];
    if (e - b == 0 || e - b > IN_SMALL) return;
    MapSeg g = mo.seg[m];
    int32_t *keys = mo.keys + g.base;
    int32_t *vals = mo.vals + g.base;
    int k = 0;
    for (int i = b; i < e; ++i) {
        int y = d.rc_idx[i];
        if (y == m) continue;
        int32_t key = d.owner[y];
        int j = k++;
        while (j > 0 && keys[j - 1] > key) {
            keys[j] = keys[j - 1];
            --j;
        }
        keys[j] = key;
    }
    int K = 0;
    const int S = d.owner[m];
    for (int i = 0; i < k;) {
        int32_t key = keys[i];
        int j = i + 1;
        while (j < k && keys[j] == key) ++j;
        int32_t v = j - i;
        if (map_get(wv, key, S) == v) v |= (int32_t)0x80000000;
        keys[K] = key;
        vals[K] = v;
        ++K;
        i = j;
    }
    if (g.nparts > 0) mo.plen[g.item0] = K;
}

// One wave per (class, row tile of 16 methods): full rows of G_C = B_C B_C^T on
// v_mfma_i32_16x16x64_i8, counting for each of the tile's methods the other
// methods of C with which it shares an own attribute.
__global__ __launch_bounds__(256) void k_coaccess(DevSys d, const int2 *__restrict__ items, int nitems,
                                                 MethodAgg *__restrict__ out) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nitems) return;
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int2 it = items[w];
    const int C = it.x, ti = it.y;
    const int mb = d.mem_off[C];
    const int n = d.mem_off[C + 1] - mb;
    const int a = d.acnt[C];
    const int nt = (n + 15) >> 4, nkb = (a + 63) >> 6;
    const int ri = ti * 16 + r;
    const int mi = ri < n ? d.mem_idx[mb + ri] : -1;
    int rowcnt = 0;
    if (nkb > 0) {
        v4i A0 = attr_operand(d, mi, C, 0, grp);
        for (int tj = 0; tj < nt; ++tj) {
            const int cj = tj * 16 + r;
            const int mj = cj < n ? d.mem_idx[mb + cj] : -1;
            v4i acc = {0, 0, 0, 0};
            for (int kb = 0; kb < nkb; ++kb) {
                v4i A = kb == 0 ? A0 : attr_operand(d, mi, C, kb, grp);
                v4i B = attr_operand(d, mj, C, kb, grp);
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, B, acc, 0, 0, 0);
            }
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

// One wave per class: n, a, CBO, RFC, P, Q, LCOM_HS.
__global__ __launch_bounds__(256) void k_finalize(DevSys d, const MethodAgg *__restrict__ meth, MapOut w,
                                                 MapOut cnt, ClassAgg *__restrict__ out) {
    const int C = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (C >= d.c) return;
    const int lane = threadIdx.x & 63;
    const int mb = d.mem_off[C], me = d.mem_off[C + 1];
    long long rs = 0, us = 0;
    for (int i = mb + lane; i < me; i += WAVE) {
        MethodAgg x = meth[d.mem_idx[i]];
        rs += x.rnz;
        us += x.u_own;
    }
    const MapSeg gw = w.seg[C], gc = cnt.seg[C];
    int cbo = 0, rfo = 0;
    for (int p = lane; p < gw.nparts; p += WAVE) cbo += w.plen[gw.item0 + p];
    for (int p = lane; p < gc.nparts; p += WAVE) rfo += cnt.pforeign[gc.item0 + p];
    rs = wave_sum64(rs);
    us = wave_sum64(us);
    cbo = wave_sum(cbo);
    rfo = wave_sum(rfo);
    if (lane == 0) {
        const int64_t n = me - mb, a = d.acnt[C];
        ClassAgg o;
        o.n = (int32_t)n;
        o.a = (int32_t)a;
        o.cbo = cbo;
        o.rfc = (int32_t)n + rfo;
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
    }
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_compute_metrics(const DevSys &d, const MetricsPlan &p, hipStream_t st) {
    if (d.n > 0) k_method_basic<<<blocks_for(d.n, 256), 256, 0, st>>>(d, p.meth);
    if (p.n_w_items > 0)
        k_map_build<KIND_W><<<p.n_w_items, 64, 0, st>>>(d, p.w_items, nullptr, p.w, MapView{}, p.err);
    if (p.n_cnt_items > 0)
        k_map_build<KIND_CNT><<<p.n_cnt_items, 64, 0, st>>>(d, p.cnt_items, nullptr, p.cnt, MapView{}, p.err);
    MapView wv{p.w.seg, p.w.plen, p.w.keys, p.w.vals};
    if (d.n > 0) k_in_small<<<blocks_for(d.n, 256), 256, 0, st>>>(d, p.in, wv);
    if (p.n_in_wave > 0)
        k_map_build<KIND_IN><<<p.n_in_wave, 64, 0, st>>>(d, p.in_items, p.in_wave_list, p.in, wv, p.err);
    if (p.n_co_items > 0) k_coaccess<<<blocks_for(p.n_co_items, 4), 256, 0, st>>>(d, p.co_items, p.n_co_items, p.meth);
    if (d.c > 0) k_finalize<<<blocks_for(d.c, 4), 256, 0, st>>>(d, p.meth, p.w, p.cnt, p.cls);
}

}  // namespace mm

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
//         share an attribute of T with m (INT8 MFMA, grouped by T).
//   HS    U_S' = U_S - |acc(m) in A_S|, U_T' = U_T + |acc(m) in A_T|.
#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

constexpr int ERR_HEAVY_OVERFLOW = 2;

__global__ __launch_bounds__(256) void k_prep(DevSys d, ScorePlan p, int32_t *__restrict__ ref_count) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    const int S = d.owner[m];
    const int cb = d.call_off[m], ce = d.call_off[m + 1];
    const int ab = d.acc_off[m], ae = d.acc_off[m + 1];
    const int64_t off = (int64_t)ab + cb;
    int32_t *ok = p.outk + off;
    int32_t *oc = p.outc + off;
    int32_t *oa = p.outa + off;
    // referenced classes, tagged call (0) / access (1), insertion-sorted
    int k = 0, self = 0;
    for (int e = cb; e < ce + (ae - ab); ++e) {
        int32_t key;
        if (e < ce) {
            int x = d.call_idx[e];
            if (x == m) { self = 1; continue; }
            key = d.owner[x] * 2;
        } else {
            key = d.acls[d.acc_idx[ab + (e - ce)]] * 2 + 1;
        }
        int j = k++;
        while (j > 0 && ok[j - 1] > key) {
            ok[j] = ok[j - 1];
            --j;
        }
        ok[j] = key;
    }
    int K = 0;
    for (int i = 0; i < k;) {
        const int32_t D = ok[i] >> 1;
        int j = i, na = 0;
        while (j < k && (ok[j] >> 1) == D) na += ok[j++] & 1;
        ok[K] = D;
        oc[K] = j - i;
        oa[K] = na;
        ++K;
        i = j;
    }
    int s_entry = -1, lose = 0;
    for (int q = 0; q < K; ++q) {
        const int32_t D = ok[q];
        if (D == S) { s_entry = q; continue; }
        lose += map_get(p.w, S, D) == oc[q];
    }
    int drs = (map_get(p.cnt, S, m) - self == 0) ? -1 : 0;
    for (int e = cb; e < ce; ++e) {
        int x = d.call_idx[e];
        if (x == m) continue;
        if (d.owner[x] != S && map_get(p.cnt, S, x) == 1) --drs;
    }
    const MapSeg gi = p.in.seg[m];
    int nin = 0;
    for (int q = 0; q < gi.nparts; ++q) nin += p.in.plen[gi.item0 + q];
    MethodPrep r;
    r.S = S;
    r.nout = K;
    r.s_entry = s_entry;
    r.lose_src = lose;
    r.d_rfc_src = drs;
    r.in_src = map_get(p.in, m, S) & 0x7fffffff;
    r.nin = nin;
    r.ncand = K - (s_entry >= 0 ? 1 : 0);
    p.prep[m] = r;
    if (ref_count) ref_count[m] = r.ncand;
}

__global__ __launch_bounds__(256) void k_ref_fill(DevSys d, ScorePlan p, int32_t *__restrict__ cm,
                                                 int32_t *__restrict__ ct, int32_t *__restrict__ ce) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    const MethodPrep r = p.prep[m];
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    int64_t pos = p.cand_off[m];
    for (int q = 0; q < r.nout; ++q) {
        const int32_t D = p.outk[off + q];
        if (D == r.S) continue;
        cm[pos] = m;
        ct[pos] = D;
        ce[pos] = q;
        ++pos;
    }
}

__device__ __forceinline__ int sgn64(long long v) { return (v > 0) - (v < 0); }

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

__global__ __launch_bounds__(256) void k_delta(DevSys d, ScorePlan p) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_cand) return;
    int m, T, e = -2;
    if (p.mode == 1) {  // ALL
        m = (int)(k / p.cm1);
        int t = (int)(k - (int64_t)m * p.cm1);
        int S0 = d.owner[m];
        T = t < S0 ? t : t + 1;
    } else {
        m = p.cand_m[k];
        T = p.cand_t[k];
        if (p.mode == 2) e = p.cand_e[k];
    }
    const MethodPrep P = p.prep[m];
    const int S = P.S;
    const int64_t off = (int64_t)d.acc_off[m] + d.call_off[m];
    if (e == -2) {
        e = lower_bound_i32(p.outk + off, P.nout, T);
        if (!(e < P.nout && p.outk[off + e] == T)) e = -1;
    }
    const int outT = e >= 0 ? p.outc[off + e] : 0;
    const int accT = e >= 0 ? p.outa[off + e] : 0;
    const int outS = P.s_entry >= 0 ? p.outc[off + P.s_entry] : 0;
    const int wST = map_get(p.w, S, T);
    const int wTS = map_get(p.w, T, S);
    const int inT = map_get(p.in, m, T) & 0x7fffffff;
    const int inS = P.in_src;

    MoveRec r;
    r.method = m;
    r.src = S;
    r.dst = T;
    r.d_cbo_src = -P.lose_src + ((outT > 0 && wST == outT) ? 1 : 0) +
                  ((wST - outT + inS > 0 ? 1 : 0) - (wST > 0 ? 1 : 0));
    int dct = (wTS + outS - inT > 0 ? 1 : 0) - (wTS > 0 ? 1 : 0);
    for (int q = 0; q < P.nout; ++q) {
        const int32_t D = p.outk[off + q];
        if (D == S || D == T) continue;
        dct += map_get(p.w, T, D) == 0;
    }
    r.d_cbo_dst = dct;
    r.d_rfc_src = P.d_rfc_src;
    int drt = map_get(p.cnt, T, m) == 0 ? 1 : 0;
    for (int q = d.call_off[m]; q < d.call_off[m + 1]; ++q) {
        const int x = d.call_idx[q];
        if (x == m) continue;
        if (d.owner[x] != T && map_get(p.cnt, T, x) == 0) ++drt;
    }
    r.d_rfc_dst = drt;

    const ClassAgg cS = p.cls[S], cT = p.cls[T];
    const MethodAgg mm_ = p.meth[m];
    r.d_lcom_src = lcom_pq(cS.n - 1, cS.q - mm_.rnz) - lcom_pq(cS.n, cS.q);
    r.d_lcom_dst = lcom_pq(cT.n + 1, cT.q) - lcom_pq(cT.n, cT.q);  // h_T(m) added below if > 0
    hs_after(cS.n - 1, cS.a, own_uses(cS) - mm_.u_own, r.hs_num_src, r.hs_den_src);
    hs_after(cT.n + 1, cT.a, own_uses(cT) + accT, r.hs_num_dst, r.hs_den_dst);

    r.n_caller_cls = P.nin - (inS > 0 ? 1 : 0) - (inT > 0 ? 1 : 0);
    int worse = 0, better = 0;
    const MapSeg gi = p.in.seg[m];
    if (P.nin <= CALLER_LIGHT) {
        for (int q = 0; q < gi.nparts; ++q) {
            const int len = p.in.plen[gi.item0 + q];
            const int64_t b = (int64_t)gi.base + (int64_t)q * gi.rcap;
            for (int j = 0; j < len; ++j) {
                const int32_t X = p.in.keys[b + j];
                if (X == S || X == T) continue;
                const int gain = map_get(p.w, X, T) == 0 ? 1 : 0;
                const int loss = (int)((uint32_t)p.in.vals[b + j] >> 31);
                worse += gain > loss;
                better += gain < loss;
            }
        }
    } else {
        const int base = atomicAdd(p.heavy_count, gi.nparts);
        for (int q = 0; q < gi.nparts; ++q) {
            if ((int64_t)base + q < p.heavy_cap) p.heavy[base + q] = make_int2((int)k, q);
            else atomicOr(p.err, ERR_HEAVY_OVERFLOW);
        }
    }
    r.n_caller_worse = worse;
    r.n_caller_better = better;
    r.keep = 0;
    r.pad = 0;
    p.rec[k] = r;
    p.gslot[k] = accT > 0 ? atomicAdd(&p.gcnt[T], 1) : -1;
}

__global__ __launch_bounds__(256) void k_a9_scatter(ScorePlan p) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_cand) return;
    const int s = p.gslot[k];
    if (s < 0) return;
    p.glist[p.goff[p.rec[k].dst] + s] = (int32_t)k;
}

// One wave per destination class T: h_T(m) for its candidates that access an
// attribute of T, as column counts of B_T X^T on v_mfma_i32_16x16x64_i8 (rows:
// T's methods, columns: 16 candidates).
__global__ __launch_bounds__(256) void k_a9(DevSys d, ScorePlan p) {
    const int T = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (T >= d.c) return;
    const int64_t gb = p.goff[T];
    const int cnt = (int)(p.goff[T + 1] - gb);
    if (cnt == 0) return;
    const int lane = threadIdx.x & 63, r = lane & 15, grp = lane >> 4;
    const int mb = d.mem_off[T];
    const int n = d.mem_off[T + 1] - mb;
    const int nt = (n + 15) >> 4, nkb = (d.acnt[T] + 63) >> 6;
    const ClassAgg cT = p.cls[T];
    for (int c0 = 0; c0 < cnt; c0 += 16) {
        const int kc = c0 + r < cnt ? p.glist[gb + c0 + r] : -1;
        const int mc = kc >= 0 ? p.rec[kc].method : -1;
        int h = 0;
        for (int ti = 0; ti < nt; ++ti) {
            const int ri = ti * 16 + r;
            const int mi = ri < n ? d.mem_idx[mb + ri] : -1;
            v4i acc = {0, 0, 0, 0};
            for (int kb = 0; kb < nkb; ++kb) {
                v4i A = attr_operand(d, mi, T, kb, grp);
                v4i B = attr_operand(d, mc, T, kb, grp);
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, B, acc, 0, 0, 0);
            }
            // acc[q] = G[4*grp + q][r]: row = method of T, column = candidate r
#pragma unroll
            for (int q = 0; q < 4; ++q) h += (ti * 16 + 4 * grp + q < n) && acc[q] > 0;
        }
        h += __shfl_xor(h, 16, WAVE);
        h += __shfl_xor(h, 32, WAVE);
        if (grp == 0 && kc >= 0) p.rec[kc].d_lcom_dst = lcom_pq(cT.n + 1, cT.q + h) - lcom_pq(cT.n, cT.q);
    }
}

// One wave per (candidate, partition of its method's caller classes).
__global__ __launch_bounds__(256) void k_heavy(ScorePlan p) {
    const int lane = threadIdx.x & 63;
    int64_t count = *p.heavy_count;
    if (count > p.heavy_cap) count = p.heavy_cap;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < count; i += nw) {
        const int2 it = p.heavy[i];
        const int k = it.x, q = it.y;
        const int m = p.rec[k].method, S = p.rec[k].src, T = p.rec[k].dst;
        const MapSeg gi = p.in.seg[m];
        const int len = p.in.plen[gi.item0 + q];
        const int64_t b = (int64_t)gi.base + (int64_t)q * gi.rcap;
        int worse = 0, better = 0;
        for (int j = lane; j < len; j += WAVE) {
            const int32_t X = p.in.keys[b + j];
            if (X == S || X == T) continue;
            const int gain = map_get(p.w, X, T) == 0 ? 1 : 0;
            const int loss = (int)((uint32_t)p.in.vals[b + j] >> 31);
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

// sign of num1/den1 - num0/den0 (denominators > 0)
__device__ __forceinline__ int frac_cmp(int64_t num0, int64_t den0, int64_t num1, int64_t den1) {
    __int128 l = (__int128)num1 * den0, r = (__int128)num0 * den1;
    return (l > r) - (l < r);
}

__global__ __launch_bounds__(256) void k_keep(ScorePlan p, int keep_only) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_cand) return;
    MoveRec &r = p.rec[k];
    const ClassAgg cS = p.cls[r.src], cT = p.cls[r.dst];
    const int hsS = frac_cmp(cS.hs_num, cS.hs_den, r.hs_num_src, r.hs_den_src);
    const int hsT = frac_cmp(cT.hs_num, cT.hs_den, r.hs_num_dst, r.hs_den_dst);
    int keep;
    if (p.rule == 1) {  // PAPER_LCOM
        keep = 1;
        if (p.mask & 2u) keep &= (r.d_lcom_src < 0) & (r.d_lcom_dst < 0);
        if (p.mask & 4u) keep &= (hsS < 0) & (hsT < 0);
    } else if (p.rule == 2) {  // PAPER_CBO
        keep = (r.d_cbo_src < 0) & (r.d_cbo_dst <= 0) & (r.n_caller_worse == 0);
    } else {  // PARETO
        int up = 0, down = 0;
        if (p.mask & 1u) {
            up |= (r.d_cbo_src > 0) | (r.d_cbo_dst > 0) | (r.n_caller_worse > 0);
            down |= (r.d_cbo_src < 0) | (r.d_cbo_dst < 0) | (r.n_caller_better > 0);
        }
        if (p.mask & 2u) {
            up |= (r.d_lcom_src > 0) | (r.d_lcom_dst > 0);
            down |= (r.d_lcom_src < 0) | (r.d_lcom_dst < 0);
        }
        if (p.mask & 4u) {
            up |= (hsS > 0) | (hsT > 0);
            down |= (hsS < 0) | (hsT < 0);
        }
        if (p.mask & 8u) {
            up |= (r.d_rfc_src > 0) | (r.d_rfc_dst > 0);
            down |= (r.d_rfc_src < 0) | (r.d_rfc_dst < 0);
        }
        keep = !up && down;
    }
    r.keep = keep;
    if (keep_only) p.flags[k] = keep;
}

__global__ __launch_bounds__(256) void k_compact(ScorePlan p, MoveRec *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_cand) return;
    if (p.flags[k]) out[p.kpos[k]] = p.rec[k];
}

// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_prep(const DevSys &d, const ScorePlan &p, int32_t *ref_count, hipStream_t st) {
    if (d.n > 0) k_prep<<<nblk(d.n, 256), 256, 0, st>>>(d, p, ref_count);
}

void launch_ref_fill(const DevSys &d, const ScorePlan &p, int32_t *cm, int32_t *ct, int32_t *ce, hipStream_t st) {
    if (d.n > 0) k_ref_fill<<<nblk(d.n, 256), 256, 0, st>>>(d, p, cm, ct, ce);
}

void launch_deltas(const DevSys &d, const ScorePlan &p, int64_t *tmp, hipStream_t st) {
    fill_i32(p.gcnt, 0, (int64_t)d.c + 1, st);
    fill_i32(p.heavy_count, 0, 1, st);
    if (p.n_cand == 0) {
        scan_i32(p.gcnt, p.goff, d.c, tmp, st);
        return;
    }
    k_delta<<<nblk(p.n_cand, 256), 256, 0, st>>>(d, p);
    scan_i32(p.gcnt, p.goff, d.c, tmp, st);
    k_a9_scatter<<<nblk(p.n_cand, 256), 256, 0, st>>>(p);
    if (d.c > 0) k_a9<<<nblk(d.c, 4), 256, 0, st>>>(d, p);
    if (p.heavy_cap > 0) {
        int64_t blocks = (p.heavy_cap + 3) / 4;
        if (blocks > 4096) blocks = 4096;
        k_heavy<<<(unsigned)blocks, 256, 0, st>>>(p);
    }
}

void launch_keep(const DevSys &d, const ScorePlan &p, int keep_only, hipStream_t st) {
    (void)d;
    if (p.n_cand > 0) k_keep<<<nblk(p.n_cand, 256), 256, 0, st>>>(p, keep_only);
}

void launch_compact(const ScorePlan &p, MoveRec *out, hipStream_t st) {
    if (p.n_cand > 0) k_compact<<<nblk(p.n_cand, 256), 256, 0, st>>>(p, out);
}

}  // namespace mm

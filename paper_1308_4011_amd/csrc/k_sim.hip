// k_sim.hip -- Jaccard similarity of method pairs (Sec. II-A) and the moves it
// suggests (Sec. III-A).
//
// The properties of a method are the methods it calls and the attributes it
// accesses (its two rows, which are sets). For methods r and y, the shared count
// i(r, y) is the number of properties in both rows and the union is
// deg(r) + deg(y) - i(r, y); the similarity is i / union. Only pairs with i > 0
// matter (the others have similarity 0).
//
// i(r, .) for one row r is a sparse product: for each property of r, every other
// user of that property (the callers of a called method, the accessors of an
// accessed attribute) gains one. k_sim_rows gives each row to one workgroup
// (rows taken from an atomic ticket by a persistent grid). The workgroup adds
// into its own dense array of n counters with atomicAdd, then walks the same
// users again and claims each partner's count with atomicExch(.., 0): the first
// claim sees the full count, later ones see 0, and the array is left zeroed for
// the next row. Modes:
//   SIM_STATS  partners y > r: per union size u, the sum of i over the pairs
//              with that union, and the number of pairs with i > 0 (the exact
//              average similarity is built from these on the host)
//   SIM_COUNT  all partners y != r: a pair is high when i >= imin[u] (the host's
//              exact threshold table); count high pairs with y > r, and mark the
//              class of every high partner outside r's class in an LDS class
//              bitmap; a row with any mark also marks the classes of the methods
//              it calls (Sec. III-A's "classes holding one of the called
//              methods"); the bitmap row and its population go out
//   SIM_PAIRS  partners y > r: high pairs written in y order (an LDS bitmap over
//              the methods gives the order) at the row's offset
#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

constexpr int SIM_THREADS = 256;
constexpr int SIM_PROPS = 256;  // properties of a row staged in LDS at a time

// accessor lists of the attributes: count per attribute
__global__ __launch_bounds__(256) void k_at_count(DevSys d, int32_t *__restrict__ cnt) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    for (int e = d.acc_off[m]; e < d.acc_off[m + 1]; ++e) atomicAdd(&cnt[d.acc_idx[e]], 1);
}

// place each accessor (order within a list is arbitrary; only counts are used)
__global__ __launch_bounds__(256) void k_at_fill(DevSys d, const int64_t *__restrict__ at_off,
                                                 int32_t *__restrict__ cur, int32_t *__restrict__ at_idx) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    for (int e = d.acc_off[m]; e < d.acc_off[m + 1]; ++e) {
        const int a = d.acc_idx[e];
        at_idx[at_off[a] + atomicAdd(&cur[a], 1)] = m;
    }
}

// number of properties of each method
__global__ __launch_bounds__(256) void k_sim_deg(DevSys d, int32_t *__restrict__ deg) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n) return;
    deg[m] = (d.call_off[m + 1] - d.call_off[m]) + (d.acc_off[m + 1] - d.acc_off[m]);
}

__device__ __forceinline__ int block_excl_scan(int v, int *ws, int &total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int incl = wave_incl_scan(v);
    if (lane == WAVE - 1) ws[wid] = incl;
    __syncthreads();
    int pre = 0;
    total = 0;
    for (int w = 0; w < SIM_THREADS / WAVE; ++w) {
        if (w < wid) pre += ws[w];
        total += ws[w];
    }
    __syncthreads();
    return pre + incl - v;
}

__device__ __forceinline__ int block_sum(int v, int *ws) {
    int total;
    (void)block_excl_scan(v, ws, total);
    return total;
}

__global__ __launch_bounds__(SIM_THREADS) void k_sim_rows(DevSys d, SimPlan p) {
    __shared__ int32_t s_start[SIM_PROPS + 1];
    __shared__ int32_t s_base[SIM_PROPS];
    __shared__ int32_t s_kind[SIM_PROPS];
    __shared__ unsigned long long s_hist[SIM_HIST];
    __shared__ uint32_t s_bits[SIM_BITS_WORDS];
    __shared__ int s_ws[SIM_THREADS / WAVE];
    __shared__ int s_row, s_any;
    const int tid = threadIdx.x;
    int32_t *dense = p.dense + (int64_t)blockIdx.x * d.n;
    int32_t *cnt2 = p.cnt2 ? p.cnt2 + (int64_t)blockIdx.x * d.n : nullptr;
    for (int i = tid; i < SIM_HIST; i += SIM_THREADS) s_hist[i] = 0;
    for (int i = tid; i < SIM_BITS_WORDS; i += SIM_THREADS) s_bits[i] = 0;
    if (tid == 0) s_any = 0;
    unsigned long long nnz = 0;
    const bool upper_only = p.mode != SIM_COUNT;
    __syncthreads();
    while (true) {
        if (tid == 0) s_row = atomicAdd(p.ticket, 1);
        __syncthreads();
        const int r = s_row;
        __syncthreads();
        if (r >= d.n) break;  // every workgroup ends once the tickets pass n
        const int cb = d.call_off[r], nc = d.call_off[r + 1] - cb;
        const int ab = d.acc_off[r], P = nc + (d.acc_off[r + 1] - ab);
        const int S = d.owner[r];
        int pairs = 0;
        for (int phase = 0; phase < 2; ++phase) {
            for (int j0 = 0; j0 < P; j0 += SIM_PROPS) {
                const int j = j0 + tid;
                int len = 0, base = 0, kind = 0;
                if (tid < SIM_PROPS && j < P) {
                    if (j < nc) {
                        const int x = d.call_idx[cb + j];
                        base = d.rc_off[x];
                        len = d.rc_off[x + 1] - base;
                    } else {
                        const int a = d.acc_idx[ab + j - nc];
                        base = (int)p.at_off[a];
                        len = (int)(p.at_off[a + 1] - p.at_off[a]);
                        kind = 1;
                    }
                }
                int T;
                const int start = block_excl_scan(len, s_ws, T);
                if (tid < SIM_PROPS) {
                    s_start[tid] = start;
                    s_base[tid] = base;
                    s_kind[tid] = kind;
                }
                const int nj = min(SIM_PROPS, P - j0);
                __syncthreads();
                for (int e = tid; e < T; e += SIM_THREADS) {
                    int lo = 0, hi = nj - 1;  // last property whose users start at or before e
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    const int off = s_base[lo] + e - s_start[lo];
                    const int y = s_kind[lo] ? p.at_idx[off] : d.rc_idx[off];
                    if (y == r || (upper_only && y < r)) continue;
                    if (phase == 0) {
                        atomicAdd(&dense[y], 1);
                        continue;
                    }
                    const int c = atomicExch(&dense[y], 0);
                    if (c == 0) continue;
                    const int u = P + p.deg[y] - c;
                    if (p.mode == SIM_STATS) {
                        if (u < SIM_HIST) atomicAdd(&s_hist[u], (unsigned long long)c);
                        else atomicAdd(&p.hist[u], (unsigned long long)c);
                        ++nnz;
                    } else if (c >= p.imin[u]) {
                        if (p.mode == SIM_COUNT) {
                            pairs += y > r;
                            const int Ty = d.owner[y];
                            if (Ty != S) {
                                atomicOr(&s_bits[Ty >> 5], 1u << (Ty & 31));
                                s_any = 1;
                            }
                        } else {
                            atomicOr(&s_bits[y >> 5], 1u << (y & 31));
                            cnt2[y] = c;
                        }
                    }
                }
                __syncthreads();
            }
            if (phase == 0) __threadfence();  // every add lands before the claims start
            __syncthreads();
        }
        if (p.mode == SIM_COUNT) {
            const int total_pairs = block_sum(pairs, s_ws);
            if (tid == 0) p.row_pairs[r] = total_pairs;
            const bool any = s_any != 0;
            if (any) {
                for (int q = tid; q < nc; q += SIM_THREADS) {
                    const int Tx = d.owner[d.call_idx[cb + q]];
                    if (Tx != S) atomicOr(&s_bits[Tx >> 5], 1u << (Tx & 31));
                }
            }
            __syncthreads();
            int pop = 0;
            if (any) {
                uint32_t *row = p.cand_bits + (int64_t)r * p.cw;
                for (int w = tid; w < p.cw; w += SIM_THREADS) {
                    const uint32_t v = s_bits[w];
                    row[w] = v;
                    pop += __popc(v);
                    s_bits[w] = 0;
                }
            }
            const int total = block_sum(pop, s_ws);
            if (tid == 0) {
                p.row_cands[r] = total;
                s_any = 0;
            }
            __syncthreads();
        } else if (p.mode == SIM_PAIRS) {
            // partners in ascending order: rounds of SIM_THREADS bitmap words
            int64_t out = p.pair_off[r];
            const int nw = (d.n + 31) >> 5;
            for (int w0 = (r + 1) >> 5; w0 < nw; w0 += SIM_THREADS) {
                const int w = w0 + tid;
                const uint32_t v = w < nw ? s_bits[w] : 0u;
                int total;
                const int rank = block_excl_scan(__popc(v), s_ws, total);
                if (total == 0) continue;
                uint32_t bits = v;
                int k = 0;
                while (bits) {
                    const int b = __ffs(bits) - 1;
                    bits &= bits - 1;
                    const int y = w * 32 + b;
                    const int c = cnt2[y];
                    if (out + rank + k < p.out_cap) p.pairs[out + rank + k] = make_int4(r, y, c, P + p.deg[y] - c);
                    ++k;
                }
                if (w < nw) s_bits[w] = 0;
                out += total;
            }
            __syncthreads();
        }
    }
    if (p.mode == SIM_STATS) {
        for (int i = tid; i < SIM_HIST; i += SIM_THREADS)
            if (s_hist[i]) atomicAdd(&p.hist[i], s_hist[i]);
        const long long t = wave_sum64((long long)nnz);
        if ((tid & (WAVE - 1)) == 0 && t) atomicAdd(p.nnz, (unsigned long long)t);
    }
}

// similarity-driven candidates in (method, class) order: one wave per method,
// bitmap words spread over the lanes
__global__ __launch_bounds__(256) void k_sim_emit(DevSys d, SimPlan p, const int64_t *__restrict__ cand_off,
                                                  int32_t *__restrict__ cm, int32_t *__restrict__ ct) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int r = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (r >= d.n || p.row_cands[r] == 0) return;
    const uint32_t *row = p.cand_bits + (int64_t)r * p.cw;
    int64_t out = cand_off[r];
    for (int w0 = 0; w0 < p.cw; w0 += WAVE) {
        const int w = w0 + lane;
        const uint32_t v = w < p.cw ? row[w] : 0u;
        const int pc = __popc(v);
        const int incl = wave_incl_scan(pc);
        const int total = __shfl(incl, WAVE - 1, WAVE);
        uint32_t bits = v;
        int k = incl - pc;
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            if (out + k < p.out_cap) {
                cm[out + k] = r;
                ct[out + k] = w * 32 + b;
            }
            ++k;
        }
        out += total;
    }
}

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_at_build(const DevSys &d, const int64_t *at_off, int32_t *cnt_or_cur, int32_t *at_idx, int pass,
                     hipStream_t st) {
    if (d.n == 0) return;
    if (pass == 0) k_at_count<<<nblk(d.n, 256), 256, 0, st>>>(d, cnt_or_cur);
    else k_at_fill<<<nblk(d.n, 256), 256, 0, st>>>(d, at_off, cnt_or_cur, at_idx);
}

void launch_sim_deg(const DevSys &d, int32_t *deg, hipStream_t st) {
    if (d.n > 0) k_sim_deg<<<nblk(d.n, 256), 256, 0, st>>>(d, deg);
}

void launch_sim_rows(const DevSys &d, const SimPlan &p, int grid, hipStream_t st) {
    if (d.n > 0 && grid > 0) MM_TIMED(p.timer, "k_sim_rows", st, k_sim_rows<<<grid, SIM_THREADS, 0, st>>>(d, p));
}

void launch_sim_emit(const DevSys &d, const SimPlan &p, const int64_t *cand_off, int32_t *cm, int32_t *ct,
                     hipStream_t st) {
    if (d.n > 0)
        MM_TIMED(p.timer, "k_sim_emit", st,
                 k_sim_emit<<<nblk((int64_t)d.n * WAVE, 256), 256, 0, st>>>(d, p, cand_off, cm, ct));
}

}  // namespace mm

// k_rank.hip -- ranked suggestions (Sec. III-A): the class sum behind the
// above-average threshold, and the order of the kept moves (methods with the
// highest fan-out first for LCOM-driven moves, the highest fan-in + fan-out
// first for CBO-driven ones; equal keys keep candidate order, which the stable
// radix sort preserves).
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

// sum over the classes of LCOM = P - Q (which 1) or CBO (which 2)
__global__ __launch_bounds__(256) void k_class_sum(const ClassAgg *__restrict__ cls, int c, int which,
                                                  long long *__restrict__ sum) {
    long long v = 0;
    for (int C = blockIdx.x * blockDim.x + threadIdx.x; C < c; C += gridDim.x * blockDim.x)
        v += which == 1 ? (long long)(cls[C].p - cls[C].q) : (long long)cls[C].cbo;
    v = wave_sum64(v);
    if ((threadIdx.x & (WAVE - 1)) == 0 && v) atomicAdd((unsigned long long *)sum, (unsigned long long)v);
}

// key of each kept record: fan-out (kind 0) or fan-in + fan-out (kind 1), or 0
__global__ __launch_bounds__(256) void k_rank_keys(const MoveRec *__restrict__ rec, int64_t n,
                                                  const MethodAgg *__restrict__ meth, int kind,
                                                  uint32_t *__restrict__ key, int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const MethodAgg a = meth[rec[i].method];
    key[i] = kind == 0 ? (uint32_t)a.fan_out : kind == 1 ? (uint32_t)a.fan_in + (uint32_t)a.fan_out : 0u;
    idx[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_rank_gather(const MoveRec *__restrict__ rec, const int32_t *__restrict__ idx,
                                                    int64_t n, MoveRec *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = rec[idx[i]];
}

// Conflict-free subset of the ranked moves: one wave walks them in rank order
// and takes a move when none of its affected classes (origin, destination and
// the classes owning a caller of the method) is marked yet, then marks them.
// The marks live in an LDS bitmap of the classes; taken moves are written in
// order, their number to *count.
constexpr int IND_WORDS = 16384;  // classes up to 2^19

__global__ __launch_bounds__(64) void k_independent(const MoveRec *__restrict__ rec, int64_t n, MapView in, int c,
                                                   MoveRec *__restrict__ out, int64_t *__restrict__ count) {
    __shared__ uint32_t used[IND_WORDS];
    const int lane = threadIdx.x;
    const int words = (c + 31) >> 5;
    for (int w = lane; w < words; w += WAVE) used[w] = 0u;
    __syncthreads();
    int64_t taken = 0;
    for (int64_t i = 0; i < n; ++i) {
        const MoveRec r = rec[i];
        const MapHdr hi = in.hdr[r.method];
        const int ns = map_slots(hi);
        bool clash = lane == 0 && (((used[r.src >> 5] >> (r.src & 31)) & 1u) || ((used[r.dst >> 5] >> (r.dst & 31)) & 1u));
        for (int j = lane; j < ns; j += WAVE) {
            const int32_t X = in.keys[hi.base + j];
            if (X != EMPTY_KEY && ((used[X >> 5] >> (X & 31)) & 1u)) clash = true;
        }
        if (__ballot(clash)) continue;
        __syncthreads();  // every lane has read the marks before any is set
        if (lane == 0) {
            atomicOr(&used[r.src >> 5], 1u << (r.src & 31));
            atomicOr(&used[r.dst >> 5], 1u << (r.dst & 31));
            out[taken] = r;
        }
        for (int j = lane; j < ns; j += WAVE) {
            const int32_t X = in.keys[hi.base + j];
            if (X != EMPTY_KEY) atomicOr(&used[X >> 5], 1u << (X & 31));
        }
        __syncthreads();
        ++taken;
    }
    if (lane == 0) *count = taken;
}

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_independent(const MoveRec *rec, int64_t n, const MapView &in, int c, MoveRec *out, int64_t *count,
                        hipStream_t st) {
    k_independent<<<1, 64, 0, st>>>(rec, n, in, c, out, count);
}

void launch_class_sum(const ClassAgg *cls, int c, int which, long long *sum, hipStream_t st) {
    if (c > 0) k_class_sum<<<std::min<unsigned>(nblk(c, 256), 1024u), 256, 0, st>>>(cls, c, which, sum);
}

void launch_rank_keys(const MoveRec *rec, int64_t n, const MethodAgg *meth, int kind, uint32_t *key, int32_t *idx,
                      hipStream_t st) {
    if (n > 0) k_rank_keys<<<nblk(n, 256), 256, 0, st>>>(rec, n, meth, kind, key, idx);
}

void launch_rank_gather(const MoveRec *rec, const int32_t *idx, int64_t n, MoveRec *out, hipStream_t st) {
    if (n > 0) k_rank_gather<<<nblk(n, 256), 256, 0, st>>>(rec, idx, n, out);
}

// stable descending sort of (key, index); tmp == nullptr queries tmp_bytes
hipError_t rank_sort(void *tmp, size_t &tmp_bytes, const uint32_t *key_in, uint32_t *key_out, const int32_t *idx_in,
                     int32_t *idx_out, int64_t n, hipStream_t st) {
    return rocprim::radix_sort_pairs_desc(tmp, tmp_bytes, key_in, key_out, idx_in, idx_out, (size_t)n, 0,
                                          8 * (int)sizeof(uint32_t), st);
}

// stable ascending sort of (callee, caller) edge pairs; callees lie in [0, n);
// tmp == nullptr queries tmp_bytes
hipError_t callers_sort(void *tmp, size_t &tmp_bytes, const int32_t *callee_in, int32_t *callee_out,
                        const int32_t *caller_in, int32_t *caller_out, int64_t nnz, int n, hipStream_t st) {
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < (int64_t)n) ++bits;
    return rocprim::radix_sort_pairs(tmp, tmp_bytes, reinterpret_cast<const uint32_t *>(callee_in),
                                     reinterpret_cast<uint32_t *>(callee_out), caller_in, caller_out, (size_t)nnz, 0,
                                     bits, st);
}

}  // namespace mm

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

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

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

}  // namespace mm

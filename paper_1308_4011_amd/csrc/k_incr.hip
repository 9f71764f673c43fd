// k_incr.hip -- device passes of the incremental recompute after moves and
// edits: finding the caller maps a change reaches and sorting them by how their
// segments are rebuilt.
//
// The loss flag of a caller-map entry (x, X) compares w_X(class of x) with the
// callers of x in X. After a change it can differ for every method x called
// from a class X whose W table changed, when x's class is one of the W keys that
// changed. k_incr_flag_walk visits the calls of every member of those classes
// (a block per class, the member rows flattened over its lanes) and marks such
// x; k_incr_in_lists then files every marked method by the kind of its caller
// map (runs of up to 4 / 8 / 16 / 32 callers, tables grouped in LDS, hash-table
// segments built in two passes) into compact lists and clears its mark.
#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

// a block per listed class, a thread per member (rows are short: a member's
// calls are walked by its thread)
__global__ __launch_bounds__(256) void k_incr_flag_walk(DevSys d, const int32_t *__restrict__ classes,
                                                       const uint8_t *__restrict__ key_class,
                                                       uint8_t *__restrict__ mark) {
    const int X = classes[blockIdx.x];
    for (int j = d.mem_off[X] + threadIdx.x; j < d.mem_end[X]; j += blockDim.x) {
        const int y = d.mem_idx[j];
        for (int e = d.call_off[y]; e < d.call_off[y + 1]; ++e) {
            const int x = d.call_idx[e];
            if (key_class[d.owner[x]]) mark[x] = 1;
        }
    }
}

// mark the listed methods
__global__ __launch_bounds__(256) void k_incr_mark(const int32_t *__restrict__ list, int n, uint8_t *__restrict__ mark) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mark[list[i]] = 1;
}

// lists: 0 hash-table segments (k_big_stage / k_big_build), 1..4 run groups by caller count
// (up to 4, 8, 16, 32), 5 tables grouped in LDS; counts[q] their lengths (zero on
// entry)
__global__ __launch_bounds__(256) void k_incr_in_lists(DevSys d, const MapHdr *__restrict__ in_hdr,
                                                      uint8_t *__restrict__ mark, int32_t *__restrict__ lists,
                                                      int64_t stride, int32_t *__restrict__ counts) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.n || !mark[m]) return;
    mark[m] = 0;
    const MapHdr h = in_hdr[m];
    const int r = d.rc_off[m + 1] - d.rc_off[m];
    int q;
    if (h.kind == MAP_RUN) q = r <= 4 ? 1 : r <= 8 ? 2 : r <= 16 ? 3 : 4;
    else if (h.kind == MAP_TABLE) q = h.cap <= MAP_HMAX ? 5 : 0;
    else return;  // no callers: nothing stored
    lists[(int64_t)q * stride + atomicAdd(&counts[q], 1)] = m;
}

void launch_incr_flag_walk(const DevSys &d, const int32_t *classes, int n_classes, const uint8_t *key_class,
                           uint8_t *mark, hipStream_t st) {
    if (n_classes > 0) k_incr_flag_walk<<<n_classes, 256, 0, st>>>(d, classes, key_class, mark);
}

void launch_incr_mark(const int32_t *list, int n, uint8_t *mark, hipStream_t st) {
    if (n > 0) k_incr_mark<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(list, n, mark);
}

void launch_incr_in_lists(const DevSys &d, const MapHdr *in_hdr, uint8_t *mark, int32_t *lists, int64_t stride,
                          int32_t *counts, hipStream_t st) {
    if (d.n > 0) k_incr_in_lists<<<(unsigned)((d.n + 255) / 256), 256, 0, st>>>(d, in_hdr, mark, lists, stride, counts);
}

}  // namespace mm

// k_util.hip -- exclusive prefix sums (reduce, scan of block sums, scan-down)
// and fills used to lay out variable-size outputs.
#include "mm_internal.h"

namespace mm {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const T *__restrict__ in, int64_t n,
                                                             int64_t *__restrict__ tmp) {
    __shared__ long long ws[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    long long s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (k < n) s += (long long)in[k];
    }
    s = wave_sum64(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) t += ws[w];
        tmp[blockIdx.x] = t;
    }
}

// exclusive scan of tmp[0..nb) in place; tmp[nb] = total
__global__ __launch_bounds__(1024) void k_scan_top(int64_t *tmp, int64_t nb) {
    __shared__ long long ws[16];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t k = base + threadIdx.x;
        long long v = k < nb ? tmp[k] : 0;
        long long x = v;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            long long t = __shfl_up(x, d, WAVE);
            if (lane >= d) x += t;
        }
        if (lane == 63) ws[wid] = x;
        __syncthreads();
        long long pre = carry;
        for (int w = 0; w < wid; ++w) pre += ws[w];
        if (k < nb) tmp[k] = pre + x - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = pre + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) tmp[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const T *__restrict__ in, int64_t *__restrict__ out,
                                                           int64_t n, const int64_t *__restrict__ tmp,
                                                           int64_t nb) {
    __shared__ long long ws[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    long long v[SCAN_ITEMS];
    long long s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + i;
        v[i] = k < n ? (long long)in[k] : 0;
        s += v[i];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    long long x = s;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        long long t = __shfl_up(x, d, WAVE);
        if (lane >= d) x += t;
    }
    if (lane == 63) ws[wid] = x;
    __syncthreads();
    long long pre = tmp[blockIdx.x];
    for (int w = 0; w < wid; ++w) pre += ws[w];
    pre += x - s;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + i;
        if (k < n) out[k] = pre;
        pre += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tmp[nb];
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_total(int64_t *out) { out[0] = 0; }

template <typename T>
static void scan_impl(const T *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st, KTimer *t) {
    if (n == 0) {
        k_zero_total<<<1, 1, 0, st>>>(out);
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    MM_TIMED(t, "k_scan", st,
             k_scan_reduce<T><<<(unsigned)nb, SCAN_THREADS, 0, st>>>(in, n, tmp);
             k_scan_top<<<1, 1024, 0, st>>>(tmp, nb);
             k_scan_down<T><<<(unsigned)nb, SCAN_THREADS, 0, st>>>(in, out, n, tmp, nb));
}

void scan_i32(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st, KTimer *t) {
    scan_impl<int32_t>(in, out, n, tmp, st, t);
}
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st, KTimer *t) {
    scan_impl<int64_t>(in, out, n, tmp, st, t);
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n > 0) k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, v, n);
}

}  // namespace mm

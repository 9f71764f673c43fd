// k_util.hip -- exclusive prefix sums (one pass, decoupled look-back) and fills
// used to lay out variable-size outputs.
#include <stdexcept>

#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_total(int64_t *out) { out[0] = 0; }

// Single-pass exclusive scan (decoupled look-back): one launch. The work area
// holds a control word {epoch:32, tickets drawn:32}, a spare word and one
// status word per tile. A tile takes its index and the epoch from one atomic
// add on the control word, so every tile it waits for has already started; the
// tile that draws the last ticket stores the next epoch with no tickets drawn
// (every other tile has its ticket by then). Nothing the host passes changes
// from one scan to the next. Each tile publishes its own sum before looking
// back, so every wait ends. A status word packs {epoch:16, flag:2, value:46}
// (flag 1: the tile's sum, 2: the sum of everything up to and including the
// tile); a word of another epoch reads as unpublished. The host counts the
// scans since the area was cleared and clears it (zeros) when it is new and
// before the 16-bit epoch could wrap, so a word from an earlier scan never
// matches. The look-back gives up after SP_SPIN_MAX sleeps and sets an error
// bit instead of waiting on.
constexpr int SP_THREADS = 256;
constexpr int SP_ITEMS = 8;
constexpr int SP_TILE = SP_THREADS * SP_ITEMS;
constexpr int SP_SPIN_MAX = 1 << 22;
constexpr unsigned long long SP_VALUE = (1ull << 46) - 1;

int64_t scan_area_elems(int64_t n) { return 3 + (n + SP_TILE - 1) / SP_TILE; }

// one or two arrays scanned by one launch: tiles [0, nt1) take the first,
// tiles [nt1, nt1 + nt2) the second
template <typename T>
struct ScanArrays {
    const T *in1;
    int64_t *out1;
    int64_t n1, nt1;
    const T *in2;
    int64_t *out2;
    int64_t n2, nt2;
};

__device__ __forceinline__ unsigned long long sp_word(uint32_t epoch, uint32_t flag, unsigned long long v) {
    return ((unsigned long long)epoch << 48) | ((unsigned long long)flag << 46) | (v & SP_VALUE);
}

template <typename T>
__global__ __launch_bounds__(SP_THREADS) void k_scan1(ScanArrays<T> sa, unsigned long long *__restrict__ area,
                                                     int *err) {
    __shared__ long long ws[SP_THREADS / WAVE];
    __shared__ long long s_tile, s_excl;
    __shared__ unsigned long long s_epoch;
    const int64_t ntiles = sa.nt1 + sa.nt2;
    if (threadIdx.x == 0) {
        // one word holds {epoch:32, tickets drawn:32}: a single relaxed add
        // returns the tile's ticket together with the epoch it belongs to
        const unsigned long long w =
            __hip_atomic_fetch_add(&area[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t = w & 0xffffffffull, e = w >> 32;
        if (t == (unsigned long long)(ntiles - 1))  // every tile holds its ticket: next epoch, no tickets
            __hip_atomic_store(&area[0], (e + 1) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_tile = (long long)t;
        s_epoch = e;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    const uint32_t epoch = (uint32_t)(s_epoch & 0xffffu);
    // the array this tile belongs to; the look-back never leaves it
    const bool second = tile >= sa.nt1;
    const T *__restrict__ in = second ? sa.in2 : sa.in1;
    int64_t *__restrict__ out = second ? sa.out2 : sa.out1;
    const int64_t n = second ? sa.n2 : sa.n1;
    const int64_t first = second ? sa.nt1 : 0;
    const int64_t last = second ? ntiles - 1 : sa.nt1 - 1;
    if (tile < 0 || tile >= ntiles) {  // a miscounted ticket: report, never wait
        if (threadIdx.x == 0 && err) atomicOr(err, ERR_SCAN);
        return;
    }
    unsigned long long *status = area + 2;
    const int64_t b0 = (tile - first) * SP_TILE + (int64_t)threadIdx.x * SP_ITEMS;
    long long v[SP_ITEMS];
    long long sum = 0;
#pragma unroll
    for (int i = 0; i < SP_ITEMS; ++i) {
        v[i] = b0 + i < n ? (long long)in[b0 + i] : 0;
        sum += v[i];
    }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    long long x = sum;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const long long t = __shfl_up(x, d, WAVE);
        if (lane >= d) x += t;
    }
    if (lane == WAVE - 1) ws[wid] = x;
    __syncthreads();
    long long pre = 0, total = 0;
    for (int w = 0; w < SP_THREADS / WAVE; ++w) {
        if (w < wid) pre += ws[w];
        total += ws[w];
    }
    if (wid == 0) {
        // wave 0: publish the tile's sum, then look back 64 predecessors at a
        // time (lane l reads tile j_hi - l); the nearest full prefix ends the walk
        long long excl = 0;
        if (tile == first) {
            if (lane == 0)
                __hip_atomic_store(&status[tile], sp_word(epoch, 2, total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&status[tile], sp_word(epoch, 1, total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int64_t j_hi = tile - 1;
            int spins = 0;
            while (true) {
                const int64_t j = j_hi - lane;
                unsigned long long w = sp_word(epoch, 2, 0);  // before the array's first tile: an empty prefix
                if (j >= first) w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t flag = (uint32_t)(w >> 46) & 3u;
                const bool ready = (uint32_t)(w >> 48) == epoch && flag != 0;
                const unsigned long long unready = __ballot(!ready);
                const unsigned long long prefix = __ballot(ready && flag == 2);
                const int pl = prefix ? __ffsll((long long)prefix) - 1 : WAVE;  // nearest prefix lane
                const unsigned long long needed = pl >= WAVE - 1 ? ~0ull : ((2ull << pl) - 1);
                if (unready & needed) {  // a tile up to the nearest prefix has not published yet
                    if (++spins > SP_SPIN_MAX) {
                        if (lane == 0 && err) atomicOr(err, ERR_SCAN);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                long long val = lane <= pl ? (long long)(w & SP_VALUE) : 0;
#pragma unroll
                for (int d = WAVE / 2; d >= 1; d >>= 1) val += __shfl_xor(val, d, WAVE);
                excl += val;
                if (pl < WAVE) break;
                j_hi -= WAVE;
            }
            if (lane == 0)
                __hip_atomic_store(&status[tile], sp_word(epoch, 2, excl + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    long long run = s_excl + pre + x - sum;
#pragma unroll
    for (int i = 0; i < SP_ITEMS; ++i) {
        if (b0 + i < n) out[b0 + i] = run;
        run += v[i];
    }
    if (tile == last && threadIdx.x == 0) out[n] = s_excl + total;
}

template <typename T>
static void scan_impl(const T *in, int64_t *out, int64_t n, const T *in2, int64_t *out2, int64_t n2, ScanArea &a,
                      hipStream_t st, KTimer *t) {
    if (n == 0 && n2 == 0) {
        k_zero_total<<<1, 1, 0, st>>>(out);
        if (out2) k_zero_total<<<1, 1, 0, st>>>(out2);
        return;
    }
    if (n == 0 || n2 == 0) {  // one array left to scan
        if (n == 0) {
            k_zero_total<<<1, 1, 0, st>>>(out);
            in = in2;
            out = out2;
            n = n2;
        } else if (out2) {
            k_zero_total<<<1, 1, 0, st>>>(out2);
        }
        in2 = nullptr;
        out2 = nullptr;
        n2 = 0;
    }
    ScanArrays<T> sa{in, out, n, (n + SP_TILE - 1) / SP_TILE, in2, out2, n2, (n2 + SP_TILE - 1) / SP_TILE};
    const int64_t ntiles = sa.nt1 + sa.nt2;
    if (ntiles + 2 > a.cap_words) throw std::logic_error("scan area too small");
    if (a.need_clear || a.scans >= SCAN_EPOCHS) {
        // new area or epoch wrap ahead: clear the counter, the epoch and every status word
        const int64_t words = a.cap_words;
        k_fill_i32<<<(unsigned)((2 * words + 255) / 256), 256, 0, st>>>((int32_t *)a.dev, 0, 2 * words);
        a.need_clear = false;
        a.scans = 0;
    }
    ++a.scans;
    MM_TIMED(t, "k_scan", st,
             k_scan1<T><<<(unsigned)ntiles, SP_THREADS, 0, st>>>(sa, (unsigned long long *)a.dev, a.err));
}

void scan_i32(const int32_t *in, int64_t *out, int64_t n, ScanArea &a, hipStream_t st, KTimer *t) {
    scan_impl<int32_t>(in, out, n, nullptr, nullptr, 0, a, st, t);
}
void scan2_i32(const int32_t *in1, int64_t *out1, int64_t n1, const int32_t *in2, int64_t *out2, int64_t n2,
               ScanArea &a, hipStream_t st, KTimer *t) {
    scan_impl<int32_t>(in1, out1, n1, in2, out2, n2, a, st, t);
}
void scan_i64(const int64_t *in, int64_t *out, int64_t n, ScanArea &a, hipStream_t st, KTimer *t) {
    scan_impl<int64_t>(in, out, n, nullptr, nullptr, 0, a, st, t);
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n > 0) k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, v, n);
}

}  // namespace mm

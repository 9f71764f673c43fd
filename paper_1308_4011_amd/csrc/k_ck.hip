// k_ck.hip -- the rest of the Chidamber-Kemerer suite that Sec. II-B names
// beside CBO, RFC and LCOM: WMC (sum of the complexity weights of a class's
// methods), NOC (immediate subclasses) and DIT (proper ancestors), over a class
// hierarchy (parent[c], -1 = no parent in the system) and method weights.
//
// NOC and DIT depend on the hierarchy only, so they are computed once when the
// hierarchy is set: NOC by one atomic increment per class with a parent, DIT by
// pointer jumping (each round every class adds the depth already counted at its
// current ancestor and jumps to that ancestor's ancestor, so after r rounds a
// class has climbed min(2^r, its depth) steps). WMC follows the membership,
// which moves and edits change, so it is summed per class on every call.
#include <utility>

#include "mm_dev.h"
#include "mm_internal.h"

namespace mm {

static inline unsigned ck_blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// anc = parent, dep = 1 for a class with a parent; noc (zero on entry) counts
// each class's children
__global__ __launch_bounds__(256) void k_ck_init(const int32_t *__restrict__ parent, int c, int32_t *__restrict__ noc,
                                                 int32_t *__restrict__ anc, int32_t *__restrict__ dep) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= c) return;
    const int32_t p = parent[C];
    anc[C] = p;
    dep[C] = p >= 0 ? 1 : 0;
    if (p >= 0) atomicAdd(&noc[p], 1);
}

// one pointer-jumping round: out = in advanced by the ancestor's own progress
__global__ __launch_bounds__(256) void k_ck_jump(const int32_t *__restrict__ anc_in, const int32_t *__restrict__ dep_in,
                                                 int c, int32_t *__restrict__ anc_out, int32_t *__restrict__ dep_out) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= c) return;
    const int32_t a = anc_in[C];
    if (a >= 0) {
        dep_out[C] = dep_in[C] + dep_in[a];
        anc_out[C] = anc_in[a];
    } else {
        dep_out[C] = dep_in[C];
        anc_out[C] = -1;
    }
}

// After enough rounds every chain of an acyclic hierarchy has ended; a class
// that still has an ancestor lies on a cycle or under one.
__global__ __launch_bounds__(256) void k_ck_cycle(const int32_t *__restrict__ anc, int c, int *__restrict__ err) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C < c && anc[C] >= 0) atomicOr(err, ERR_CYCLE);
}

// One wave per class: WMC over the members (unit weights when weight is NULL),
// with NOC and DIT copied beside it.
__global__ __launch_bounds__(256) void k_ck_class(DevSys d, const int32_t *__restrict__ weight,
                                                  const int32_t *__restrict__ noc, const int32_t *__restrict__ dit,
                                                  CkOut *__restrict__ out) {
    const int C = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (C >= d.c) return;
    const int lane = threadIdx.x & 63;
    const int mb = d.mem_off[C], me = d.mem_end[C];
    long long s = 0;
    if (weight) {
        for (int i = mb + lane; i < me; i += WAVE) s += weight[d.mem_idx[i]];
        s = wave_sum64(s);
    } else {
        s = me - mb;
    }
    if (lane == 0) {
        CkOut o;
        o.wmc = s;
        o.noc = noc ? noc[C] : 0;
        o.dit = dit ? dit[C] : 0;
        out[C] = o;
    }
}

int ck_rounds(int64_t c) {
    int r = 1;
    while (((int64_t)1 << r) < c) ++r;  // 2^r >= c > longest chain of an acyclic hierarchy
    return r + 1;
}

void launch_ck_hierarchy(const int32_t *parent, int c, int32_t *noc, int32_t *dit, int32_t *anc, int32_t *anc2,
                         int32_t *dep2, int *err, hipStream_t st) {
    if (c <= 0) return;
    const unsigned g = ck_blocks(c, 256);
    fill_i32(noc, 0, c, st);
    k_ck_init<<<g, 256, 0, st>>>(parent, c, noc, anc, dit);
    int32_t *ai = anc, *di = dit, *ao = anc2, *dout = dep2;
    const int rounds = ck_rounds(c);
    for (int r = 0; r < rounds; ++r) {
        k_ck_jump<<<g, 256, 0, st>>>(ai, di, c, ao, dout);
        std::swap(ai, ao);
        std::swap(di, dout);
    }
    if (di != dit) (void)hipMemcpyAsync(dit, di, (size_t)c * 4, hipMemcpyDeviceToDevice, st);
    k_ck_cycle<<<g, 256, 0, st>>>(ai, c, err);
}

void launch_ck_class(const DevSys &d, const int32_t *weight, const int32_t *noc, const int32_t *dit, CkOut *out,
                     hipStream_t st) {
    if (d.c > 0) k_ck_class<<<ck_blocks(d.c, 4), 256, 0, st>>>(d, weight, noc, dit, out);
}

}  // namespace mm

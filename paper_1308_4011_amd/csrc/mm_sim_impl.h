// mm_sim_impl.h -- host side of the similarity of method pairs (Sec. II-A) and
// of the candidates it suggests (Sec. III-A); included by mm_api.hip, whose
// engine it shares. The kernels are in k_sim.hip.
//
// The average similarity is an exact fraction: with hist[u] = sum of shared
// counts over the pairs whose union has size u, the sum of similarities is
// A / B where B = lcm of the union sizes present and A = sum hist[u] * (B / u).
// A pair (shared i, union u) is above the average over `cnt` pairs iff
// i * B * cnt > A * u, so the least such i per union size, imin[u], is found by
// exact integer comparison and handed to the kernels as a table.

namespace {

// unsigned big integer, 32-bit limbs, little endian (only what the threshold needs)
struct BigU {
    std::vector<uint32_t> w;
    explicit BigU(uint64_t v = 0) {
        while (v) {
            w.push_back((uint32_t)v);
            v >>= 32;
        }
    }
    void trim() {
        while (!w.empty() && w.back() == 0) w.pop_back();
    }
    void mul32(uint32_t m) {
        uint64_t carry = 0;
        for (auto &x : w) {
            const uint64_t t = (uint64_t)x * m + carry;
            x = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) w.push_back((uint32_t)carry);
        trim();
    }
    void add(const BigU &o) {
        if (o.w.size() > w.size()) w.resize(o.w.size(), 0);
        uint64_t carry = 0;
        for (size_t i = 0; i < w.size(); ++i) {
            const uint64_t t = (uint64_t)w[i] + (i < o.w.size() ? o.w[i] : 0) + carry;
            w[i] = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) w.push_back((uint32_t)carry);
    }
    void mul(uint64_t m) {  // *= m
        BigU hi = *this;
        mul32((uint32_t)m);
        const uint32_t h = (uint32_t)(m >> 32);
        if (h) {
            hi.mul32(h);
            hi.w.insert(hi.w.begin(), 0u);
            hi.trim();
            add(hi);
        }
    }
    uint32_t mod(uint32_t d) const {
        uint64_t r = 0;
        for (size_t i = w.size(); i-- > 0;) r = ((r << 32) | w[i]) % d;
        return (uint32_t)r;
    }
    void div(uint32_t d) {  // floor division
        uint64_t r = 0;
        for (size_t i = w.size(); i-- > 0;) {
            const uint64_t cur = (r << 32) | w[i];
            w[i] = (uint32_t)(cur / d);
            r = cur % d;
        }
        trim();
    }
    size_t bits() const { return w.empty() ? 0 : 32 * (w.size() - 1) + (32 - __builtin_clz(w.back())); }
    int cmp(const BigU &o) const {
        if (w.size() != o.w.size()) return w.size() < o.w.size() ? -1 : 1;
        for (size_t i = w.size(); i-- > 0;)
            if (w[i] != o.w[i]) return w[i] < o.w[i] ? -1 : 1;
        return 0;
    }
};

uint32_t gcd_u32(uint32_t a, uint32_t b) {
    while (b) {
        const uint32_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

void check_threshold(int32_t threshold) {
    if (threshold < MM_SIM_NONZERO || threshold > MM_SIM_ABOVE_AVG_NZ) fail(MM_EINVAL, "bad similarity threshold");
}

SimPlan sim_plan(mm_system *s, int32_t mode) {
    SimPlan p;
    memset(&p, 0, sizeof(p));
    p.mode = mode;
    p.cw = s->sim.cw;
    p.at_off = s->sim_at_off.as<int64_t>();
    p.at_idx = s->sim_at_idx.as<int32_t>();
    p.deg = s->sim_deg.as<int32_t>();
    p.dense = s->sim_dense.as<int32_t>();
    p.cnt2 = s->sim_cnt2.as<int32_t>();
    p.ticket = s->sim_ctr.as<int32_t>();
    p.nnz = (unsigned long long *)(s->sim_ctr.as<char>() + 8);
    p.hist = s->sim_hist.as<unsigned long long>();
    p.imin = s->sim_imin.as<int32_t>();
    p.row_pairs = s->sim_row_pairs.as<int32_t>();
    p.row_cands = s->sim_row_cands.as<int32_t>();
    p.cand_bits = s->sim_cand_bits.as<uint32_t>();
    p.pair_off = s->sim_pair_off.as<int64_t>();
    p.pairs = s->sim_pairs.as<int4>();
    p.timer = s->ctx->timer.enabled() ? &s->ctx->timer : nullptr;
    return p;
}

// Accessor lists, property counts and the per-workgroup counters of one version.
void sim_prepare(mm_system *s) {
    if (s->part_cls.size() > 2) fail(MM_EINVAL, "similarity of a batch would average over several systems");
    ensure_metrics(s);
    if (s->sim.at_version == s->version && s->sim_dense.p) return;
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    const int32_t n = s->n, na = s->na;
    const DevSys d = s->view();
    s->sim_at_off.reserve(ctx, cb, ((size_t)na + 1) * 8);
    s->sim_at_idx.reserve(ctx, cb, std::max<size_t>(s->acc_idx.size(), 1) * 4);
    s->sim_at_cur.reserve(ctx, cb, ((size_t)na + 1) * 4);
    s->sim_deg.reserve(ctx, cb, ((size_t)n + 1) * 4);
    fill_i32(s->sim_at_cur.as<int32_t>(), 0, na, st);
    launch_at_build(d, nullptr, s->sim_at_cur.as<int32_t>(), nullptr, 0, st);
    scan_i32(s->sim_at_cur.as<int32_t>(), s->sim_at_off.as<int64_t>(), na, scan_area(s, na), st);
    fill_i32(s->sim_at_cur.as<int32_t>(), 0, na, st);
    launch_at_build(d, s->sim_at_off.as<int64_t>(), s->sim_at_cur.as<int32_t>(), s->sim_at_idx.as<int32_t>(), 1, st);
    launch_sim_deg(d, s->sim_deg.as<int32_t>(), st);
    // longest property set, and the users a row walks (callers of its callees
    // plus accessors of its attributes), which the kernel counts in 32 bits
    int32_t maxdeg = 0;
    std::vector<int64_t> accessors(na, 0);
    for (int32_t a : s->acc_idx) accessors[a]++;
    for (int32_t m = 0; m < n; ++m) {
        maxdeg = std::max(maxdeg, (s->call_off[m + 1] - s->call_off[m]) + (s->acc_off[m + 1] - s->acc_off[m]));
        int64_t walk = 0;
        for (int32_t e = s->call_off[m]; e < s->call_off[m + 1]; ++e)
            walk += s->rc_off[s->call_idx[e] + 1] - s->rc_off[s->call_idx[e]];
        for (int32_t e = s->acc_off[m]; e < s->acc_off[m + 1]; ++e) walk += accessors[s->acc_idx[e]];
        if (walk > INT32_MAX) fail(MM_EOVERFLOW, "a method shares properties with more than 2^31 users");
    }
    s->sim.umax = 2 * maxdeg;
    // persistent workgroups: three per CU (LDS bound), no more than rows, and
    // their private counters (two arrays of n) under 1 GiB
    int64_t g = std::min<int64_t>(3 * (int64_t)ctx->n_cu, std::max<int32_t>(n, 1));
    g = std::max<int64_t>(1, std::min<int64_t>(g, (1LL << 30) / std::max<int64_t>(8 * (int64_t)n, 1)));
    s->sim.grid = (int32_t)g;
    s->sim_dense.reserve(ctx, cb, (size_t)g * std::max(n, 1) * 4);
    s->sim_ctr.reserve(ctx, cb, 16);
    HIPCHK(hipGetLastError());
    s->sim.at_version = s->version;
    s->sim.stats_version = s->sim.count_version = -1;
}

// Sum of shared counts by union size and the number of pairs sharing a property.
void sim_stats(mm_system *s) {
    sim_prepare(s);
    if (s->sim.stats_version == s->version) return;
    mm_context *ctx = s->ctx;
    hipStream_t st = s->stream;
    const int32_t U = s->sim.umax + 1;
    s->sim_hist.reserve(ctx, &s->bytes, (size_t)U * 8);
    fill_i32(s->sim_hist.as<int32_t>(), 0, 2 * (int64_t)U, st);
    fill_i32(s->sim_ctr.as<int32_t>(), 0, 4, st);
    fill_i32(s->sim_dense.as<int32_t>(), 0, (int64_t)s->sim.grid * s->n, st);
    launch_sim_rows(s->view(), sim_plan(s, SIM_STATS), s->sim.grid, st);
    HIPCHK(hipGetLastError());
    s->sim.hist.assign(U, 0);
    HIPCHK(hipMemcpyAsync(s->sim.hist.data(), s->sim_hist.p, (size_t)U * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&s->sim.nnz, s->sim_ctr.as<char>() + 8, 8, hipMemcpyDeviceToHost, st));
    check_kernel_errors(s);  // synchronizes; the accessor lists were laid out by a scan
    s->sim.stats_version = s->version;
}

// imin[u] for u in [0, umax]: least shared count of a high pair of union u
// (u + 1 when none), and the average rounded to double.
void sim_threshold(mm_system *s, int32_t threshold, std::vector<int32_t> &imin, double &avg) {
    const int32_t U = s->sim.umax + 1;
    imin.assign(U, 1);
    avg = 0;
    if (threshold == MM_SIM_NONZERO) return;
    const uint64_t n = (uint64_t)s->n;
    const uint64_t cnt = threshold == MM_SIM_ABOVE_AVG ? (n >= 2 ? n * (n - 1) / 2 : 0) : s->sim.nnz;
    if (cnt == 0 || s->sim.nnz == 0) {
        for (int32_t u = 0; u < U; ++u) imin[u] = u + 1;
        return;
    }
    BigU B(1);
    long double approx = 0;
    for (int32_t u = 1; u < U; ++u) {
        if (!s->sim.hist[u]) continue;
        B.mul(u / gcd_u32(B.mod((uint32_t)u), (uint32_t)u));
        if (B.bits() > 8192) fail(MM_EOVERFLOW, "union sizes too varied for an exact average");
        approx += (long double)s->sim.hist[u] / u;
    }
    BigU A(0);
    for (int32_t u = 1; u < U; ++u) {
        if (!s->sim.hist[u]) continue;
        BigU t = B;
        t.div((uint32_t)u);
        t.mul(s->sim.hist[u]);
        A.add(t);
    }
    avg = (double)(approx / (long double)cnt);
    BigU Y = B;
    Y.mul(cnt);  // i is high iff i * Y > A * u
    imin[0] = 1;
    for (int32_t u = 1; u < U; ++u) {
        BigU X = A;
        X.mul((uint64_t)u);
        int32_t lo = 1, hi = u + 1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            BigU Z = Y;
            Z.mul((uint64_t)mid);
            if (Z.cmp(X) > 0) hi = mid; else lo = mid + 1;
        }
        imin[u] = lo;
    }
}

// High pairs per row and the candidate-class bitmap under `threshold`.
void sim_count(mm_system *s, int32_t threshold) {
    check_threshold(threshold);
    sim_stats(s);
    if (s->sim.count_version == s->version && s->sim.count_threshold == threshold) return;
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    const int32_t n = s->n, c = s->c;
    const int32_t cw = (c + 31) / 32;
    if (cw > SIM_BITS_WORDS) fail(MM_EOVERFLOW, "similarity candidates support at most 2^18 classes");
    s->sim.cw = cw;
    double avg;
    sim_threshold(s, threshold, s->sim.imin, avg);
    const int32_t U = s->sim.umax + 1;
    s->sim_imin.reserve(ctx, cb, (size_t)U * 4);
    s->sim_row_pairs.reserve(ctx, cb, ((size_t)n + 1) * 4);
    s->sim_row_cands.reserve(ctx, cb, ((size_t)n + 1) * 4);
    s->sim_pair_off.reserve(ctx, cb, ((size_t)n + 1) * 8);
    s->sim_cand_off.reserve(ctx, cb, ((size_t)n + 1) * 8);
    s->sim_cand_bits.reserve(ctx, cb, std::max<size_t>((size_t)n * cw, 1) * 4);
    HIPCHK(hipMemcpyAsync(s->sim_imin.p, s->sim.imin.data(), (size_t)U * 4, hipMemcpyHostToDevice, st));
    fill_i32(s->sim_ctr.as<int32_t>(), 0, 1, st);
    fill_i32(s->sim_dense.as<int32_t>(), 0, (int64_t)s->sim.grid * n, st);
    launch_sim_rows(s->view(), sim_plan(s, SIM_COUNT), s->sim.grid, st);
    HIPCHK(hipGetLastError());
    scan_i32(s->sim_row_pairs.as<int32_t>(), s->sim_pair_off.as<int64_t>(), n, scan_area(s, n), st);
    scan_i32(s->sim_row_cands.as<int32_t>(), s->sim_cand_off.as<int64_t>(), n, scan_area(s, n), st);
    s->sim.row_cands.assign(n, 0);
    if (n) HIPCHK(hipMemcpyAsync(s->sim.row_cands.data(), s->sim_row_cands.p, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&s->sim.n_kept, s->sim_pair_off.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&s->sim.n_cands, s->sim_cand_off.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st));
    check_kernel_errors(s);  // synchronizes
    s->sim.average = avg;
    s->sim.count_version = s->version;
    s->sim.count_threshold = threshold;
}

// MM_CAND_SIMILAR candidates into cm / ct (device); returns their number.
int64_t sim_candidates(mm_system *s, int32_t threshold, DBuf &cm, DBuf &ct) {
    sim_count(s, threshold);
    const int64_t nc = s->sim.n_cands;
    if (nc > INT32_MAX) fail(MM_EOVERFLOW, "more than 2^31-1 similarity candidates");
    cm.reserve(s->ctx, &s->bytes, (size_t)std::max<int64_t>(nc, 1) * 4);
    ct.reserve(s->ctx, &s->bytes, (size_t)std::max<int64_t>(nc, 1) * 4);
    SimPlan p = sim_plan(s, SIM_COUNT);
    p.out_cap = nc;
    if (nc) launch_sim_emit(s->view(), p, s->sim_cand_off.as<int64_t>(), cm.as<int32_t>(), ct.as<int32_t>(),
                            s->stream);
    HIPCHK(hipGetLastError());
    return nc;
}

// The high pairs under `threshold`, (m1, m2) ascending, into host memory.
void sim_pairs(mm_system *s, int32_t threshold, mm_sim_pair *out, int64_t cap, int64_t *n_out) {
    if (!n_out) fail(MM_EINVAL, "n is NULL");
    sim_count(s, threshold);
    const int64_t total = s->sim.n_kept;
    *n_out = total;
    if (!out) return;
    if (cap < total) fail(MM_ERANGE, "output capacity " + std::to_string(cap) + " < " + std::to_string(total));
    if (total == 0) return;
    if (((int64_t)s->n + 31) / 32 > SIM_BITS_WORDS) fail(MM_EOVERFLOW, "pair listing supports at most 2^18 methods");
    mm_context *ctx = s->ctx;
    hipStream_t st = s->stream;
    s->sim_cnt2.reserve(ctx, &s->bytes, (size_t)s->sim.grid * std::max(s->n, 1) * 4);
    s->sim_pairs.reserve(ctx, &s->bytes, (size_t)total * sizeof(int4));
    fill_i32(s->sim_ctr.as<int32_t>(), 0, 1, st);
    fill_i32(s->sim_dense.as<int32_t>(), 0, (int64_t)s->sim.grid * s->n, st);
    SimPlan p = sim_plan(s, SIM_PAIRS);
    p.out_cap = total;
    launch_sim_rows(s->view(), p, s->sim.grid, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, s->sim_pairs.p, (size_t)total * sizeof(int4), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
}

}  // namespace

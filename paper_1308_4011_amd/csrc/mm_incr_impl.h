// mm_incr_impl.h -- incremental recompute after moves (included by mm_api.hip,
// whose engine it extends).
//
// A move of method m from S to T (Sec. III-A; Sec. IV-C re-runs the metrics on
// the changed membership) changes only what these sets reach:
//   W (classes used, with counts): S and T, whose members' references change,
//     and every class X owning a caller of m, whose references to m now go to
//     T instead of S;
//   CNT (methods called, with counts) and the co-access of LCOM: S and T;
//   caller maps: m itself (its own class changed), the methods m calls (their
//     callers in S and T changed), and every method x called from a class X
//     whose W changed, when x's class is one of the W keys that changed (the
//     loss flag of the entry (x, X) compares w_X(class of x) with x's callers
//     in X). The keys that change are S, T and the classes m references; the
//     union over the moves since the last recompute is used for every X;
//   per-method counts: m (its own-attribute uses and mask);
//   class aggregates: every class above.
// The host keeps the membership rows and the W / CNT table sizes current: a
// class row that outgrows its region, or a table that needs more slots, moves to
// the end of its pool; when a pool is full the move falls back to a full layout
// rebuild. The device structure is patched at once (owner, membership, table
// headers); the recompute of the touched segments runs at the next metric
// request and leaves every other segment as it was. Its results equal a full
// recompute bit for bit (the integer counts do not depend on the order of
// their terms).

namespace {

enum : uint8_t { DC_W = 1, DC_CNT = 2, DC_CO = 4, DC_KEY = 8 };  // dirty bits of a class
enum : uint8_t { DM_IN = 1, DM_BASIC = 2 };                      // dirty bits of a method

void mark_class(mm_system *s, int32_t C, uint8_t bits) {
    uint8_t &f = s->incr.fc[(size_t)C];
    if (!f) s->incr.lc.push_back(C);
    f |= bits;
}

void mark_method(mm_system *s, int32_t m, uint8_t bits) {
    uint8_t &f = s->incr.fm[(size_t)m];
    if (!f) s->incr.lm.push_back(m);
    f |= bits;
}

void clear_dirty(mm_system *s) {
    for (int32_t C : s->incr.lc) s->incr.fc[(size_t)C] = 0;
    for (int32_t m : s->incr.lm) s->incr.fm[(size_t)m] = 0;
    s->incr.lc.clear();
    s->incr.lm.clear();
    s->incr.active = false;
}

// Called at the end of build_layout: pools sized with room to grow, no pending work.
void incr_reset(mm_system *s, const std::vector<int64_t> &Rw, const std::vector<int64_t> &Rc) {
    Incr &ic = s->incr;
    ic.fc.assign((size_t)s->c, 0);
    ic.fm.assign((size_t)s->n, 0);
    ic.lc.clear();
    ic.lm.clear();
    ic.active = false;
    ic.stale = false;
    ic.base = false;  // no metric computed on this layout yet
    ic.Rw = Rw;
    ic.Rc = Rc;
    ic.mem_lim = s->mem_end;
    ic.mem_used = s->n;
}

// Mark W dirty for every class owning a caller of the given methods, read on
// the device from the callers as they stand (before any pending patch).
void mark_caller_classes(mm_system *s, const std::vector<int32_t> &methods) {
    if (methods.empty()) return;
    Incr &ic = s->incr;
    mm_context *ctx = s->ctx;
    hipStream_t st = s->stream;
    const size_t c = (size_t)s->c;
    ic.d_flags.reserve(ctx, &s->bytes, std::max<size_t>(c, 1) * 4 + methods.size() * 4);
    int32_t *flag = ic.d_flags.as<int32_t>();
    int32_t *list = flag + std::max<size_t>(c, 1);
    fill_i32(flag, 0, (int64_t)c, st);
    HIPCHK(hipMemcpyAsync(list, methods.data(), methods.size() * 4, hipMemcpyHostToDevice, st));
    launch_caller_classes(s->view(), list, (int)methods.size(), flag, st);
    ic.h_flags.resize(c);
    if (c) HIPCHK(hipMemcpyAsync(ic.h_flags.data(), flag, c * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t X = 0; X < c; ++X)
        if (ic.h_flags[X]) mark_class(s, (int32_t)X, DC_W);
}

// Upload the pending patch ops and apply them on the stream. The staging
// buffer is reused only after the event of its previous copy.
void flush_patches(mm_system *s) {
    Incr &ic = s->incr;
    if (ic.ops.empty()) return;
    if (ic.ops_ev_set) HIPCHK(hipEventSynchronize(ic.ops_ev));
    // the kernel applies ops in parallel: keep only the last op of each
    // (target, index), so a word patched twice ends with its latest value
    ic.ops_stage.clear();
    std::unordered_map<int64_t, int> seen;
    seen.reserve(ic.ops.size() * 2);
    for (size_t i = ic.ops.size(); i-- > 0;) {
        const int4 &op = ic.ops[i];
        if (seen.emplace(((int64_t)op.x << 32) | (uint32_t)op.y, 1).second) ic.ops_stage.push_back(op);
    }
    ic.ops.clear();
    const int n = (int)ic.ops_stage.size();
    ic.d_ops.reserve(s->ctx, &s->bytes, (size_t)n * sizeof(int4));
    HIPCHK(hipMemcpyAsync(ic.d_ops.p, ic.ops_stage.data(), (size_t)n * sizeof(int4), hipMemcpyHostToDevice,
                          s->stream));
    if (!ic.ops_ev) HIPCHK(hipEventCreateWithFlags(&ic.ops_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ic.ops_ev, s->stream));
    ic.ops_ev_set = true;
    PatchTargets t;
    t.t[PATCH_OWNER] = s->d_owner.as<int32_t>();
    t.t[PATCH_MEM_IDX] = s->d_mem_idx.as<int32_t>();
    t.t[PATCH_MEM_OFF] = s->d_mem_off.as<int32_t>();
    t.t[PATCH_MEM_END] = s->d_mem_end.as<int32_t>();
    t.t[PATCH_W_HDR] = s->w.hdr.as<int32_t>();
    t.t[PATCH_CNT_HDR] = s->cnt.hdr.as<int32_t>();
    t.t[PATCH_IN_HDR] = s->in.hdr.as<int32_t>();
    t.t[PATCH_PREP] = s->d_prep_runs.as<int32_t>();
    launch_patch(ic.d_ops.as<int4>(), n, t, s->stream);
    HIPCHK(hipGetLastError());
}

// queue a device word write; flush_patches applies the queue in one launch
void patch(mm_system *s, int target, int64_t index, int32_t value) {
    s->incr.ops.push_back(make_int4(target, (int)index, value, 0));
}

// slots a class table needs for R references (the rule of make_map)
int64_t class_table_slots(int64_t R, int64_t keyspace) {
    if (R <= 0) return 0;
    return R <= MAP_CAP ? pow2_at_least(2 * std::min(R, keyspace), 4) : pow2_at_least(2 * std::min(R, keyspace), 1024);
}

// room a table of class C needs (0: fits where it is)
int64_t table_growth(const DevMap &dm, int32_t C, int64_t R, int64_t keyspace) {
    const int64_t need = class_table_slots(R, keyspace);
    return need > dm.host_hdr[(size_t)C].cap ? need : 0;
}

void relocate_table(mm_system *s, DevMap &dm, int target, int32_t C, int64_t cap) {
    MapHdr &h = dm.host_hdr[(size_t)C];
    h = MapHdr{(int32_t)dm.slots, 0, MAP_TABLE, (int32_t)cap};
    dm.slots += cap;
    patch(s, target, 4 * (int64_t)C + 0, h.base);
    patch(s, target, 4 * (int64_t)C + 2, h.kind);
    patch(s, target, 4 * (int64_t)C + 3, h.cap);
}

// membership: m leaves C (the last member takes its place)
void member_remove(mm_system *s, int32_t C, int32_t m) {
    int32_t j = s->mem_off[C];
    while (s->mem_idx[(size_t)j] != m) ++j;
    const int32_t last = s->mem_end[C] - 1;
    s->mem_idx[(size_t)j] = s->mem_idx[(size_t)last];
    patch(s, PATCH_MEM_IDX, j, s->mem_idx[(size_t)j]);
    s->mem_end[C] = last;
    patch(s, PATCH_MEM_END, C, last);
}

// region a class row needs to take one more member (0: it fits)
int64_t member_growth(const mm_system *s, int32_t C) {
    if (s->mem_end[C] < s->incr.mem_lim[(size_t)C]) return 0;
    const int64_t n = s->mem_end[C] - s->mem_off[C];
    return std::max<int64_t>(8, 2 * (n + 1));
}

void member_insert(mm_system *s, int32_t C, int32_t m, int64_t grow) {
    Incr &ic = s->incr;
    if (grow) {  // move the row to the end of the pool with room to grow
        if (ic.mem_used + grow > ic.mem_cap) fail(MM_EINTERNAL, "membership pool exhausted");
        const int32_t b = s->mem_off[C], e = s->mem_end[C];
        const int32_t nb = (int32_t)ic.mem_used;
        for (int32_t j = b; j < e; ++j) {
            s->mem_idx[(size_t)(nb + j - b)] = s->mem_idx[(size_t)j];
            patch(s, PATCH_MEM_IDX, nb + j - b, s->mem_idx[(size_t)j]);
        }
        s->mem_off[C] = nb;
        s->mem_end[C] = nb + (e - b);
        ic.mem_lim[(size_t)C] = (int32_t)(nb + grow);
        ic.mem_used += grow;
        patch(s, PATCH_MEM_OFF, C, s->mem_off[C]);
    }
    const int32_t at = s->mem_end[C];
    if (at >= ic.mem_lim[(size_t)C]) fail(MM_EINTERNAL, "class row region full");
    s->mem_idx[(size_t)at] = m;
    patch(s, PATCH_MEM_IDX, at, m);
    s->mem_end[C] = at + 1;
    patch(s, PATCH_MEM_END, C, at + 1);
}

// Apply the move m -> T incrementally; false (nothing changed) when a pool has
// no room for it, so the caller takes the full path.
bool move_incremental(mm_system *s, int32_t m, int32_t T) {
    Incr &ic = s->incr;
    const int32_t S = s->owner[m];
    const int64_t nc = s->call_off[m + 1] - s->call_off[m];
    const int64_t na = s->acc_off[m + 1] - s->acc_off[m];
    // room first: the member row of T and the W / CNT tables of T
    const int64_t mg = member_growth(s, T);
    const int64_t wg = table_growth(s->w, T, ic.Rw[(size_t)T] + nc + na, s->c);
    const int64_t cg = table_growth(s->cnt, T, ic.Rc[(size_t)T] + nc, s->n);
    if (ic.mem_used + mg > ic.mem_cap || s->w.slots + wg > s->w.pool_cap || s->cnt.slots + cg > s->cnt.pool_cap)
        return false;
    // what the move touches, from the state before it
    mark_class(s, S, DC_W | DC_CNT | DC_CO | DC_KEY);
    mark_class(s, T, DC_W | DC_CNT | DC_CO | DC_KEY);
    if (s->rc_off[m + 1] > s->rc_off[m]) mark_caller_classes(s, {m});
    for (int32_t e = s->call_off[m]; e < s->call_off[m + 1]; ++e) {
        const int32_t x = s->call_idx[(size_t)e];
        mark_class(s, s->owner[x], DC_KEY);
        if (x != m) mark_method(s, x, DM_IN);
    }
    for (int32_t e = s->acc_off[m]; e < s->acc_off[m + 1]; ++e) mark_class(s, s->acls[s->acc_idx[(size_t)e]], DC_KEY);
    mark_method(s, m, DM_IN | DM_BASIC);
    // the move itself
    s->owner[m] = T;
    patch(s, PATCH_OWNER, m, T);
    member_remove(s, S, m);
    member_insert(s, T, m, mg);
    ic.Rw[(size_t)S] -= nc + na;
    ic.Rc[(size_t)S] -= nc;
    ic.Rw[(size_t)T] += nc + na;
    ic.Rc[(size_t)T] += nc;
    if (wg) relocate_table(s, s->w, PATCH_W_HDR, T, wg);
    if (cg) relocate_table(s, s->cnt, PATCH_CNT_HDR, T, cg);
    flush_patches(s);
    ic.active = true;
    ic.stale = true;  // the layout's full work lists describe the old membership
    return true;
}

// ---------------------------------------------------------------------------
// Edits (rows of k methods replaced, owners maybe changed). Besides what a move
// of each owner-changing method touches: the classes owning an edited method
// (W, CNT, co-access of the old and new owner), the callers maps and fan-in of
// every method an edited method called before or calls after, the row-length
// work list of the edited methods, and the rows and callers on the device
// (edited rows uploaded and spliced in on the device, callers rebuilt there).

// row-length group of the scoring work list (segments of 8 / 16 / 32 / 64 lanes, or longer)
int prep_group(int64_t len) { return len <= 8 ? 0 : len <= 16 ? 1 : len <= 32 ? 2 : len <= 64 ? 3 : 4; }

// Host view of an edit after validation: methods in ascending order (ord) and
// their canonical new rows (ao/ai, co/ci indexed by the edit's own order).
struct EditView {
    const mm_edit_desc *e;
    const std::vector<int32_t> &ord, &ao, &ai, &co, &ci;
    int32_t new_owner(int32_t i, const mm_system *s) const {
        return e->new_class ? e->new_class[i] : s->owner[e->method[i]];
    }
};

// caller-map slots a method with R callers needs: (kind, capacity)
std::pair<int32_t, int64_t> in_region(int64_t R, int64_t c) {
    if (R <= IN_SMALL) return {MAP_RUN, R};
    return {MAP_TABLE, R <= MAP_CAP ? pow2_at_least(2 * std::min(R, c), 4) : pow2_at_least(2 * std::min(R, c), 1024)};
}

bool in_fits(const MapHdr &h, int64_t R, int64_t c) {
    if (R == 0) return true;
    if (h.kind == MAP_RUN) return R <= IN_SMALL && R <= h.cap;
    if (h.kind == MAP_TABLE) return pow2_at_least(2 * std::min(R, c), 4) <= h.cap;
    return false;
}

// The sizes an edit changes, gathered before anything changes: per class the
// change of its W and CNT references and of its member count, per method the
// change of its caller count. fits() tells whether the pools hold the growth.
struct EditPlan {
    std::unordered_map<int32_t, int64_t> dw, dc, dmem, drc;
    int64_t grow_w = 0, grow_c = 0, grow_i = 0, grow_mem = 0;
};

bool edit_plan(const mm_system *s, const EditView &v, EditPlan &P) {
    const int32_t k = v.e->k;
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = v.e->method[i], S = s->owner[m], S2 = v.new_owner(i, s);
        const int64_t onc = s->call_off[m + 1] - s->call_off[m], ona = s->acc_off[m + 1] - s->acc_off[m];
        const int64_t nnc = v.co[i + 1] - v.co[i], nna = v.ao[i + 1] - v.ao[i];
        P.dw[S] -= onc + ona;
        P.dc[S] -= onc;
        P.dw[S2] += nnc + nna;
        P.dc[S2] += nnc;
        if (S2 != S) {
            P.dmem[S] -= 1;
            P.dmem[S2] += 1;
        }
        for (int32_t e = s->call_off[m]; e < s->call_off[m + 1]; ++e) P.drc[s->call_idx[(size_t)e]] -= 1;
        for (int32_t e = v.co[i]; e < v.co[i + 1]; ++e) P.drc[v.ci[(size_t)e]] += 1;
    }
    for (auto &kv : P.dw)
        P.grow_w += table_growth(s->w, kv.first, s->incr.Rw[(size_t)kv.first] + kv.second, s->c);
    for (auto &kv : P.dc)
        P.grow_c += table_growth(s->cnt, kv.first, s->incr.Rc[(size_t)kv.first] + kv.second, s->n);
    for (auto &kv : P.dmem) {
        const int32_t C = kv.first;
        const int64_t n_after = (s->mem_end[C] - s->mem_off[C]) + kv.second;
        if (s->mem_off[C] + n_after > s->incr.mem_lim[(size_t)C]) P.grow_mem += std::max<int64_t>(8, 2 * n_after);
    }
    for (auto &kv : P.drc) {
        const int32_t x = kv.first;
        const int64_t R = (s->rc_off[x + 1] - s->rc_off[x]) + kv.second;
        if (!in_fits(s->in.host_hdr[(size_t)x], R, s->c)) P.grow_i += in_region(R, s->c).second;
    }
    const Incr &ic = s->incr;
    return ic.mem_used + P.grow_mem <= ic.mem_cap && s->w.slots + P.grow_w <= s->w.pool_cap &&
           s->cnt.slots + P.grow_c <= s->cnt.pool_cap && s->in.slots + P.grow_i <= s->in.pool_cap;
}

// What the edit touches, marked from the state before it.
void edit_mark(mm_system *s, const EditView &v) {
    const int32_t k = v.e->k;
    std::vector<int32_t> movers;  // edited methods that change owner and have callers
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = v.e->method[i];
        if (v.new_owner(i, s) != s->owner[m] && s->rc_off[m + 1] > s->rc_off[m]) movers.push_back(m);
    }
    mark_caller_classes(s, movers);
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = v.e->method[i], S = s->owner[m], S2 = v.new_owner(i, s);
        mark_class(s, S, DC_W | DC_CNT | DC_CO | DC_KEY);
        mark_class(s, S2, DC_W | DC_CNT | DC_CO | DC_KEY);
        // callees before and after: their callers change (and with them fan-in)
        for (int pass = 0; pass < 2; ++pass) {
            const int32_t *row = pass ? v.ci.data() + v.co[i] : s->call_idx.data() + s->call_off[m];
            const int64_t len = pass ? v.co[i + 1] - v.co[i] : s->call_off[m + 1] - s->call_off[m];
            for (int64_t e = 0; e < len; ++e) {
                const int32_t x = row[e];
                mark_class(s, s->owner[x], DC_KEY);
                mark_method(s, x, x != m ? (DM_IN | DM_BASIC) : DM_IN);
            }
            const int32_t *arow = pass ? v.ai.data() + v.ao[i] : s->acc_idx.data() + s->acc_off[m];
            const int64_t alen = pass ? v.ao[i + 1] - v.ao[i] : s->acc_off[m + 1] - s->acc_off[m];
            for (int64_t e = 0; e < alen; ++e) mark_class(s, s->acls[arow[e]], DC_KEY);
        }
        mark_method(s, m, DM_IN | DM_BASIC);
    }
}

// Move method m from group a to group b of the row-length work list: it walks
// group boundary by group boundary, swapping with the boundary element (order
// inside a group is free).
void prep_regroup(mm_system *s, int32_t m, int a, int b) {
    auto place = [&](int32_t pos, int32_t x) {
        s->prep_host[(size_t)pos] = x;
        s->prep_pos[(size_t)x] = pos;
        patch(s, PATCH_PREP, pos, x);
    };
    while (a < b) {
        const int32_t p = s->prep_pos[(size_t)m], last = s->prep_run_off[a + 1] - 1;
        const int32_t o = s->prep_host[(size_t)last];
        place(p, o);
        place(last, m);
        s->prep_run_off[a + 1] -= 1;  // m is now the first member of group a + 1
        ++a;
    }
    while (a > b) {
        const int32_t p = s->prep_pos[(size_t)m], first = s->prep_run_off[a];
        const int32_t o = s->prep_host[(size_t)first];
        place(p, o);
        place(first, m);
        s->prep_run_off[a] += 1;  // m is now the last member of group a - 1
        --a;
    }
}

// After the host rows hold the edit: owners, membership, table sizes, caller
// maps, callers offsets and the row-length list on the host; then the device
// rows, callers and patches.
void edit_apply(mm_system *s, const EditView &v, const EditPlan &P, const std::vector<int64_t> &old_len) {
    Incr &ic = s->incr;
    const int32_t k = v.e->k, n = s->n;
    // members leave their classes first; a class that gains members then gets
    // one region for its final size, so the inserts never move it again
    std::vector<std::pair<int32_t, int32_t>> arrive;  // (method, new class)
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = v.e->method[i], S = s->owner[m], S2 = v.new_owner(i, s);
        if (S2 == S) continue;
        s->owner[m] = S2;
        patch(s, PATCH_OWNER, m, S2);
        member_remove(s, S, m);
        arrive.emplace_back(m, S2);
    }
    std::unordered_map<int32_t, int64_t> gains;
    for (auto &a : arrive) gains[a.second] += 1;
    for (auto &kv : gains) {
        const int32_t C = kv.first;
        const int64_t n_final = (s->mem_end[C] - s->mem_off[C]) + kv.second;
        if (s->mem_off[C] + n_final > ic.mem_lim[(size_t)C]) {
            // move the row to the end of the pool with room for n_final members
            const int64_t region = std::max<int64_t>(8, 2 * n_final);
            const int32_t b0 = s->mem_off[C], keep_end = s->mem_end[C], nb = (int32_t)ic.mem_used;
            if (ic.mem_used + region > ic.mem_cap) fail(MM_EINTERNAL, "membership pool exhausted");
            for (int32_t j = b0; j < keep_end; ++j) {
                s->mem_idx[(size_t)(nb + j - b0)] = s->mem_idx[(size_t)j];
                patch(s, PATCH_MEM_IDX, nb + j - b0, s->mem_idx[(size_t)j]);
            }
            s->mem_off[C] = nb;
            s->mem_end[C] = nb + (keep_end - b0);
            ic.mem_lim[(size_t)C] = (int32_t)(nb + region);
            ic.mem_used += region;
            patch(s, PATCH_MEM_OFF, C, s->mem_off[C]);
            patch(s, PATCH_MEM_END, C, s->mem_end[C]);
        }
    }
    for (auto &a : arrive) member_insert(s, a.second, a.first, 0);
    for (auto &kv : P.dw) {
        ic.Rw[(size_t)kv.first] += kv.second;
        const int64_t g = table_growth(s->w, kv.first, ic.Rw[(size_t)kv.first], s->c);
        if (g) relocate_table(s, s->w, PATCH_W_HDR, kv.first, g);
    }
    for (auto &kv : P.dc) {
        ic.Rc[(size_t)kv.first] += kv.second;
        const int64_t g = table_growth(s->cnt, kv.first, ic.Rc[(size_t)kv.first], s->n);
        if (g) relocate_table(s, s->cnt, PATCH_CNT_HDR, kv.first, g);
    }
    // caller-map regions of the methods whose callers change, then the callers
    // offsets on the host (the device builds its own): one pass from the first
    // changed method with the running change
    std::vector<std::pair<int32_t, int64_t>> dl(P.drc.begin(), P.drc.end());
    std::sort(dl.begin(), dl.end());
    for (auto &kv : dl) {
        const int32_t x = kv.first;
        const int64_t R = (s->rc_off[x + 1] - s->rc_off[x]) + kv.second;
        MapHdr &h = s->in.host_hdr[(size_t)x];
        if (!in_fits(h, R, s->c)) {
            const auto r = in_region(R, s->c);
            h = MapHdr{(int32_t)s->in.slots, 0, r.first, (int32_t)r.second};
            s->in.slots += r.second;
            patch(s, PATCH_IN_HDR, 4 * (int64_t)x + 0, h.base);
            patch(s, PATCH_IN_HDR, 4 * (int64_t)x + 2, h.kind);
            patch(s, PATCH_IN_HDR, 4 * (int64_t)x + 3, h.cap);
        }
    }
    int64_t run = 0;
    for (size_t q = 0, x = dl.empty() ? (size_t)n : (size_t)dl[0].first; x < (size_t)n; ++x) {
        while (q < dl.size() && (size_t)dl[q].first == x) run += dl[q++].second;
        s->rc_off[x + 1] += (int32_t)run;
    }
    for (int32_t i = 0; i < k; ++i) {
        const int32_t m = v.e->method[i];
        const int64_t now = (s->call_off[m + 1] - s->call_off[m]) + (s->acc_off[m + 1] - s->acc_off[m]);
        const int a = prep_group(old_len[(size_t)i]), b = prep_group(now);
        if (a != b) prep_regroup(s, m, a, b);
    }
    // the device rows: the new rows of the edited methods in ascending method
    // order, uploaded once, spliced in on the device
    std::vector<int32_t> &H = ic.edit_stage;
    if (ic.edit_ev_set) HIPCHK(hipEventSynchronize(ic.edit_ev));
    H.clear();
    H.reserve((size_t)(3 * k + 2) + v.ai.size() + v.ci.size());
    for (int32_t j = 0; j < k; ++j) H.push_back(v.e->method[v.ord[(size_t)j]]);
    const size_t o_ao = H.size();
    H.push_back(0);
    for (int32_t j = 0; j < k; ++j) {
        const int32_t i = v.ord[(size_t)j];
        H.push_back(H.back() + (v.ao[i + 1] - v.ao[i]));
    }
    const size_t o_co = H.size();
    H.push_back(0);
    for (int32_t j = 0; j < k; ++j) {
        const int32_t i = v.ord[(size_t)j];
        H.push_back(H.back() + (v.co[i + 1] - v.co[i]));
    }
    const size_t o_ai = H.size();
    for (int32_t j = 0; j < k; ++j) {
        const int32_t i = v.ord[(size_t)j];
        H.insert(H.end(), v.ai.begin() + v.ao[i], v.ai.begin() + v.ao[i + 1]);
    }
    const size_t o_ci = H.size();
    for (int32_t j = 0; j < k; ++j) {
        const int32_t i = v.ord[(size_t)j];
        H.insert(H.end(), v.ci.begin() + v.co[i], v.ci.begin() + v.co[i + 1]);
    }
    mm_context *ctx = s->ctx;
    int64_t *cb = &s->bytes;
    hipStream_t st = s->stream;
    ic.d_edit.reserve(ctx, cb, std::max<size_t>(H.size(), 1) * 4);
    HIPCHK(hipMemcpyAsync(ic.d_edit.p, H.data(), H.size() * 4, hipMemcpyHostToDevice, st));
    if (!ic.edit_ev) HIPCHK(hipEventCreateWithFlags(&ic.edit_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ic.edit_ev, st));
    ic.edit_ev_set = true;
    const int32_t *D = ic.d_edit.as<int32_t>();
    const int64_t nacc = (int64_t)s->acc_idx.size(), ncall = (int64_t)s->call_idx.size();
    DBuf lens, pos, nao, nai, nco, nci;
    lens.alloc(ctx, nullptr, (size_t)2 * std::max<int32_t>(n, 1) * 4);
    pos.alloc(ctx, nullptr, (size_t)2 * ((size_t)n + 1) * 8);
    nao.alloc(ctx, cb, ((size_t)n + 1) * 4);
    nco.alloc(ctx, cb, ((size_t)n + 1) * 4);
    nai.alloc(ctx, cb, (size_t)std::max<int64_t>(nacc, 1) * 4);
    nci.alloc(ctx, cb, (size_t)std::max<int64_t>(ncall, 1) * 4);
    EditRows er;
    er.n = n;
    er.k = k;
    er.meth = D;
    er.e_acc_off = D + o_ao;
    er.e_call_off = D + o_co;
    er.e_acc_idx = D + o_ai;
    er.e_call_idx = D + o_ci;
    er.acc_off = s->d_acc_off.as<int32_t>();
    er.acc_idx = s->d_acc_idx.as<int32_t>();
    er.call_off = s->d_call_off.as<int32_t>();
    er.call_idx = s->d_call_idx.as<int32_t>();
    er.len_acc = lens.as<int32_t>();
    er.len_call = lens.as<int32_t>() + std::max<int32_t>(n, 1);
    int64_t *pa = pos.as<int64_t>(), *pc = pos.as<int64_t>() + n + 1;
    launch_edit_lengths(er, st);
    scan2_i32(er.len_acc, pa, n, er.len_call, pc, n, scan_area(s, 2 * (int64_t)n + 2), st);
    launch_edit_copy(er, pa, pc, nao.as<int32_t>(), nai.as<int32_t>(), nco.as<int32_t>(), nci.as<int32_t>(), st);
    HIPCHK(hipGetLastError());
    s->d_acc_off.swap(nao);
    s->d_acc_idx.swap(nai);
    s->d_call_off.swap(nco);
    s->d_call_idx.swap(nci);
    rebuild_callers(s);
    ++s->structure_version;  // the host copy of the callers is out of date
    flush_patches(s);
    ic.active = true;
    ic.stale = true;
}

// The recompute of everything the pending moves touched; the caller's buffers
// (if any) then receive the whole metric arrays.
void dirty_recompute(mm_system *s, ClassAgg *cls_dst, MethodAgg *meth_dst) {
    Incr &ic = s->incr;
    flush_patches(s);
    ensure_entry_classes(s);  // the owners or rows changed
    hipStream_t st = s->stream;
    mm_context *ctx = s->ctx;
    const DevSys dv = s->view();
    // Caller maps to rebuild, found and filed on the device: the marked
    // methods, plus every method called from a class whose W changed and owned
    // by a class among the changed W keys (its loss flag may differ); each filed
    // by the kind of its caller map. Only the counts and the few hash-table
    // segments come back.
    if (ic.plan_ev_set) HIPCHK(hipEventSynchronize(ic.plan_ev));
    std::vector<int32_t> &H1 = ic.plan_stage;
    H1.clear();
    ic.key_host.assign((size_t)s->c, 0);
    int32_t n_wdirty = 0, n_inmark = 0;
    for (int32_t C : ic.lc)
        if (ic.fc[(size_t)C] & DC_W) {
            H1.push_back(C);
            ++n_wdirty;
        }
    for (int32_t C : ic.lc)
        if (ic.fc[(size_t)C] & DC_KEY) ic.key_host[(size_t)C] = 1;
    for (int32_t m : ic.lm)
        if (ic.fm[(size_t)m] & DM_IN) {
            H1.push_back(m);
            ++n_inmark;
        }
    const int64_t n = s->n, stride = std::max<int64_t>(n, 1);
    ic.d_mark.reserve(ctx, &s->bytes, (size_t)stride + 64);
    if (ic.mark_block != ic.d_mark.p) {  // a new block: clear it (each pass clears the marks it files)
        fill_i32(ic.d_mark.as<int32_t>(), 0, (int64_t)(ic.d_mark.bytes / 4), st);
        ic.mark_block = ic.d_mark.p;
    }
    ic.d_inl.reserve(ctx, &s->bytes, ((size_t)8 + 6 * (size_t)stride) * 4);
    ic.d_key.reserve(ctx, &s->bytes, std::max<size_t>((size_t)s->c, 1) + H1.size() * 4 + 64);
    uint8_t *kdev = ic.d_key.as<uint8_t>();
    int32_t *h1dev = reinterpret_cast<int32_t *>(kdev + ((std::max<size_t>((size_t)s->c, 1) + 15) / 16) * 16);
    if (s->c) HIPCHK(hipMemcpyAsync(kdev, ic.key_host.data(), (size_t)s->c, hipMemcpyHostToDevice, st));
    if (!H1.empty()) HIPCHK(hipMemcpyAsync(h1dev, H1.data(), H1.size() * 4, hipMemcpyHostToDevice, st));
    int32_t *counts = ic.d_inl.as<int32_t>();
    int32_t *lists = counts + 8;  // group q at lists + q * stride; the global-table group 0 right after the counts
    fill_i32(counts, 0, 8, st);
    uint8_t *mark = ic.d_mark.as<uint8_t>();
    launch_incr_mark(h1dev + n_wdirty, n_inmark, mark, st);
    launch_incr_flag_walk(dv, h1dev, n_wdirty, kdev, mark, st);
    launch_incr_in_lists(dv, s->in.hdr.as<MapHdr>(), mark, lists, stride, counts, st);
    HIPCHK(hipGetLastError());
    // counts and the start of the global-table list in one copy
    const size_t head = 8 + (size_t)std::min<int64_t>(stride, 4096);
    ic.inl_host.resize(head);
    HIPCHK(hipMemcpyAsync(ic.inl_host.data(), counts, head * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int32_t in_cnt[6];  // 0 global tables, 1..4 run groups, 5 LDS tables
    for (int q = 0; q < 6; ++q) in_cnt[q] = ic.inl_host[(size_t)q];
    std::vector<int32_t> in_big_list(ic.inl_host.begin() + 8,
                                     ic.inl_host.begin() + 8 + std::min<int32_t>(in_cnt[0], 4096));
    if (in_cnt[0] > 4096) {
        in_big_list.resize((size_t)in_cnt[0]);
        HIPCHK(hipMemcpyAsync(in_big_list.data(), lists, (size_t)in_cnt[0] * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    std::vector<int32_t> w_small, w_large, w_mid, c_small, c_large, c_mid, fin, co_small;
    std::vector<int4> i_flag;
    for (BigHost &bh : ic.big) bh.clear();
    std::vector<int2> co_groups, co_wide;
    for (int32_t C : ic.lc) {
        const uint8_t f = ic.fc[(size_t)C];
        if (f & DC_W) {
            const MapHdr &h = s->w.host_hdr[(size_t)C];
            if (h.kind == MAP_TABLE && h.cap > MID_HMAX) {
                big_class_items(s, ic.big[0], C, h.cap, false, BIG_CHUNK);
            } else if (h.kind == MAP_TABLE && h.cap > MAP_HMAX) {
                w_mid.push_back(C);
            } else if (h.kind == MAP_TABLE) {
                (h.cap > MAP_HSMALL ? w_large : w_small).push_back(C);
            }
        }
        if (f & DC_CNT) {
            const MapHdr &h = s->cnt.host_hdr[(size_t)C];
            if (h.kind == MAP_TABLE && h.cap > MID_HMAX) {
                big_class_items(s, ic.big[1], C, h.cap, true, BIG_CHUNK);
            } else if (h.kind == MAP_TABLE && h.cap > MAP_HMAX) {
                c_mid.push_back(C);
            } else if (h.kind == MAP_TABLE) {
                (h.cap > MAP_HSMALL ? c_large : c_small).push_back(C);
            }
        }
        if ((f & DC_CO) && s->acnt[C] > 0) {
            const int32_t nm = s->mem_end[C] - s->mem_off[C];
            if (nm > 0) {
                if (s->acnt[C] <= 64 && nm <= 64)
                    co_small.push_back(C);
                else if (s->acnt[C] <= 64)
                    for (int32_t t = 0; t * 16 < nm; t += 4) co_groups.push_back(make_int2(C, t));
                else
                    for (int32_t t = 0; t * 16 < nm; ++t) co_wide.push_back(make_int2(C, t));
            }
        }
        if (f & (DC_W | DC_CNT | DC_CO)) fin.push_back(C);
    }
    std::vector<int32_t> basic_zero, basic_keep;
    for (int32_t m : in_big_list) {
        const MapHdr &h = s->in.host_hdr[(size_t)m];
        big_caller_items(s, ic.big[2], m, h.cap, BIG_CHUNK);
        for (int32_t a = 0; a < h.cap; a += BIG_CHUNK) i_flag.push_back(make_int4(m, a, std::min(a + BIG_CHUNK, h.cap), 0));
    }
    for (int32_t m : ic.lm) {
        const uint8_t f = ic.fm[(size_t)m];
        if (f & DM_BASIC) {
            const int32_t C = s->owner[m];
            ((ic.fc[(size_t)C] & DC_CO) || s->acnt[C] == 0 ? basic_zero : basic_keep).push_back(m);
        }
    }
    // one upload: every list, 16-byte aligned pieces (the stream has drained:
    // the staging buffer is free)
    std::vector<int32_t> &H = ic.plan_stage;
    H.clear();
    auto put32 = [&](const std::vector<int32_t> &v) {
        const size_t at = H.size();
        H.insert(H.end(), v.begin(), v.end());
        while (H.size() % 4) H.push_back(0);
        return at;
    };
    auto put128 = [&](const std::vector<int4> &v) {
        const size_t at = H.size();
        for (const int4 &x : v) H.insert(H.end(), {x.x, x.y, x.z, x.w});
        return at;
    };
    auto put64 = [&](const std::vector<int2> &v) {
        const size_t at = H.size();
        for (const int2 &x : v) H.insert(H.end(), {x.x, x.y});
        while (H.size() % 4) H.push_back(0);
        return at;
    };
    std::vector<int32_t> wl(w_large), cl(c_large), basic(basic_zero);
    wl.insert(wl.end(), w_small.begin(), w_small.end());
    cl.insert(cl.end(), c_small.begin(), c_small.end());
    basic.insert(basic.end(), basic_keep.begin(), basic_keep.end());
    int in_run_off[5] = {0, 0, 0, 0, 0};
    for (int q = 0; q < 4; ++q) in_run_off[q + 1] = in_run_off[q] + in_cnt[q + 1];
    co_groups.insert(co_groups.end(), co_wide.begin(), co_wide.end());
    const size_t o_wl = put32(wl), o_cl = put32(cl), o_wm = put32(w_mid), o_cm = put32(c_mid),
                 o_basic = put32(basic), o_cos = put32(co_small), o_fin = put32(fin);
    const size_t o_if = put128(i_flag);
    const size_t o_cog = put64(co_groups);
    ic.d_plan.reserve(s->ctx, &s->bytes, (std::max<size_t>(H.size(), 4) + (size_t)in_run_off[4] + 4) * 4);
    if (!H.empty()) HIPCHK(hipMemcpyAsync(ic.d_plan.p, H.data(), H.size() * 4, hipMemcpyHostToDevice, st));
    // the four run groups side by side after the uploaded lists
    int32_t *runs_dev = ic.d_plan.as<int32_t>() + ((H.size() + 3) / 4) * 4;
    for (int q = 0; q < 4; ++q)
        if (in_cnt[q + 1])
            HIPCHK(hipMemcpyAsync(runs_dev + in_run_off[q], lists + (q + 1) * stride, (size_t)in_cnt[q + 1] * 4,
                                  hipMemcpyDeviceToDevice, st));
    if (!ic.plan_ev) HIPCHK(hipEventCreateWithFlags(&ic.plan_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ic.plan_ev, st));
    ic.plan_ev_set = true;
    const int32_t *D = ic.d_plan.as<int32_t>();
    DirtyPlan p;
    memset(&p, 0, sizeof(p));
    p.meth = s->d_meth.as<MethodAgg>();
    p.cls = s->d_cls.as<ClassAgg>();
    p.own_mask = s->d_own_mask.as<uint64_t>();
    p.w = map_out(s->w);
    p.cnt = map_out(s->cnt);
    p.in = map_out(s->in);
    p.w_list = D + o_wl;
    p.n_w = (int)wl.size();
    p.n_w_large = (int)w_large.size();
    p.c_list = D + o_cl;
    p.n_c = (int)cl.size();
    p.n_c_large = (int)c_large.size();
    p.w_mid = D + o_wm;
    p.n_w_mid = (int)w_mid.size();
    p.c_mid = D + o_cm;
    p.n_c_mid = (int)c_mid.size();
    {
        // the hash-table segments to rebuild: their own item and partition
        // lists (the layout's stay for the next full recompute), the map's
        // staging area and partition tables (work areas of either recompute)
        DevMap *dm[3] = {&s->w, &s->cnt, &s->in};
        p.big.np_max = 1;
        for (int q = 0; q < 3; ++q) {
            const BigHost &bh = ic.big[q];
            upload(ctx, &s->bytes, ic.d_big_items[q], bh.items, st);
            upload(ctx, &s->bytes, ic.d_big_parts[q], bh.parts, st);
            dm[q]->big_stage.reserve(ctx, &s->bytes, (size_t)std::max<int64_t>(bh.stage, 1) * sizeof(int2));
            dm[q]->big_bt.reserve(ctx, &s->bytes, (size_t)std::max<int64_t>(bh.bt, 1) * sizeof(int32_t));
            p.big.m[q] = BigMap{ic.d_big_items[q].as<BigItem>(), ic.d_big_parts[q].as<BigPart>(), (int)bh.items.size(),
                                (int)bh.parts.size(), dm[q]->big_stage.as<int2>(), dm[q]->big_bt.as<int32_t>(),
                                map_out(*dm[q])};
            p.big.np_max = std::max(p.big.np_max, bh.np_max);
        }
        p.big.lds_slots = big_lds_slots(BIG_CHUNK);
    }
    p.basic = D + o_basic;
    p.n_basic = (int)basic.size();
    p.n_basic_zero = (int)basic_zero.size();
    p.co_small = D + o_cos;
    p.n_co_small = (int)co_small.size();
    p.co_groups = reinterpret_cast<const int2 *>(D + o_cog);
    p.n_co_groups = (int)(co_groups.size() - co_wide.size());
    p.co_items = p.co_groups + p.n_co_groups;
    p.n_co_items = (int)co_wide.size();
    p.in_wave = lists + 5 * stride;
    p.n_in_wave = in_cnt[5];
    p.in_runs = runs_dev;
    for (int q = 0; q < 5; ++q) p.in_run_off[q] = in_run_off[q];
    p.in_flag = reinterpret_cast<const int4 *>(D + o_if);
    p.n_in_flag = (int)i_flag.size();
    p.fin = D + o_fin;
    p.n_fin = (int)fin.size();
    p.err = s->d_err.as<int>();
    p.timer = s->ctx->timer.enabled() ? &s->ctx->timer : nullptr;
    launch_dirty_metrics(dv, p, st);
    HIPCHK(hipGetLastError());
    if (cls_dst && s->c)
        HIPCHK(hipMemcpyAsync(cls_dst, s->d_cls.p, (size_t)s->c * sizeof(ClassAgg), hipMemcpyDeviceToDevice, st));
    if (meth_dst && s->n)
        HIPCHK(hipMemcpyAsync(meth_dst, s->d_meth.p, (size_t)s->n * sizeof(MethodAgg), hipMemcpyDeviceToDevice, st));
    ic.last_dirty = {(int64_t)fin.size(), (int64_t)(wl.size() + w_mid.size()) + ic.big[0].n_segs,
                     (int64_t)(cl.size() + c_mid.size()) + ic.big[1].n_segs,
                     (int64_t)(in_run_off[4] + in_cnt[5] + in_cnt[0]), (int64_t)basic.size()};
    clear_dirty(s);
}

}  // namespace

// mm_server_impl.h -- the request server of the C ABI (included by mm_api.hip,
// which it shares the engine with).
//
// Resident systems stay on the device between requests (the paper's motivation
// for analysing a system continuously while it evolves, Sec. I). Requests are
// queued; n_slots worker threads, each with its own HIP stream, take the first
// queued request whose system is idle, so requests on different systems run at
// the same time and their kernels overlap on the GPU, while requests on one
// system keep their submission order. A request that arrives while others run
// starts as soon as a slot is free (continuous batching). Requests are admitted
// by device memory: idle systems first give up their scoring scratch, then are
// evicted, least recently used first. An evicted system keeps its current state
// (edits and moves included) in host memory; the next request that names it
// reloads it first, inside that request, whose latency still counts from its
// submission. A load (or reload) that cannot fit waits while other requests
// hold memory and fails with MM_ENOMEM when nothing else is running.
// A request that runs out of memory while others run goes back to the queue
// until one of them finishes; alone, it is retried after reclaiming what idle
// systems hold, at most twice (an edit replaces rows, so applying it twice is
// the same as once). A load of an id that is resident replaces that system.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// owned copy of a system description
struct DescCopy {
    int32_t c = 0, n = 0, na = 0;
    std::vector<int32_t> mc, ac, ai, ci;
    std::vector<int64_t> ao, co;
    void take(const mm_system_desc *d) {
        if (!d || d->n_classes < 0 || d->n_methods < 0 || d->n_attrs < 0 || !d->acc_off || !d->call_off)
            fail(MM_EINVAL, "bad system description");
        c = d->n_classes;
        n = d->n_methods;
        na = d->n_attrs;
        if ((n && !d->method_class) || (na && !d->attr_class)) fail(MM_EINVAL, "NULL arrays in description");
        mc.assign(d->method_class, d->method_class + n);
        ac.assign(d->attr_class, d->attr_class + na);
        ao.assign(d->acc_off, d->acc_off + n + 1);
        co.assign(d->call_off, d->call_off + n + 1);
        if (ao[0] != 0 || co[0] != 0 || ao[n] < 0 || co[n] < 0) fail(MM_EINVAL, "bad offsets in description");
        if ((ao[n] && !d->acc_idx) || (co[n] && !d->call_idx)) fail(MM_EINVAL, "NULL rows in description");
        ai.assign(d->acc_idx, d->acc_idx + ao[n]);
        ci.assign(d->call_idx, d->call_idx + co[n]);
    }
    mm_system_desc desc() const {
        return mm_system_desc{c, n, na, mc.data(), ac.data(), ao.data(), ai.data(), co.data(), ci.data()};
    }
    // the current state of a system about to be freed (its host mirror: owners
    // after moves, rows after edits). The offsets are widened first, the only
    // step that can fail (then the system is left whole); the large arrays are
    // moved out, not copied.
    void take_state(mm_system *s) {
        std::vector<int64_t> o1(s->acc_off.begin(), s->acc_off.end()), o2(s->call_off.begin(), s->call_off.end());
        c = s->c;
        n = s->n;
        na = s->na;
        ao.swap(o1);
        co.swap(o2);
        mc = std::move(s->owner);
        ac = std::move(s->acls);
        ai = std::move(s->acc_idx);
        ci = std::move(s->call_idx);
    }
};

struct EditCopy {
    std::vector<int32_t> m, nc, ai, ci;
    std::vector<int64_t> ao, co;
    bool has_class = false;
    void take(const mm_edit_desc *e) {
        if (!e || e->k < 0 || !e->acc_off || !e->call_off) fail(MM_EINVAL, "bad edit description");
        const int32_t k = e->k;
        if (k && !e->method) fail(MM_EINVAL, "NULL edit methods");
        m.assign(e->method, e->method + k);
        has_class = e->new_class != nullptr;
        if (has_class) nc.assign(e->new_class, e->new_class + k);
        ao.assign(e->acc_off, e->acc_off + k + 1);
        co.assign(e->call_off, e->call_off + k + 1);
        if (ao[0] != 0 || co[0] != 0 || ao[k] < 0 || co[k] < 0) fail(MM_EINVAL, "bad edit offsets");
        if ((ao[k] && !e->acc_idx) || (co[k] && !e->call_idx)) fail(MM_EINVAL, "NULL edit rows");
        ai.assign(e->acc_idx, e->acc_idx + ao[k]);
        ci.assign(e->call_idx, e->call_idx + co[k]);
    }
    mm_edit_desc desc() const {
        return mm_edit_desc{(int32_t)m.size(), m.data(), has_class ? nc.data() : nullptr, ao.data(), ai.data(),
                            co.data(), ci.data()};
    }
};

struct Req {
    uint64_t ticket = 0;
    int32_t kind = 0, sys_id = 0;
    DescCopy load;
    EditCopy edit;
    int32_t cand_mode = MM_CAND_REFERENCED;
    std::vector<int32_t> cm, ct;
    uint32_t mask = MM_CBO | MM_LCOM_PQ;
    int32_t rule = MM_RULE_PARETO, keep_only = 1;
    int64_t est_bytes = 0;
    uint64_t wait_finish = 0;  // after running out of memory: start again once this many requests finished
    std::shared_ptr<DescCopy> reload;  // state of an evicted system to load before running the request
    bool settled = false;              // finished when taken from the queue (nothing runs on the device)
    bool heavy = false;                // a load or a reload: counted against the server's heavy_cap
    // result
    int32_t state = 0;  // 0 queued, 1 running, 2 done
    int32_t status = MM_OK;
    int32_t slot = -1;
    std::vector<mm_move_score> records;
    std::string error;
    double t_submit = 0, t_start = 0, t_end = 0;
};

struct Resident {
    mm_system *sys = nullptr;
    bool busy = false;
    double last_use = 0;
};

}  // namespace

struct mm_server {
    mm_context *ctx = nullptr;
    int32_t n_slots = 1, queue_cap = 1024;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    std::deque<std::shared_ptr<Req>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
    std::unordered_map<int32_t, Resident> systems;
    std::unordered_map<int32_t, std::shared_ptr<DescCopy>> swapped;  // evicted systems' states (host memory)
    uint64_t next_ticket = 1;
    int32_t running = 0;
    // loads and reloads (a whole system uploaded and its layout built) run on
    // at most heavy_cap slots at once, so edits and scores always have slots
    int32_t heavy_running = 0, heavy_cap = 1;
    uint64_t finished = 0;  // requests finished (any status)
    // statistics since the last reset
    std::vector<double> lat;
    int64_t submitted = 0, completed = 0, failed = 0, refused = 0, evicted = 0, records = 0, reloaded = 0;
    double t0 = 0;
};

namespace {

// device bytes a system of these sizes holds once resident: structure (rows,
// callers, membership), grouped-count tables (at most 4 slots of 8 bytes per
// reference), aggregates and per-buffer rounding -- an upper bound used for
// admission
int64_t estimate_bytes(const DescCopy &d) {
    const int64_t na = d.ao.back(), nc = d.co.back();
    return 40 * na + 72 * nc + 60 * (int64_t)d.n + 8 * (int64_t)d.na + 120 * (int64_t)d.c + (64 << 10);
}

bool fits(mm_context *ctx, int64_t need) {
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    return ctx->used + (uint64_t)std::max<int64_t>(need, 0) <= ctx->budget;
}

// Reclaim device memory until `need` more bytes fit the budget: first the
// scoring scratch of idle systems, then idle systems that no queued request
// names, least recently used first, then the idle system whose next queued
// request comes last; `keep` is never evicted. True if they fit.
bool make_room(mm_server *sv, int64_t need, int32_t keep, std::unique_lock<std::mutex> &) {
    mm_context *ctx = sv->ctx;
    if (!ctx->budget) return true;
    while (!fits(ctx, need)) {
        int32_t victim = -1;
        double oldest = 0;
        for (auto &kv : sv->systems) {
            if (kv.second.busy || !kv.second.sys || scratch_bytes(kv.second.sys) == 0) continue;
            if (victim < 0 || kv.second.last_use < oldest) {
                victim = kv.first;
                oldest = kv.second.last_use;
            }
        }
        if (victim >= 0) {
            release_scratch(sv->systems[victim].sys);
            continue;
        }
        for (auto &kv : sv->systems) {
            if (kv.second.busy || !kv.second.sys || kv.first == keep) continue;
            bool wanted = false;
            for (auto &q : sv->queue)
                if (q->sys_id == kv.first) { wanted = true; break; }
            if (wanted) continue;
            if (victim < 0 || kv.second.last_use < oldest) {
                victim = kv.first;
                oldest = kv.second.last_use;
            }
        }
        if (victim < 0) {
            // every idle system is named by a queued request: evict the one whose
            // next request comes last (its state is kept and reloaded then)
            size_t last = 0;
            for (auto &kv : sv->systems) {
                if (kv.second.busy || !kv.second.sys || kv.first == keep) continue;
                size_t at = 0;
                while (at < sv->queue.size() && sv->queue[at]->sys_id != kv.first) ++at;
                if (victim < 0 || at > last) {
                    victim = kv.first;
                    last = at;
                }
            }
        }
        if (victim < 0) return false;
        mm_system *vs = sv->systems[victim].sys;
        auto keep_state = std::make_shared<DescCopy>();
        keep_state->take_state(vs);  // a failure here leaves the system resident
        sv->swapped[victim] = std::move(keep_state);
        sv->systems.erase(victim);
        (void)mm_free_system(vs);
        sv->evicted++;
    }
    return true;
}

// device bytes a request needs beyond what its system already holds: scoring
// scratch (per method, per reference, per class and per candidate) and, for an
// edit, the growth of the structure and tables -- an upper bound for admission
int64_t work_bytes(const Req &r, mm_system *s) {
    const int64_t nref = (int64_t)s->acc_idx.size() + (int64_t)s->call_idx.size();
    int64_t cand = 0, grow = 0;
    if (r.kind == MM_REQ_EDIT) {
        cand = r.edit.ao.back() + r.edit.co.back();
        // the new rows spliced in on the device next to the old ones (with their
        // lengths and scans), and the sort that rebuilds the callers, all held
        // until the request ends
        grow = 112 * cand + 32 * (int64_t)s->n + 20 * nref;
    } else if (r.cand_mode == MM_CAND_EXPLICIT) {
        cand = (int64_t)r.cm.size();
    } else {
        cand = s->ref_version == s->version ? s->ref_count : nref;
    }
    const int64_t scratch = 48 * (int64_t)s->n + 12 * nref + 16 * (int64_t)s->c + 100 * cand + (64 << 10);
    return grow + std::max<int64_t>(scratch - scratch_bytes(s), 0);
}

// REFERENCED candidates of the given methods, (method, class) ascending
void referenced_of(mm_system *s, std::vector<int32_t> methods, std::vector<int32_t> &cm, std::vector<int32_t> &ct) {
    std::sort(methods.begin(), methods.end());
    std::vector<int32_t> cls;
    for (int32_t m : methods) {
        cls.clear();
        for (int32_t e = s->call_off[m]; e < s->call_off[m + 1]; ++e) cls.push_back(s->owner[s->call_idx[e]]);
        for (int32_t e = s->acc_off[m]; e < s->acc_off[m + 1]; ++e) cls.push_back(s->acls[s->acc_idx[e]]);
        std::sort(cls.begin(), cls.end());
        cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
        for (int32_t T : cls)
            if (T != s->owner[m]) {
                cm.push_back(m);
                ct.push_back(T);
            }
    }
}

void score_to_host(mm_system *s, const ScoreArgs &a, std::vector<mm_move_score> &out) {
    int64_t n = 0;
    score_impl(s, a, nullptr, false, 0, &n);
    out.resize((size_t)n);
    if (n) score_impl(s, a, out.data(), false, n, &n);
}

// Runs one request on the slot's stream. `sys` is the request's resident
// system; for a request on an evicted system it is set here, once reloaded.
void run_request(mm_server *sv, Req &r, int slot, mm_system *&sys) {
    hipStream_t st = sv->streams[slot];
    if (r.kind == MM_REQ_LOAD) {
        mm_system_desc d = r.load.desc();
        mm_system *s = nullptr;
        load_impl(sv->ctx, &d, &s, st);
        try {
            ensure_metrics(s);
            check_kernel_errors(s);
        } catch (...) {
            (void)mm_free_system(s);
            throw;
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        Resident &res = sv->systems[r.sys_id];
        res.sys = s;
        return;
    }
    if (r.reload) {
        // the system was evicted: load its kept state, then run the request on it
        mm_system_desc d = r.reload->desc();
        mm_system *s = nullptr;
        load_impl(sv->ctx, &d, &s, st);
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->systems[r.sys_id].sys = s;
        sv->reloaded++;
        sys = s;
        r.reload.reset();  // resident again: a retry of this request does not load it twice
    }
    sys->stream = st;
    if (r.kind == MM_REQ_EDIT) {
        mm_edit_desc e = r.edit.desc();
        apply_edit_impl(sys, &e);
        ensure_metrics(sys);
        std::vector<int32_t> cm, ct;
        referenced_of(sys, r.edit.m, cm, ct);
        ScoreArgs a{MM_CAND_EXPLICIT, cm.data(), ct.data(), (int64_t)cm.size(), r.mask, r.rule, r.keep_only};
        score_to_host(sys, a, r.records);
    } else if (r.kind == MM_REQ_SCORE) {
        ScoreArgs a{r.cand_mode, r.cm.data(), r.ct.data(), (int64_t)r.cm.size(), r.mask, r.rule, r.keep_only};
        score_to_host(sys, a, r.records);
    }
}

void worker(mm_server *sv, int slot) {
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        std::shared_ptr<Req> job;
        mm_system *sys = nullptr;
        // ids with an earlier queued request that cannot start yet: their later
        // requests wait too, so each system sees its requests in order
        std::vector<int32_t> held;
        auto is_held = [&](int32_t id) { return std::find(held.begin(), held.end(), id) != held.end(); };
        auto stuck = sv->queue.end();  // first load that does not fit
        for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
            Req &r = **it;
            if (is_held(r.sys_id)) continue;
            if (r.wait_finish > sv->finished && sv->running > 0) {  // ran out of memory: wait for a finish
                held.push_back(r.sys_id);
                continue;
            }
            auto f = sv->systems.find(r.sys_id);
            if (r.kind == MM_REQ_LOAD) {
                if (sv->heavy_running >= sv->heavy_cap) {  // waits for a slot for long requests
                    held.push_back(r.sys_id);
                    continue;
                }
                sv->swapped.erase(r.sys_id);  // a load replaces a kept state
                if (f != sv->systems.end()) {
                    if (f->second.busy || !f->second.sys) {  // running: wait for it
                        held.push_back(r.sys_id);
                        continue;
                    }
                    (void)mm_free_system(f->second.sys);  // replaced by this load
                    sv->systems.erase(f);
                }
                if (!make_room(sv, r.est_bytes, -1, lk)) {
                    // wait: running or runnable requests will release their systems
                    if (stuck == sv->queue.end()) stuck = it;
                    held.push_back(r.sys_id);
                    continue;
                }
                job = *it;
                sv->queue.erase(it);
                if (job->status == MM_OK) sv->systems[job->sys_id] = Resident{nullptr, true, now_ms()};
                job->heavy = true;
                sv->heavy_running++;
                break;
            }
            if (f == sv->systems.end()) {
                auto k = sv->swapped.find(r.sys_id);
                if (k != sv->swapped.end() && r.kind == MM_REQ_FREE) {  // an evicted system: drop its state
                    job = *it;
                    sv->queue.erase(it);
                    sv->swapped.erase(k);
                    job->settled = true;
                    break;
                }
                if (k != sv->swapped.end()) {
                    // evicted: reload it within this request, once it fits
                    if (sv->heavy_running >= sv->heavy_cap) {
                        held.push_back(r.sys_id);
                        continue;
                    }
                    if (!make_room(sv, estimate_bytes(*k->second), -1, lk)) {
                        if (stuck == sv->queue.end()) stuck = it;
                        held.push_back(r.sys_id);
                        continue;
                    }
                    job = *it;
                    sv->queue.erase(it);
                    job->reload = k->second;
                    sv->swapped.erase(k);
                    sv->systems[job->sys_id] = Resident{nullptr, true, now_ms()};
                    job->heavy = true;
                    sv->heavy_running++;
                    break;
                }
                // no earlier load is queued or running
                job = *it;
                sv->queue.erase(it);
                job->status = MM_ENOTFOUND;
                job->error = "no resident system with this id";
                break;
            }
            if (f->second.busy || !f->second.sys) {
                held.push_back(r.sys_id);
                continue;
            }
            job = *it;
            sv->queue.erase(it);
            f->second.busy = true;
            sys = f->second.sys;
            if (job->kind != MM_REQ_FREE) (void)make_room(sv, work_bytes(*job, sys), job->sys_id, lk);
            break;
        }
        if (!job && stuck != sv->queue.end() && sv->running == 0) {
            // nothing runs and nothing else can start: no memory will be freed
            job = *stuck;
            sv->queue.erase(stuck);
            job->status = MM_ENOMEM;
            job->error = "system does not fit the memory budget";
        }
        if (!job) {
            if (sv->stopping && sv->queue.empty()) return;
            sv->cv_work.wait(lk);
            continue;
        }
        job->state = 1;
        job->slot = slot;
        job->t_start = now_ms();
        sv->running++;
        bool requeue = false;
        // a request whose evicted system could not be reloaded gives its kept
        // state back, so that a later request can try again
        auto give_back_state = [&] {
            if (!job->reload) return;
            sv->swapped[job->sys_id] = job->reload;
            job->reload.reset();
            auto f = sv->systems.find(job->sys_id);
            if (f != sv->systems.end() && !f->second.sys) sv->systems.erase(f);
        };
        for (int attempt = 0; attempt < 4 && job->status == MM_OK && !job->settled; ++attempt) {
            lk.unlock();
            bool device_oom = false;
            // blocks released while this request's kernels may still run go to
            // the shared pool only once the slot's stream has drained
            std::vector<std::pair<size_t, void *>> deferred;
            tl_defer = &deferred;
            try {
                run_request(sv, *job, slot, sys);
            } catch (const MmError &e) {
                job->status = e.code;
                job->error = e.msg;
                device_oom = e.code == MM_ENOMEM;
            } catch (const std::bad_alloc &) {
                job->status = MM_ENOMEM;
                job->error = "host allocation failed";
            } catch (...) {
                job->status = MM_EINTERNAL;
                job->error = "unexpected internal error";
            }
            (void)hipStreamSynchronize(sv->streams[slot]);
            tl_defer = nullptr;
            flush_deferred(sv->ctx, deferred);
            lk.lock();
            if (!device_oom) break;
            // out of memory while other requests run (sv->running counts this
            // one too): they will release what they hold, so wait for one of them
            if (sv->running > 1) {
                requeue = true;
                break;
            }
            if (attempt == 3) break;  // alone, with every idle system evicted: MM_ENOMEM
            // alone: reclaim what idle systems hold, a step more on each attempt
            // (twice the estimate, then four times, then everything idle), and
            // try again
            const int64_t need = job->kind == MM_REQ_LOAD ? job->est_bytes
                                 : sys ? work_bytes(*job, sys) : estimate_bytes(*job->reload);
            const int64_t want = attempt == 0 ? 2 * need : attempt == 1 ? 4 * need : (int64_t)1 << 62;
            if (!make_room(sv, want, job->sys_id, lk) && attempt < 2)
                (void)make_room(sv, need, job->sys_id, lk);
            job->status = MM_OK;
            job->error.clear();
            job->records.clear();
        }
        sv->running--;
        if (job->heavy) {
            sv->heavy_running--;
            job->heavy = false;
        }
        if (requeue) {
            // out of memory while other requests hold it: back to the front of the
            // queue until one of them finishes (an edit replaces rows, so running
            // it again is safe)
            job->status = MM_OK;
            job->error.clear();
            job->records.clear();
            job->state = 0;
            job->slot = -1;
            job->wait_finish = sv->finished + 1;
            give_back_state();
            auto f = sv->systems.find(job->sys_id);
            if (job->kind == MM_REQ_LOAD) {
                if (f != sv->systems.end() && !f->second.sys) sv->systems.erase(f);
            } else if (f != sv->systems.end()) {
                f->second.busy = false;
            }
            sv->queue.push_front(job);
            sv->cv_work.notify_all();
            continue;
        }
        sv->finished++;
        give_back_state();
        if (sys && job->kind != MM_REQ_FREE) release_scratch(sys);  // pooled: the next request of any system reuses it
        job->t_end = now_ms();
        job->state = 2;
        if (job->kind == MM_REQ_LOAD) {
            auto f = sv->systems.find(job->sys_id);
            if (f != sv->systems.end()) {
                if (job->status != MM_OK || !f->second.sys) sv->systems.erase(f);
                else f->second.busy = false;
            }
        } else if (sys) {
            auto f = sv->systems.find(job->sys_id);
            if (job->kind == MM_REQ_FREE && job->status == MM_OK) {
                (void)mm_free_system(sys);
                sv->systems.erase(f);
            } else {
                f->second.busy = false;
                f->second.last_use = job->t_end;
            }
        }
        if (job->status == MM_OK) {
            sv->completed++;
            sv->records += (int64_t)job->records.size();
            sv->lat.push_back(job->t_end - job->t_submit);
        } else {
            sv->failed++;
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
    return v[i];
}

}  // namespace

extern "C" {

mm_status mm_server_create(const mm_server_opts *o, mm_server **out) {
    return guarded([&] {
        if (!o || !out) fail(MM_EINVAL, "NULL argument");
        if (o->n_slots < 1 || o->n_slots > 16) fail(MM_EINVAL, "n_slots must be in [1, 16]");
        if (o->queue_capacity < 1) fail(MM_EINVAL, "queue_capacity must be positive");
        std::unique_ptr<mm_server> sv(new mm_server());
        mm_context *ctx = nullptr;
        mm_status rc = mm_context_create(o->device, nullptr, o->mem_budget_bytes, &ctx);
        if (rc != MM_OK) fail(rc, g_last_error);
        sv->ctx = ctx;
        sv->n_slots = o->n_slots;
        sv->heavy_cap = std::max(1, o->n_slots / 2);
        sv->queue_cap = o->queue_capacity;
        for (int i = 0; i < o->n_slots; ++i) {
            hipStream_t st;
            HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            sv->streams.push_back(st);
        }
        sv->t0 = now_ms();
        for (int i = 0; i < o->n_slots; ++i) sv->workers.emplace_back(worker, sv.get(), i);
        *out = sv.release();
    });
}

mm_status mm_server_destroy(mm_server *sv) {
    return guarded([&] {
        if (!sv) fail(MM_EINVAL, "server is NULL");
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stopping = true;
        }
        sv->cv_work.notify_all();
        for (auto &t : sv->workers) t.join();
        (void)hipSetDevice(sv->ctx->device);
        for (auto &kv : sv->systems)
            if (kv.second.sys) (void)mm_free_system(kv.second.sys);
        for (auto st : sv->streams) (void)hipStreamDestroy(st);
        (void)mm_context_destroy(sv->ctx);
        delete sv;
    });
}

mm_status mm_server_submit(mm_server *sv, const mm_request *q, uint64_t *ticket) {
    return guarded([&] {
        if (!sv || !q || !ticket) fail(MM_EINVAL, "NULL argument");
        auto r = std::make_shared<Req>();
        r->kind = q->kind;
        r->sys_id = q->system_id;
        r->cand_mode = q->cand_mode;
        r->mask = q->metric_mask;
        r->rule = q->rule;
        r->keep_only = q->keep_only;
        if (q->kind == MM_REQ_LOAD) {
            r->load.take(q->load);
            r->est_bytes = estimate_bytes(r->load);
        } else if (q->kind == MM_REQ_EDIT) {
            r->edit.take(q->edit);
        } else if (q->kind == MM_REQ_SCORE) {
            if (q->cand_mode == MM_CAND_EXPLICIT) {
                if (q->n_cand < 0 || (q->n_cand && (!q->cand_method || !q->cand_class)))
                    fail(MM_EINVAL, "bad explicit candidates");
                r->cm.assign(q->cand_method, q->cand_method + q->n_cand);
                r->ct.assign(q->cand_class, q->cand_class + q->n_cand);
            }
        } else if (q->kind != MM_REQ_FREE) {
            fail(MM_EINVAL, "unknown request kind");
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if ((int32_t)sv->queue.size() >= sv->queue_cap) {
            sv->refused++;
            fail(MM_EBUSY, "request queue is full");
        }
        r->ticket = sv->next_ticket++;
        r->t_submit = now_ms();
        sv->queue.push_back(r);
        sv->reqs[r->ticket] = r;
        sv->submitted++;
        *ticket = r->ticket;
        sv->cv_work.notify_one();
    });
}

mm_status mm_server_wait(mm_server *sv, uint64_t ticket, int32_t timeout_ms, mm_result *out) {
    return guarded([&] {
        if (!sv || !out) fail(MM_EINVAL, "NULL argument");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) fail(MM_ENOTFOUND, "unknown ticket");
        std::shared_ptr<Req> r = it->second;
        auto done = [&] { return r->state == 2; };
        if (timeout_ms < 0) sv->cv_done.wait(lk, done);
        else sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
        out->state = r->state;
        out->status = r->status;
        out->slot = r->slot;
        out->n_records = r->state == 2 ? (int64_t)r->records.size() : 0;
        out->records = r->state == 2 && !r->records.empty() ? r->records.data() : nullptr;
        out->submit_ms = r->t_submit - sv->t0;
        out->start_ms = r->state >= 1 ? r->t_start - sv->t0 : 0;
        out->end_ms = r->state == 2 ? r->t_end - sv->t0 : 0;
        out->error = r->state == 2 && r->status != MM_OK ? r->error.c_str() : "";
        if (r->state != 2) fail(MM_EBUSY, "request not finished");
    });
}

mm_status mm_server_release(mm_server *sv, uint64_t ticket) {
    return guarded([&] {
        if (!sv) fail(MM_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) fail(MM_ENOTFOUND, "unknown ticket");
        if (it->second->state != 2) fail(MM_EBUSY, "request not finished");
        sv->reqs.erase(it);
    });
}

mm_status mm_server_drain(mm_server *sv) {
    return guarded([&] {
        if (!sv) fail(MM_EINVAL, "server is NULL");
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->queue.empty() && sv->running == 0; });
    });
}

mm_status mm_server_stats(mm_server *sv, int32_t reset, mm_server_counters *out) {
    return guarded([&] {
        if (!sv || !out) fail(MM_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        out->submitted = sv->submitted;
        out->completed = sv->completed;
        out->failed = sv->failed;
        out->refused = sv->refused;
        out->evicted = sv->evicted;
        out->reloaded = sv->reloaded;
        out->records = sv->records;
        out->p50_ms = percentile(sv->lat, 0.50);
        out->p99_ms = percentile(sv->lat, 0.99);
        out->max_ms = sv->lat.empty() ? 0 : *std::max_element(sv->lat.begin(), sv->lat.end());
        double sum = 0;
        for (double v : sv->lat) sum += v;
        out->mean_ms = sv->lat.empty() ? 0 : sum / sv->lat.size();
        out->elapsed_s = (now_ms() - sv->t0) / 1000.0;
        out->resident = (int32_t)sv->systems.size();
        out->queued = (int32_t)sv->queue.size();
        {
            std::lock_guard<std::mutex> lk2(sv->ctx->mem_mu);
            out->device_bytes = sv->ctx->used;
            out->peak_bytes = sv->ctx->peak;
            if (reset) sv->ctx->peak = sv->ctx->used;
        }
        if (reset) {
            sv->lat.clear();
            sv->submitted = sv->completed = sv->failed = sv->refused = sv->evicted = sv->records = 0;
            sv->reloaded = 0;
            sv->t0 = now_ms();
        }
    });
}

}  // extern "C"

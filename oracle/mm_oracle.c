/*
 * mm_oracle.c -- CPU oracle for the modularity metrics and Move Method scores.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product (the HIP
 * library) never calls it, and the two share no code, headers or tables.
 *
 * Everything here is the plain definition, written out with stamped "sets" over
 * ids, single-threaded, integer only:
 *
 *   fan-in(m)   number of methods calling m                 (Sec. II-A)
 *   fan-out(m)  number of methods m calls                   (Sec. II-A)
 *   CBO(C)      number of other classes that C's methods use, through method
 *               calls or attribute accesses (efferent)      (Sec. II-B)
 *   LCOM(C)     pairs of C's methods that share no attribute of C, minus the
 *               pairs that share at least one (the original form, Sec. II-B),
 *               returned as P and Q; unclamped
 *   LCOM_HS(C)  1 - mean over C's methods of (own attributes used / a_C), the
 *               later ratio form of Sec. II-B, kept as the exact fraction
 *               (n*a - U) / (n*a), (0,1) when n*a = 0
 *   RFC(C)      |M_C union calls(M_C)| (one level, CK suite named in Sec. II-B)
 *
 * A Move Method (m -> T) is scored by its definition (Sec. III-A, and Sec. IV-C
 * which re-runs the metric functions on the changed membership): the metrics of
 * a class after moving m (attributes stay, ids stay) minus the metrics before.
 * The scorer re-evaluates the origin S, the destination T and every class that
 * owns a caller of m; a separate brute-force check (the test suite re-running
 * orc_metrics on the moved system) pins that no other class changes.
 *
 * Readings where the paper is silent: rows are sets (duplicates ignored); a
 * self-call is kept (counts in fan-in/out, is intra-class for CBO/RFC); only
 * attributes of C count for either LCOM form; P = Q = 0 when n < 2.
 *
 * Similarity (Sec. II-A): the properties of a method are the methods it calls
 * and the attributes it accesses (as sets; a self-call is a property like any
 * other call); the Jaccard similarity of two methods is |shared| / |union|, 0
 * when the union is empty. orc_similarity lists every pair m1 < m2 with a
 * shared property, with the two sizes, by comparing each pair's sets.
 *
 * Suggestion rules (Sec. III-A, Sec. IV-A, abstract): lower is better for every
 * metric; "improve" means delta < 0, "worsen" delta > 0.
 *   PARETO     every affected (class, masked metric) has delta <= 0 and one < 0
 *   PAPER_LCOM every masked LCOM form improves in both origin and destination
 *   PAPER_CBO  origin CBO lowered, destination CBO not higher, no caller class
 *              CBO higher
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_classes, n_methods, n_attrs;
    const int32_t *method_class;
    const int32_t *attr_class;
    const int64_t *acc_off;
    const int32_t *acc_idx;
    const int64_t *call_off;
    const int32_t *call_idx;
} orc_sys;

typedef struct {
    int32_t n_methods, n_attrs, cbo, rfc;
    int64_t lcom_p, lcom_q, hs_num, hs_den;
} orc_class;

typedef struct {
    int32_t fan_in, fan_out, own_attr_uses, own_coaccess_partners;
} orc_method;

typedef struct {
    int32_t method, src, dst;
    int32_t d_cbo_src, d_cbo_dst, d_rfc_src, d_rfc_dst;
    int32_t n_caller_cls, n_caller_worse, n_caller_better;
    int32_t keep, pad;
    int64_t d_lcom_src, d_lcom_dst;
    int64_t hs_num_src, hs_den_src, hs_num_dst, hs_den_dst;
} orc_move;

enum { ORC_CBO = 1, ORC_LCOM_PQ = 2, ORC_LCOM_HS = 4, ORC_RFC = 8 };
enum { ORC_PARETO = 0, ORC_PAPER_LCOM = 1, ORC_PAPER_CBO = 2 };
enum { ORC_EXPLICIT = 0, ORC_ALL = 1, ORC_REFERENCED = 2 };

/* stamped sets: an id is "in" the set iff its mark equals the current stamp */
typedef struct {
    const orc_sys *s;
    const int32_t *owner;   /* class of each method (may differ from the input after a move) */
    int32_t *attrs_of;      /* a_C per class */
    int32_t *mk_cls, *mk_m, *mk_a;
    int32_t st_cls, st_m, st_a;
} orc_ctx;

static int ctx_init(orc_ctx *x, const orc_sys *s, const int32_t *owner) {
    x->s = s;
    x->owner = owner;
    x->attrs_of = (int32_t *)calloc((size_t)s->n_classes + 1, sizeof(int32_t));
    x->mk_cls = (int32_t *)calloc((size_t)s->n_classes + 1, sizeof(int32_t));
    x->mk_m = (int32_t *)calloc((size_t)s->n_methods + 1, sizeof(int32_t));
    x->mk_a = (int32_t *)calloc((size_t)s->n_attrs + 1, sizeof(int32_t));
    if (!x->attrs_of || !x->mk_cls || !x->mk_m || !x->mk_a) return -1;
    for (int32_t a = 0; a < s->n_attrs; ++a) x->attrs_of[s->attr_class[a]]++;
    x->st_cls = x->st_m = x->st_a = 0;
    return 0;
}

static void ctx_free(orc_ctx *x) {
    free(x->attrs_of);
    free(x->mk_cls);
    free(x->mk_m);
    free(x->mk_a);
}

/* Do methods i and j access a common attribute that belongs to class C? */
static int share_attr(orc_ctx *x, int32_t C, int32_t i, int32_t j) {
    const orc_sys *s = x->s;
    int32_t st = ++x->st_a;
    for (int64_t e = s->acc_off[i]; e < s->acc_off[i + 1]; ++e) {
        int32_t a = s->acc_idx[e];
        if (s->attr_class[a] == C) x->mk_a[a] = st;
    }
    for (int64_t e = s->acc_off[j]; e < s->acc_off[j + 1]; ++e) {
        int32_t a = s->acc_idx[e];
        if (s->attr_class[a] == C && x->mk_a[a] == st) return 1;
    }
    return 0;
}

/* |acc(y) intersect A_C| with acc(y) read as a set */
static int32_t own_uses(orc_ctx *x, int32_t C, int32_t y) {
    const orc_sys *s = x->s;
    int32_t st = ++x->st_a, n = 0;
    for (int64_t e = s->acc_off[y]; e < s->acc_off[y + 1]; ++e) {
        int32_t a = s->acc_idx[e];
        if (s->attr_class[a] == C && x->mk_a[a] != st) {
            x->mk_a[a] = st;
            ++n;
        }
    }
    return n;
}

/* CBO of class C whose methods are `mem[0..n)`, under the current owner array */
static int32_t class_cbo(orc_ctx *x, int32_t C, const int32_t *mem, int32_t n) {
    const orc_sys *s = x->s;
    int32_t st = ++x->st_cls, cbo = 0;
    for (int32_t k = 0; k < n; ++k) {
        int32_t y = mem[k];
        for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
            int32_t D = x->owner[s->call_idx[e]];
            if (D != C && x->mk_cls[D] != st) { x->mk_cls[D] = st; ++cbo; }
        }
        for (int64_t e = s->acc_off[y]; e < s->acc_off[y + 1]; ++e) {
            int32_t D = s->attr_class[s->acc_idx[e]];
            if (D != C && x->mk_cls[D] != st) { x->mk_cls[D] = st; ++cbo; }
        }
    }
    return cbo;
}

/* All class metrics of class C whose methods are mem[0..n). If `rnz` is given,
 * rnz[k] receives the number of other methods of C sharing an attribute of C
 * with mem[k]. */
static void class_eval(orc_ctx *x, int32_t C, const int32_t *mem, int32_t n,
                       orc_class *out, int32_t *rnz) {
    const orc_sys *s = x->s;
    int64_t a = x->attrs_of[C];
    int64_t U = 0, Q = 0;
    for (int32_t k = 0; k < n; ++k) U += own_uses(x, C, mem[k]);
    if (rnz) for (int32_t k = 0; k < n; ++k) rnz[k] = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (share_attr(x, C, mem[i], mem[j])) {
                ++Q;
                if (rnz) { rnz[i]++; rnz[j]++; }
            }
    int64_t pairs = (int64_t)n * (n - 1) / 2;
    out->n_methods = n;
    out->n_attrs = (int32_t)a;
    out->lcom_q = Q;
    out->lcom_p = pairs - Q;
    if ((int64_t)n * a == 0) {
        out->hs_num = 0;
        out->hs_den = 1;
    } else {
        out->hs_num = (int64_t)n * a - U;
        out->hs_den = (int64_t)n * a;
    }
    out->cbo = class_cbo(x, C, mem, n);
    /* RFC: the methods of C plus every method they call */
    int32_t st = ++x->st_m, rfc = 0;
    for (int32_t k = 0; k < n; ++k)
        if (x->mk_m[mem[k]] != st) { x->mk_m[mem[k]] = st; ++rfc; }
    for (int32_t k = 0; k < n; ++k) {
        int32_t y = mem[k];
        for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
            int32_t t = s->call_idx[e];
            if (x->mk_m[t] != st) { x->mk_m[t] = st; ++rfc; }
        }
    }
    out->rfc = rfc;
}

/* members of every class, in method id order */
typedef struct { int32_t *off, *idx; } orc_members;

static int members_build(const orc_sys *s, const int32_t *owner, orc_members *M) {
    int32_t c = s->n_classes, nm = s->n_methods;
    M->off = (int32_t *)calloc((size_t)c + 1, sizeof(int32_t));
    M->idx = (int32_t *)malloc(((size_t)nm + 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)calloc((size_t)c + 1, sizeof(int32_t));
    if (!M->off || !M->idx || !fill) { free(fill); return -1; }
    for (int32_t m = 0; m < nm; ++m) M->off[owner[m] + 1]++;
    for (int32_t k = 0; k < c; ++k) M->off[k + 1] += M->off[k];
    for (int32_t m = 0; m < nm; ++m) M->idx[M->off[owner[m]] + fill[owner[m]]++] = m;
    free(fill);
    return 0;
}

static void members_free(orc_members *M) { free(M->off); free(M->idx); }

/* ------------------------------------------------------------------------ */

int orc_metrics(const orc_sys *s, orc_class *out_cls, orc_method *out_m) {
    orc_ctx x;
    orc_members M;
    if (ctx_init(&x, s, s->method_class) || members_build(s, s->method_class, &M)) return -1;
    int32_t *rnz = (int32_t *)malloc(((size_t)s->n_methods + 1) * sizeof(int32_t));
    if (!rnz) return -1;
    for (int32_t C = 0; C < s->n_classes; ++C) {
        orc_class tmp;
        int32_t n = M.off[C + 1] - M.off[C];
        class_eval(&x, C, M.idx + M.off[C], n, out_cls ? &out_cls[C] : &tmp, rnz + M.off[C]);
    }
    if (out_m) {
        for (int32_t m = 0; m < s->n_methods; ++m) {
            out_m[m].fan_in = 0;
            out_m[m].fan_out = 0;
        }
        for (int32_t y = 0; y < s->n_methods; ++y) {
            int32_t st = ++x.st_m;
            for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
                int32_t t = s->call_idx[e];
                if (x.mk_m[t] != st) {
                    x.mk_m[t] = st;
                    out_m[y].fan_out++;
                    out_m[t].fan_in++;
                }
            }
            out_m[y].own_attr_uses = own_uses(&x, s->method_class[y], y);
        }
        for (int32_t C = 0; C < s->n_classes; ++C)
            for (int32_t k = M.off[C]; k < M.off[C + 1]; ++k)
                out_m[M.idx[k]].own_coaccess_partners = rnz[k];
    }
    free(rnz);
    members_free(&M);
    ctx_free(&x);
    return 0;
}

static int cmp_class(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Candidate moves. ALL: every (m, T != cls(m)); REFERENCED: T among the owners of
 * what m calls or accesses, T != cls(m). Both in (m ascending, T ascending)
 * order. Returns the number of candidates; writes at most `cap` of them. */
int64_t orc_candidates(const orc_sys *s, int32_t mode, int32_t *out_m, int32_t *out_t, int64_t cap) {
    int64_t n = 0;
    int32_t c = s->n_classes;
    if (mode == ORC_ALL) {
        for (int32_t m = 0; m < s->n_methods; ++m)
            for (int32_t T = 0; T < c; ++T) {
                if (T == s->method_class[m]) continue;
                if (n < cap) { out_m[n] = m; out_t[n] = T; }
                ++n;
            }
        return n;
    }
    if (mode != ORC_REFERENCED) return -1;
    /* the classes a method references, collected in a list and then taken in
     * ascending order (sorting the list instead of scanning every class id) */
    char *used = (char *)calloc((size_t)c + 1, 1);
    int64_t longest = 0;
    for (int32_t m = 0; m < s->n_methods; ++m) {
        int64_t len = (s->call_off[m + 1] - s->call_off[m]) + (s->acc_off[m + 1] - s->acc_off[m]);
        if (len > longest) longest = len;
    }
    int32_t *list = (int32_t *)malloc(((size_t)longest + 1) * sizeof(int32_t));
    if (!used || !list) { free(used); free(list); return -1; }
    for (int32_t m = 0; m < s->n_methods; ++m) {
        int32_t k = 0;
        used[s->method_class[m]] = 1; /* never a destination */
        for (int64_t e = s->call_off[m]; e < s->call_off[m + 1]; ++e) {
            int32_t D = s->method_class[s->call_idx[e]];
            if (!used[D]) { used[D] = 1; list[k++] = D; }
        }
        for (int64_t e = s->acc_off[m]; e < s->acc_off[m + 1]; ++e) {
            int32_t D = s->attr_class[s->acc_idx[e]];
            if (!used[D]) { used[D] = 1; list[k++] = D; }
        }
        qsort(list, (size_t)k, sizeof(int32_t), cmp_class);
        for (int32_t q = 0; q < k; ++q) {
            if (n < cap) { out_m[n] = m; out_t[n] = list[q]; }
            ++n;
            used[list[q]] = 0;
        }
        used[s->method_class[m]] = 0;
    }
    free(list);
    free(used);
    return n;
}

static int sgn64(int64_t v) { return (v > 0) - (v < 0); }

/* sign of (num1/den1 - num0/den0), both denominators positive */
static int frac_delta_sign(int64_t num0, int64_t den0, int64_t num1, int64_t den1) {
    __int128 l = (__int128)num1 * den0, r = (__int128)num0 * den1;
    return (l > r) - (l < r);
}

static int32_t keep_rule(const orc_move *r, const orc_class *bs, const orc_class *bt,
                         uint32_t mask, int32_t rule) {
    int hs_s = frac_delta_sign(bs->hs_num, bs->hs_den, r->hs_num_src, r->hs_den_src);
    int hs_t = frac_delta_sign(bt->hs_num, bt->hs_den, r->hs_num_dst, r->hs_den_dst);
    if (rule == ORC_PAPER_LCOM) {
        int ok = 1;
        if (mask & ORC_LCOM_PQ) ok = ok && r->d_lcom_src < 0 && r->d_lcom_dst < 0;
        if (mask & ORC_LCOM_HS) ok = ok && hs_s < 0 && hs_t < 0;
        return ok;
    }
    if (rule == ORC_PAPER_CBO)
        return r->d_cbo_src < 0 && r->d_cbo_dst <= 0 && r->n_caller_worse == 0;
    /* PARETO */
    int worse = 0, better = 0;
    int sg[8], k = 0;
    if (mask & ORC_CBO) {
        sg[k++] = sgn64(r->d_cbo_src);
        sg[k++] = sgn64(r->d_cbo_dst);
        if (r->n_caller_worse > 0) worse = 1;
        if (r->n_caller_better > 0) better = 1;
    }
    if (mask & ORC_LCOM_PQ) { sg[k++] = sgn64(r->d_lcom_src); sg[k++] = sgn64(r->d_lcom_dst); }
    if (mask & ORC_LCOM_HS) { sg[k++] = hs_s; sg[k++] = hs_t; }
    if (mask & ORC_RFC) { sg[k++] = sgn64(r->d_rfc_src); sg[k++] = sgn64(r->d_rfc_dst); }
    for (int i = 0; i < k; ++i) {
        if (sg[i] > 0) worse = 1;
        if (sg[i] < 0) better = 1;
    }
    return !worse && better;
}

/* Score explicit candidates by re-evaluating the changed classes after each
 * move. Returns 0, or -1 on a bad argument (T == S, id out of range, bad rule). */
int orc_score(const orc_sys *s, int64_t n_cand, const int32_t *cm, const int32_t *ct,
              uint32_t mask, int32_t rule, orc_move *out) {
    if (rule < 0 || rule > 2 || (mask & ~15u)) return -1;
    if (rule == ORC_PAPER_LCOM && !(mask & (ORC_LCOM_PQ | ORC_LCOM_HS))) return -1;
    if (rule == ORC_PAPER_CBO && !(mask & ORC_CBO)) return -1;
    int32_t c = s->n_classes, nm = s->n_methods;
    int32_t *owner = (int32_t *)malloc(((size_t)nm + 1) * sizeof(int32_t));
    if (!owner) return -1;
    memcpy(owner, s->method_class, (size_t)nm * sizeof(int32_t));
    orc_ctx x;
    orc_members M;
    if (ctx_init(&x, s, owner) || members_build(s, s->method_class, &M)) return -1;
    orc_class *before = (orc_class *)malloc(((size_t)c + 1) * sizeof(orc_class));
    /* callers of every method (a caller listed once per distinct callee) */
    int32_t *cal_off = (int32_t *)calloc((size_t)nm + 2, sizeof(int32_t));
    int64_t nnz = s->call_off[nm];
    int32_t *cal_idx = (int32_t *)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    int32_t *buf = (int32_t *)malloc(((size_t)nm + 2) * sizeof(int32_t));
    int32_t *seen = (int32_t *)calloc((size_t)c + 1, sizeof(int32_t));
    if (!before || !cal_off || !cal_idx || !buf || !seen) return -1;
    for (int32_t C = 0; C < c; ++C)
        class_eval(&x, C, M.idx + M.off[C], M.off[C + 1] - M.off[C], &before[C], NULL);
    for (int32_t y = 0; y < nm; ++y) {
        int32_t st = ++x.st_m;
        for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
            int32_t t = s->call_idx[e];
            if (x.mk_m[t] != st) { x.mk_m[t] = st; cal_off[t + 1]++; }
        }
    }
    for (int32_t t = 0; t < nm; ++t) cal_off[t + 1] += cal_off[t];
    {
        int32_t *fill = (int32_t *)calloc((size_t)nm + 1, sizeof(int32_t));
        for (int32_t y = 0; y < nm; ++y) {
            int32_t st = ++x.st_m;
            for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
                int32_t t = s->call_idx[e];
                if (x.mk_m[t] != st) { x.mk_m[t] = st; cal_idx[cal_off[t] + fill[t]++] = y; }
            }
        }
        free(fill);
    }
    int32_t stamp = 0, rc = 0;
    for (int64_t k = 0; k < n_cand; ++k) {
        int32_t m = cm[k], T = ct[k];
        if (m < 0 || m >= nm || T < 0 || T >= c || T == s->method_class[m]) { rc = -1; break; }
        int32_t S = s->method_class[m];
        orc_move *r = &out[k];
        memset(r, 0, sizeof(*r));
        r->method = m; r->src = S; r->dst = T;
        owner[m] = T;
        /* S without m */
        int32_t n = 0;
        for (int32_t q = M.off[S]; q < M.off[S + 1]; ++q) if (M.idx[q] != m) buf[n++] = M.idx[q];
        orc_class aS, aT;
        class_eval(&x, S, buf, n, &aS, NULL);
        /* T with m */
        n = 0;
        for (int32_t q = M.off[T]; q < M.off[T + 1]; ++q) buf[n++] = M.idx[q];
        buf[n++] = m;
        class_eval(&x, T, buf, n, &aT, NULL);
        r->d_cbo_src = aS.cbo - before[S].cbo;
        r->d_cbo_dst = aT.cbo - before[T].cbo;
        r->d_rfc_src = aS.rfc - before[S].rfc;
        r->d_rfc_dst = aT.rfc - before[T].rfc;
        r->d_lcom_src = (aS.lcom_p - aS.lcom_q) - (before[S].lcom_p - before[S].lcom_q);
        r->d_lcom_dst = (aT.lcom_p - aT.lcom_q) - (before[T].lcom_p - before[T].lcom_q);
        r->hs_num_src = aS.hs_num; r->hs_den_src = aS.hs_den;
        r->hs_num_dst = aT.hs_num; r->hs_den_dst = aT.hs_den;
        /* every other class that owns a caller of m: its CBO may change */
        ++stamp;
        for (int32_t q = cal_off[m]; q < cal_off[m + 1]; ++q) {
            int32_t y = cal_idx[q];
            if (y == m) continue;
            int32_t X = owner[y];
            if (X == S || X == T || seen[X] == stamp) continue;
            seen[X] = stamp;
            int32_t cb = class_cbo(&x, X, M.idx + M.off[X], M.off[X + 1] - M.off[X]);
            int32_t d = cb - before[X].cbo;
            r->n_caller_cls++;
            if (d > 0) r->n_caller_worse++;
            if (d < 0) r->n_caller_better++;
        }
        owner[m] = S;
        r->keep = keep_rule(r, &before[S], &before[T], mask, rule);
    }
    free(seen); free(buf); free(cal_idx); free(cal_off); free(before);
    members_free(&M);
    ctx_free(&x);
    free(owner);
    return rc;
}

/* Number of metric values the paper counts for one system: 2m + m(m-1)/2 +
 * 2c(m+1) (Sec. III-B). */
int64_t orc_value_count(int64_t c, int64_t m) { return 2 * m + m * (m - 1) / 2 + 2 * c * (m + 1); }

/* Pairs (m1, m2), m1 in [m_lo, m_hi), m2 > m1 over all methods, whose property
 * sets intersect: intersection and union sizes. Pairs come in (m1, m2)
 * ascending order. Returns the number of pairs; writes at most `cap` of them
 * (NULL outputs: count only); -1 on a bad range or allocation failure. */
int64_t orc_similarity(const orc_sys *s, int32_t m_lo, int32_t m_hi, int32_t *out_m1, int32_t *out_m2,
                       int32_t *out_inter, int32_t *out_union, int64_t cap) {
    const int32_t n = s->n_methods, na = s->n_attrs;
    if (m_lo < 0 || m_hi > n || m_lo > m_hi) return -1;
    /* property ids: method x -> x, attribute a -> n + a */
    int32_t *mark = (int32_t *)calloc((size_t)n + (size_t)na + 1, sizeof(int32_t));
    int32_t *seen = (int32_t *)calloc((size_t)n + (size_t)na + 1, sizeof(int32_t));
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!mark || !seen || !deg) {
        free(mark); free(seen); free(deg);
        return -1;
    }
    /* size of each property set (duplicates in a row count once) */
    int32_t stamp = 0;
    for (int32_t y = 0; y < n; ++y) {
        ++stamp;
        for (int64_t e = s->call_off[y]; e < s->call_off[y + 1]; ++e) {
            int32_t p = s->call_idx[e];
            if (seen[p] != stamp) { seen[p] = stamp; ++deg[y]; }
        }
        for (int64_t e = s->acc_off[y]; e < s->acc_off[y + 1]; ++e) {
            int32_t p = n + s->acc_idx[e];
            if (seen[p] != stamp) { seen[p] = stamp; ++deg[y]; }
        }
    }
    memset(seen, 0, ((size_t)n + (size_t)na + 1) * sizeof(int32_t));
    int64_t cnt = 0;
    int32_t stamp2 = 0;
    for (int32_t a = m_lo; a < m_hi; ++a) {
        /* the set of a */
        for (int64_t e = s->call_off[a]; e < s->call_off[a + 1]; ++e) mark[s->call_idx[e]] = a + 1;
        for (int64_t e = s->acc_off[a]; e < s->acc_off[a + 1]; ++e) mark[n + s->acc_idx[e]] = a + 1;
        for (int32_t b = a + 1; b < n; ++b) {
            /* shared properties of a and b, each counted once */
            if (++stamp2 == INT32_MAX) {
                memset(seen, 0, ((size_t)n + (size_t)na + 1) * sizeof(int32_t));
                stamp2 = 1;
            }
            int32_t inter = 0;
            for (int64_t e = s->call_off[b]; e < s->call_off[b + 1]; ++e) {
                int32_t p = s->call_idx[e];
                if (mark[p] == a + 1 && seen[p] != stamp2) { seen[p] = stamp2; ++inter; }
            }
            for (int64_t e = s->acc_off[b]; e < s->acc_off[b + 1]; ++e) {
                int32_t p = n + s->acc_idx[e];
                if (mark[p] == a + 1 && seen[p] != stamp2) { seen[p] = stamp2; ++inter; }
            }
            if (inter == 0) continue;
            if (out_m1 && cnt < cap) {
                out_m1[cnt] = a;
                out_m2[cnt] = b;
                out_inter[cnt] = inter;
                out_union[cnt] = deg[a] + deg[b] - inter;
            }
            ++cnt;
        }
    }
    free(mark); free(seen); free(deg);
    return cnt;
}

/*
 * The other three metrics of the Chidamber-Kemerer suite, which Sec. II-B names
 * beside CBO, RFC and LCOM (definitions of the suite the paper cites), over a
 * class hierarchy and per-method complexity weights given with the system:
 *   WMC(C)  sum of the weights of C's methods (every weight 1 when `weight` is
 *           NULL, so WMC(C) = n_C)
 *   NOC(C)  number of classes whose parent is C (its immediate subclasses)
 *   DIT(C)  number of proper ancestors of C: the steps up the parent chain from
 *           C to a class whose parent is -1 (no parent inside the system)
 * Returns 0; -2 for a parent id outside [-1, n_classes) or a negative weight;
 * -1 when some parent chain does not end within n_classes steps (a cycle).
 */
int orc_ck(const orc_sys *s, const int32_t *parent, const int32_t *weight, int64_t *wmc, int32_t *noc,
           int32_t *dit) {
    const int32_t c = s->n_classes, n = s->n_methods;
    for (int32_t C = 0; C < c; ++C) {
        if (parent[C] < -1 || parent[C] >= c) return -2;
        wmc[C] = 0;
        noc[C] = 0;
    }
    for (int32_t m = 0; m < n; ++m) {
        const int32_t w = weight ? weight[m] : 1;
        if (w < 0) return -2;
        wmc[s->method_class[m]] += w;
    }
    for (int32_t C = 0; C < c; ++C)
        for (int32_t D = 0; D < c; ++D)
            if (parent[D] == C) ++noc[C];
    for (int32_t C = 0; C < c; ++C) {
        int32_t steps = 0;
        for (int32_t x = C; parent[x] != -1; x = parent[x])
            if (++steps > c) return -1;
        dit[C] = steps;
    }
    return 0;
}

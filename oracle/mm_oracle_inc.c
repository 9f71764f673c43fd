/*
 * mm_oracle_inc.c -- second CPU oracle: move deltas from grouped counts.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header or table with the first oracle (mm_oracle.c) or with the HIP
 * library; the two oracles are checked against each other by the tests.
 *
 * The first oracle scores a move by re-evaluating the changed classes (the
 * re-run of the metric functions on the changed membership, Sec. IV-C). This
 * one keeps, for the current system, grouped counts per class and per method,
 * and derives every delta of a move m -> T (S = the class of m) from them:
 *
 *   LCOM (pair form, Sec. II-B). Q_C = pairs of C's methods sharing an
 *     attribute of C. rnz(m) = methods of S other than m sharing an attribute
 *     of S with m; h_T(m) = methods of T sharing an attribute of T with m.
 *     Q_S' = Q_S - rnz(m), Q_T' = Q_T + h_T(m), P' = n'(n'-1)/2 - Q', with
 *     n_S' = n_S - 1 and n_T' = n_T + 1.
 *   LCOM ratio form (Sec. II-B). U_C = sum over C's methods of the attributes
 *     of C each uses. U_S' = U_S - |acc(m) in A_S|, U_T' = U_T + |acc(m) in A_T|.
 *   RFC (the CK response set, one level). cnt_C(x) = methods of C calling x.
 *     S loses m unless another method of S calls it; S loses a callee x != m of
 *     m that S does not own when m was its only caller in S; T gains m unless a
 *     method of T calls it; T gains a callee x != m it does not own that no
 *     method of T calls.
 *   CBO (Sec. II-B, efferent). w_C(D) = references (calls and attribute
 *     accesses) from C's methods to things owned by D != C. out_m(D) = m's own
 *     references to D (a self-call stays inside m's class and is left out);
 *     in_m(X) = methods of X other than m calling m. Then
 *       w_S'(D) = w_S(D) - out_m(D) for D != S, plus in_m(S) more at D = T;
 *       w_T'(D) = w_T(D) + out_m(D) for D != T, less in_m(T) at D = S;
 *       for every other class X calling m: w_X'(S) = w_X(S) - in_m(X) and
 *       w_X'(T) = w_X(T) + in_m(X), so its CBO changes by
 *       [w_X(T) = 0] - [w_X(S) = in_m(X)].
 *     CBO' counts the keys D with w'(D) > 0.
 *
 * The keep rules (abstract, Sec. III-A, Sec. IV-A) are restated here: lower is
 * better for every metric; PARETO keeps a move when no affected (class, masked
 * metric) worsens and one improves; the LCOM rule when every masked LCOM form
 * improves in both S and T; the CBO rule when S's CBO falls, T's does not rise
 * and no caller class's rises. LCOM_HS fractions compare exactly.
 *
 * Rows are read as sets. Scoring runs on `nthreads` POSIX threads over
 * contiguous candidate ranges; every thread writes only its own records.
 */
#include <pthread.h>
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
} inc_desc;

typedef struct {
    int32_t n_methods, n_attrs, cbo, rfc;
    int64_t lcom_p, lcom_q, hs_num, hs_den;
} inc_class;

typedef struct {
    int32_t fan_in, fan_out, own_attr_uses, own_coaccess_partners;
} inc_method;

typedef struct {
    int32_t method, src, dst;
    int32_t d_cbo_src, d_cbo_dst, d_rfc_src, d_rfc_dst;
    int32_t n_caller_cls, n_caller_worse, n_caller_better;
    int32_t keep, pad;
    int64_t d_lcom_src, d_lcom_dst;
    int64_t hs_num_src, hs_den_src, hs_num_dst, hs_den_dst;
} inc_move;

enum { I_CBO = 1, I_LCOM_PQ = 2, I_LCOM_HS = 4, I_RFC = 8 };
enum { I_PARETO = 0, I_PAPER_LCOM = 1, I_PAPER_CBO = 2 };

typedef struct { int32_t key, count; } kc;

typedef struct {
    int32_t c, n, na;
    int32_t *owner, *acls, *acnt;
    int64_t *ao, *co, *ro, *mo, *to, *wo, *no, *io;
    int32_t *ai, *ci, *ri, *mi, *ti;
    int64_t *U, *Q;
    int32_t *rnz, *own;
    kc *w, *cnt, *in;
} inc_state;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* sort a short array in place (insertion sort; qsort for long ones) */
static void sort_i32(int32_t *v, int64_t len) {
    if (len > 48) {
        qsort(v, (size_t)len, sizeof(int32_t), cmp_i32);
        return;
    }
    for (int64_t i = 1; i < len; ++i) {
        int32_t x = v[i];
        int64_t j = i - 1;
        while (j >= 0 && v[j] > x) { v[j + 1] = v[j]; --j; }
        v[j + 1] = x;
    }
}

/* rows as sorted sets */
static int set_rows(const int64_t *off, const int32_t *idx, int32_t rows, int64_t **oo, int32_t **oi) {
    int64_t nnz = off[rows];
    int64_t *o = (int64_t *)malloc(((size_t)rows + 1) * sizeof(int64_t));
    int32_t *v = (int32_t *)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    if (!o || !v) { free(o); free(v); return -1; }
    int64_t k = 0;
    o[0] = 0;
    for (int32_t r = 0; r < rows; ++r) {
        int64_t b = k;
        for (int64_t e = off[r]; e < off[r + 1]; ++e) v[k++] = idx[e];
        sort_i32(v + b, k - b);
        int64_t w = b;
        for (int64_t e = b; e < k; ++e)
            if (e == b || v[e] != v[e - 1]) v[w++] = v[e];
        k = w;
        o[r + 1] = k;
    }
    *oo = o;
    *oi = v;
    return 0;
}

/* lists grouped by a key: item i goes to list key[i] (keys in [0, groups)),
 * items kept in increasing i */
static int group_by(const int32_t *key, const int32_t *item, int64_t len, int32_t groups, int64_t **go, int32_t **gi) {
    int64_t *o = (int64_t *)calloc((size_t)groups + 1, sizeof(int64_t));
    int32_t *v = (int32_t *)malloc(((size_t)len + 1) * sizeof(int32_t));
    int64_t *at = (int64_t *)malloc(((size_t)groups + 1) * sizeof(int64_t));
    if (!o || !v || !at) { free(o); free(v); free(at); return -1; }
    for (int64_t i = 0; i < len; ++i) o[key[i] + 1]++;
    for (int32_t g = 0; g < groups; ++g) o[g + 1] += o[g];
    memcpy(at, o, (size_t)groups * sizeof(int64_t));
    for (int64_t i = 0; i < len; ++i) v[at[key[i]]++] = item[i];
    free(at);
    *go = o;
    *gi = v;
    return 0;
}

/* one grouped count per owner: for owner g, the multiset of keys in
 * vals[vo[g]..vo[g+1]) becomes sorted (key, count) pairs */
static int count_groups(int32_t groups, const int64_t *vo, int32_t *vals, int64_t **ko, kc **kv) {
    int64_t *o = (int64_t *)malloc(((size_t)groups + 1) * sizeof(int64_t));
    kc *p = (kc *)malloc(((size_t)vo[groups] + 1) * sizeof(kc));
    if (!o || !p) { free(o); free(p); return -1; }
    int64_t k = 0;
    o[0] = 0;
    for (int32_t g = 0; g < groups; ++g) {
        int32_t *v = vals + vo[g];
        int64_t len = vo[g + 1] - vo[g];
        sort_i32(v, len);
        for (int64_t e = 0; e < len; ++e) {
            if (e > 0 && v[e] == v[e - 1]) {
                p[k - 1].count++;
            } else {
                p[k].key = v[e];
                p[k].count = 1;
                ++k;
            }
        }
        o[g + 1] = k;
    }
    *ko = o;
    *kv = p;
    return 0;
}

static int32_t count_of(const kc *p, int64_t lo, int64_t hi, int32_t key) {
    int64_t a = lo, b = hi;
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (p[mid].key < key) a = mid + 1;
        else b = mid;
    }
    return (a < hi && p[a].key == key) ? p[a].count : 0;
}

void inc_free(void *p) {
    inc_state *s = (inc_state *)p;
    if (!s) return;
    free(s->owner); free(s->acls); free(s->acnt);
    free(s->ao); free(s->co); free(s->ro); free(s->mo); free(s->to); free(s->wo); free(s->no); free(s->io);
    free(s->ai); free(s->ci); free(s->ri); free(s->mi); free(s->ti);
    free(s->U); free(s->Q); free(s->rnz); free(s->own);
    free(s->w); free(s->cnt); free(s->in);
    free(s);
}

/* Builds the grouped counts of a system. Returns NULL on a bad argument or an
 * allocation failure. */
void *inc_build(const inc_desc *d) {
    if (!d || d->n_classes < 0 || d->n_methods < 0 || d->n_attrs < 0) return NULL;
    inc_state *s = (inc_state *)calloc(1, sizeof(inc_state));
    if (!s) return NULL;
    const int32_t c = d->n_classes, n = d->n_methods, na = d->n_attrs;
    s->c = c; s->n = n; s->na = na;
    for (int32_t m = 0; m < n; ++m)
        if (d->method_class[m] < 0 || d->method_class[m] >= c) goto fail;
    for (int32_t a = 0; a < na; ++a)
        if (d->attr_class[a] < 0 || d->attr_class[a] >= c) goto fail;
    for (int64_t e = 0; e < d->acc_off[n]; ++e)
        if (d->acc_idx[e] < 0 || d->acc_idx[e] >= na) goto fail;
    for (int64_t e = 0; e < d->call_off[n]; ++e)
        if (d->call_idx[e] < 0 || d->call_idx[e] >= n) goto fail;
    s->owner = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    s->acls = (int32_t *)malloc(((size_t)na + 1) * sizeof(int32_t));
    s->acnt = (int32_t *)calloc((size_t)c + 1, sizeof(int32_t));
    if (!s->owner || !s->acls || !s->acnt) goto fail;
    memcpy(s->owner, d->method_class, (size_t)n * sizeof(int32_t));
    memcpy(s->acls, d->attr_class, (size_t)na * sizeof(int32_t));
    for (int32_t a = 0; a < na; ++a) s->acnt[s->acls[a]]++;
    if (set_rows(d->acc_off, d->acc_idx, n, &s->ao, &s->ai)) goto fail;
    if (set_rows(d->call_off, d->call_idx, n, &s->co, &s->ci)) goto fail;
    {
        /* members of each class, ascending */
        int32_t *ids = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
        if (!ids) goto fail;
        for (int32_t m = 0; m < n; ++m) ids[m] = m;
        int rc = group_by(s->owner, ids, n, c, &s->mo, &s->mi);
        free(ids);
        if (rc) goto fail;
    }
    {
        /* callers of each method, ascending, each once (rows are sets) */
        const int64_t nc = s->co[n];
        int32_t *callee = (int32_t *)malloc(((size_t)nc + 1) * sizeof(int32_t));
        int32_t *caller = (int32_t *)malloc(((size_t)nc + 1) * sizeof(int32_t));
        if (!callee || !caller) { free(callee); free(caller); goto fail; }
        for (int32_t y = 0; y < n; ++y)
            for (int64_t e = s->co[y]; e < s->co[y + 1]; ++e) { callee[e] = s->ci[e]; caller[e] = y; }
        int rc = group_by(callee, caller, nc, n, &s->ro, &s->ri);
        free(callee); free(caller);
        if (rc) goto fail;
    }
    {
        /* accessors of each attribute among the methods of its own class */
        const int64_t nac = s->ao[n];
        int32_t *at = (int32_t *)malloc(((size_t)nac + 1) * sizeof(int32_t));
        int32_t *who = (int32_t *)malloc(((size_t)nac + 1) * sizeof(int32_t));
        if (!at || !who) { free(at); free(who); goto fail; }
        int64_t k = 0;
        for (int32_t y = 0; y < n; ++y)
            for (int64_t e = s->ao[y]; e < s->ao[y + 1]; ++e)
                if (s->acls[s->ai[e]] == s->owner[y]) { at[k] = s->ai[e]; who[k] = y; ++k; }
        int rc = group_by(at, who, k, na, &s->to, &s->ti);
        free(at); free(who);
        if (rc) goto fail;
    }
    s->U = (int64_t *)calloc((size_t)c + 1, sizeof(int64_t));
    s->Q = (int64_t *)calloc((size_t)c + 1, sizeof(int64_t));
    s->rnz = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    s->own = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!s->U || !s->Q || !s->rnz || !s->own) goto fail;
    {
        /* own uses, U; co-access partners through the own-class accessor lists */
        int32_t *mark = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        if (!mark) goto fail;
        for (int32_t y = 0; y < n; ++y) {
            const int32_t C = s->owner[y];
            int32_t uses = 0, partners = 0;
            for (int64_t e = s->ao[y]; e < s->ao[y + 1]; ++e) {
                const int32_t a = s->ai[e];
                if (s->acls[a] != C) continue;
                ++uses;
                for (int64_t q = s->to[a]; q < s->to[a + 1]; ++q) {
                    const int32_t j = s->ti[q];
                    if (j != y && mark[j] != y + 1) { mark[j] = y + 1; ++partners; }
                }
            }
            s->own[y] = uses;
            s->rnz[y] = partners;
            s->U[C] += uses;
            s->Q[C] += partners;  /* each pair counted from both ends */
        }
        for (int32_t C = 0; C < c; ++C) s->Q[C] /= 2;
        free(mark);
    }
    {
        /* w: foreign owners of every reference of the class's methods */
        const int64_t nref = s->ao[n] + s->co[n];
        int64_t *vo = (int64_t *)calloc((size_t)c + 1, sizeof(int64_t));
        int32_t *vals = (int32_t *)malloc(((size_t)nref + 1) * sizeof(int32_t));
        if (!vo || !vals) { free(vo); free(vals); goto fail; }
        int64_t k = 0;
        for (int32_t C = 0; C < c; ++C) {
            for (int64_t q = s->mo[C]; q < s->mo[C + 1]; ++q) {
                const int32_t y = s->mi[q];
                for (int64_t e = s->co[y]; e < s->co[y + 1]; ++e)
                    if (s->owner[s->ci[e]] != C) vals[k++] = s->owner[s->ci[e]];
                for (int64_t e = s->ao[y]; e < s->ao[y + 1]; ++e)
                    if (s->acls[s->ai[e]] != C) vals[k++] = s->acls[s->ai[e]];
            }
            vo[C + 1] = k;
        }
        int rc = count_groups(c, vo, vals, &s->wo, &s->w);
        /* cnt: callees of the class's methods */
        k = 0;
        for (int32_t C = 0; C < c && !rc; ++C) {
            for (int64_t q = s->mo[C]; q < s->mo[C + 1]; ++q) {
                const int32_t y = s->mi[q];
                for (int64_t e = s->co[y]; e < s->co[y + 1]; ++e) vals[k++] = s->ci[e];
            }
            vo[C + 1] = k;
        }
        if (!rc) rc = count_groups(c, vo, vals, &s->no, &s->cnt);
        free(vo); free(vals);
        if (rc) goto fail;
    }
    {
        /* in: classes of the callers y != x of every method x */
        int64_t *vo = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        int32_t *vals = (int32_t *)malloc(((size_t)s->ro[n] + 1) * sizeof(int32_t));
        if (!vo || !vals) { free(vo); free(vals); goto fail; }
        int64_t k = 0;
        for (int32_t x = 0; x < n; ++x) {
            for (int64_t e = s->ro[x]; e < s->ro[x + 1]; ++e)
                if (s->ri[e] != x) vals[k++] = s->owner[s->ri[e]];
            vo[x + 1] = k;
        }
        int rc = count_groups(n, vo, vals, &s->io, &s->in);
        free(vo); free(vals);
        if (rc) goto fail;
    }
    return s;
fail:
    inc_free(s);
    return NULL;
}

static void hs_pair(int64_t n, int64_t a, int64_t u, int64_t *num, int64_t *den) {
    if (n * a == 0) { *num = 0; *den = 1; }
    else { *num = n * a - u; *den = n * a; }
}

/* Metrics of every class and method from the grouped counts. */
int inc_metrics(void *p, inc_class *cls, inc_method *meth) {
    const inc_state *s = (const inc_state *)p;
    if (!s) return -1;
    for (int32_t C = 0; cls && C < s->c; ++C) {
        const int64_t nC = s->mo[C + 1] - s->mo[C];
        inc_class *o = &cls[C];
        o->n_methods = (int32_t)nC;
        o->n_attrs = s->acnt[C];
        o->cbo = (int32_t)(s->wo[C + 1] - s->wo[C]);
        int32_t outside = 0;
        for (int64_t e = s->no[C]; e < s->no[C + 1]; ++e) outside += s->owner[s->cnt[e].key] != C;
        o->rfc = (int32_t)nC + outside;
        o->lcom_q = s->Q[C];
        o->lcom_p = nC * (nC - 1) / 2 - s->Q[C];
        hs_pair(nC, s->acnt[C], s->U[C], &o->hs_num, &o->hs_den);
    }
    for (int32_t y = 0; meth && y < s->n; ++y) {
        meth[y].fan_in = (int32_t)(s->ro[y + 1] - s->ro[y]);
        meth[y].fan_out = (int32_t)(s->co[y + 1] - s->co[y]);
        meth[y].own_attr_uses = s->own[y];
        meth[y].own_coaccess_partners = s->rnz[y];
    }
    return 0;
}

/* REFERENCED candidates: for every method, ascending, the classes other than
 * its own that own a method it calls or an attribute it accesses, ascending.
 * Returns their number; writes at most cap of them. */
int64_t inc_referenced(void *p, int32_t *cm, int32_t *ct, int64_t cap) {
    const inc_state *s = (const inc_state *)p;
    if (!s) return -1;
    int32_t *buf = NULL;
    int64_t bufcap = 0, total = 0;
    for (int32_t m = 0; m < s->n; ++m) {
        const int64_t len = (s->co[m + 1] - s->co[m]) + (s->ao[m + 1] - s->ao[m]);
        if (len > bufcap) {
            free(buf);
            bufcap = len * 2;
            buf = (int32_t *)malloc((size_t)bufcap * sizeof(int32_t));
            if (!buf) return -1;
        }
        int64_t k = 0;
        for (int64_t e = s->co[m]; e < s->co[m + 1]; ++e) buf[k++] = s->owner[s->ci[e]];
        for (int64_t e = s->ao[m]; e < s->ao[m + 1]; ++e) buf[k++] = s->acls[s->ai[e]];
        sort_i32(buf, k);
        for (int64_t e = 0; e < k; ++e) {
            if ((e > 0 && buf[e] == buf[e - 1]) || buf[e] == s->owner[m]) continue;
            if (total < cap) { cm[total] = m; ct[total] = buf[e]; }
            ++total;
        }
    }
    free(buf);
    return total;
}

/* sign of num1/den1 - num0/den0 (positive denominators) */
static int frac_cmp(int64_t num0, int64_t den0, int64_t num1, int64_t den1) {
    const __int128 a = (__int128)num1 * den0, b = (__int128)num0 * den1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

typedef struct {
    int32_t *mark;  /* per method: last candidate that marked it (plus one) */
    int32_t *buf;
    int64_t bufcap;
    int64_t tag;
} scratch;

static int score_one(const inc_state *s, scratch *t, int32_t m, int32_t T, uint32_t mask, int32_t rule, inc_move *r) {
    const int32_t S = s->owner[m];
    memset(r, 0, sizeof(*r));
    r->method = m; r->src = S; r->dst = T;
    /* m's references by owning class (out_m), self-call left out */
    const int64_t len = (s->co[m + 1] - s->co[m]) + (s->ao[m + 1] - s->ao[m]);
    if (len > t->bufcap) {
        free(t->buf);
        t->bufcap = len * 2;
        t->buf = (int32_t *)malloc((size_t)t->bufcap * sizeof(int32_t));
        if (!t->buf) return -1;
    }
    int64_t k = 0;
    int self = 0;
    for (int64_t e = s->co[m]; e < s->co[m + 1]; ++e) {
        if (s->ci[e] == m) self = 1;
        else t->buf[k++] = s->owner[s->ci[e]];
    }
    for (int64_t e = s->ao[m]; e < s->ao[m + 1]; ++e) t->buf[k++] = s->acls[s->ai[e]];
    sort_i32(t->buf, k);
    const int32_t inS = count_of(s->in, s->io[m], s->io[m + 1], S);
    const int32_t inT = count_of(s->in, s->io[m], s->io[m + 1], T);
    /* CBO of S and T over the keys whose counts change */
    int dS = 0, dT = 0, sawT = 0, sawS = 0;
    for (int64_t e = 0; e < k;) {
        const int32_t D = t->buf[e];
        int32_t o = 0;
        while (e < k && t->buf[e] == D) { ++o; ++e; }
        if (D != S) {
            const int32_t b = count_of(s->w, s->wo[S], s->wo[S + 1], D);
            const int32_t a = b - o + (D == T ? inS : 0);
            dS += (a > 0) - (b > 0);
        }
        if (D != T) {
            const int32_t b = count_of(s->w, s->wo[T], s->wo[T + 1], D);
            const int32_t a = b + o - (D == S ? inT : 0);
            dT += (a > 0) - (b > 0);
        }
        sawT |= D == T;
        sawS |= D == S;
    }
    if (!sawT) {
        const int32_t b = count_of(s->w, s->wo[S], s->wo[S + 1], T);
        dS += (b + inS > 0) - (b > 0);
    }
    if (!sawS) {
        const int32_t b = count_of(s->w, s->wo[T], s->wo[T + 1], S);
        dT += (b - inT > 0) - (b > 0);
    }
    r->d_cbo_src = dS;
    r->d_cbo_dst = dT;
    /* caller classes other than S and T */
    for (int64_t e = s->io[m]; e < s->io[m + 1]; ++e) {
        const int32_t X = s->in[e].key, cX = s->in[e].count;
        if (X == S || X == T) continue;
        const int32_t wS = count_of(s->w, s->wo[X], s->wo[X + 1], S);
        const int32_t wT = count_of(s->w, s->wo[X], s->wo[X + 1], T);
        const int dX = (wT == 0) - (wS == cX);
        r->n_caller_cls++;
        r->n_caller_worse += dX > 0;
        r->n_caller_better += dX < 0;
    }
    /* RFC */
    int dRS = 0, dRT = 0;
    if (count_of(s->cnt, s->no[S], s->no[S + 1], m) - self == 0) dRS -= 1;
    if (count_of(s->cnt, s->no[T], s->no[T + 1], m) == 0) dRT += 1;
    for (int64_t e = s->co[m]; e < s->co[m + 1]; ++e) {
        const int32_t x = s->ci[e];
        if (x == m) continue;
        if (s->owner[x] != S && count_of(s->cnt, s->no[S], s->no[S + 1], x) == 1) dRS -= 1;
        if (s->owner[x] != T && count_of(s->cnt, s->no[T], s->no[T + 1], x) == 0) dRT += 1;
    }
    r->d_rfc_src = dRS;
    r->d_rfc_dst = dRT;
    /* LCOM: co-access partners gained in T, lost in S; own uses */
    ++t->tag;
    int32_t h = 0, uT = 0;
    for (int64_t e = s->ao[m]; e < s->ao[m + 1]; ++e) {
        const int32_t a = s->ai[e];
        if (s->acls[a] != T) continue;
        ++uT;
        for (int64_t q = s->to[a]; q < s->to[a + 1]; ++q) {
            const int32_t j = s->ti[q];
            if (t->mark[j] != (int32_t)t->tag) { t->mark[j] = (int32_t)t->tag; ++h; }
        }
    }
    const int64_t nS = s->mo[S + 1] - s->mo[S], nT = s->mo[T + 1] - s->mo[T];
    const int64_t qS = s->Q[S], qT = s->Q[T], qS1 = qS - s->rnz[m], qT1 = qT + h;
    const int64_t lS0 = nS * (nS - 1) / 2 - 2 * qS, lS1 = (nS - 1) * (nS - 2) / 2 - 2 * qS1;
    const int64_t lT0 = nT * (nT - 1) / 2 - 2 * qT, lT1 = (nT + 1) * nT / 2 - 2 * qT1;
    r->d_lcom_src = lS1 - lS0;
    r->d_lcom_dst = lT1 - lT0;
    hs_pair(nS - 1, s->acnt[S], s->U[S] - s->own[m], &r->hs_num_src, &r->hs_den_src);
    hs_pair(nT + 1, s->acnt[T], s->U[T] + uT, &r->hs_num_dst, &r->hs_den_dst);
    int64_t hn, hd;
    hs_pair(nS, s->acnt[S], s->U[S], &hn, &hd);
    const int fS = frac_cmp(hn, hd, r->hs_num_src, r->hs_den_src);
    hs_pair(nT, s->acnt[T], s->U[T], &hn, &hd);
    const int fT = frac_cmp(hn, hd, r->hs_num_dst, r->hs_den_dst);
    /* keep rule */
    if (rule == I_PAPER_CBO) {
        r->keep = r->d_cbo_src < 0 && r->d_cbo_dst <= 0 && r->n_caller_worse == 0;
    } else if (rule == I_PAPER_LCOM) {
        int ok = 1;
        if ((mask & I_LCOM_PQ) && !(r->d_lcom_src < 0 && r->d_lcom_dst < 0)) ok = 0;
        if ((mask & I_LCOM_HS) && !(fS < 0 && fT < 0)) ok = 0;
        r->keep = ok;
    } else {
        int improves = 0, worsens = 0;
#define NOTE(v) do { if ((v) < 0) improves = 1; if ((v) > 0) worsens = 1; } while (0)
        if (mask & I_CBO) {
            NOTE(r->d_cbo_src); NOTE(r->d_cbo_dst);
            if (r->n_caller_better) improves = 1;
            if (r->n_caller_worse) worsens = 1;
        }
        if (mask & I_LCOM_PQ) { NOTE(r->d_lcom_src); NOTE(r->d_lcom_dst); }
        if (mask & I_LCOM_HS) { NOTE(fS); NOTE(fT); }
        if (mask & I_RFC) { NOTE(r->d_rfc_src); NOTE(r->d_rfc_dst); }
#undef NOTE
        r->keep = improves && !worsens;
    }
    return 0;
}

typedef struct {
    const inc_state *s;
    const int32_t *cm, *ct;
    int64_t lo, hi;
    uint32_t mask;
    int32_t rule;
    inc_move *out;
    int rc;
} job;

static void *run_job(void *arg) {
    job *j = (job *)arg;
    scratch t = {NULL, NULL, 0, 0};
    t.mark = (int32_t *)calloc((size_t)j->s->n + 1, sizeof(int32_t));
    if (!t.mark) { j->rc = -1; return NULL; }
    for (int64_t q = j->lo; q < j->hi && !j->rc; ++q) {
        if (t.tag == INT32_MAX - 1) {
            memset(t.mark, 0, ((size_t)j->s->n + 1) * sizeof(int32_t));
            t.tag = 0;
        }
        if (score_one(j->s, &t, j->cm[q], j->ct[q], j->mask, j->rule, &j->out[q])) j->rc = -1;
    }
    free(t.mark);
    free(t.buf);
    return NULL;
}

/* Score explicit candidates on nthreads threads. Returns 0, or -1 on a bad
 * argument (T equal to the method's class, an id out of range, a bad rule or
 * mask) or a failure. */
int inc_score(void *p, int64_t n_cand, const int32_t *cm, const int32_t *ct, uint32_t mask, int32_t rule,
              inc_move *out, int32_t nthreads) {
    const inc_state *s = (const inc_state *)p;
    if (!s || n_cand < 0 || (mask & ~15u) || rule < 0 || rule > 2) return -1;
    if (rule == I_PAPER_LCOM && !(mask & (I_LCOM_PQ | I_LCOM_HS))) return -1;
    if (rule == I_PAPER_CBO && !(mask & I_CBO)) return -1;
    for (int64_t q = 0; q < n_cand; ++q)
        if (cm[q] < 0 || cm[q] >= s->n || ct[q] < 0 || ct[q] >= s->c || ct[q] == s->owner[cm[q]]) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (n_cand < 4096) nthreads = 1;
    job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int i = 0; i < nthreads; ++i) {
        jobs[i] = (job){s, cm, ct, n_cand * i / nthreads, n_cand * (i + 1) / nthreads, mask, rule, out, 0};
        started[i] = 0;
    }
    if (nthreads == 1) {
        run_job(&jobs[0]);
        return jobs[0].rc;
    }
    for (int i = 0; i < nthreads; ++i) started[i] = pthread_create(&th[i], NULL, run_job, &jobs[i]) == 0;
    int rc = 0;
    for (int i = 0; i < nthreads; ++i) {
        if (started[i]) pthread_join(th[i], NULL);
        else run_job(&jobs[i]);
        if (jobs[i].rc) rc = -1;
    }
    return rc;
}

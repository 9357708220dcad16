/*
 * oracle.c -- plain CPU reference for scan -> filter -> hash-join probe ->
 * group-by aggregation over UNCOMPRESSED columns.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's query path may link,
 * load or call this file; only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes (paper Section 3.1, the three kernels of the running
 * example; Section 4.1 "Fused kernel composition" and "Variable-length scan
 * operators"): data path fusion reaches exactly the plain relational result,
 * since compression is lossless (Section 3.4) and the operators are ordinary
 * filter, inner hash join and hash aggregation.  So this oracle is that plain
 * definition, evaluated one row at a time:
 *
 *   SELECT keys, aggs FROM F JOIN D_1 ... JOIN D_k
 *   WHERE psi(F) AND phi_1(D_1) AND ... AND phi_k(D_k)
 *   GROUP BY keys ORDER BY keys
 *
 * with inner-join semantics, exact int64 arithmetic (every + and * is checked;
 * overflow is an error, never a wrapped value -- Section 4.3 processes
 * decimals as 64-bit integers), empty groups not emitted, and the LIKE-style
 * string predicate of Section 4.1 read as "s1 occurs, and s2 occurs at or
 * after the end of that occurrence" (LIKE '%s1%s2%').
 *
 * Library primitives used as steps: qsort/bsearch (the join: a sorted build
 * side searched by key) and memmem (substring search).
 *
 * Pins: every function here is checked against brute force, hand-computed
 * plans, closed forms, library routines and invariants (the tests' pin
 * suite).  The paper prints no result values for any query, so agreement
 * with the paper's own numbers is parity unpinned.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------------ */
/* Predicates (conjunctive atoms, Section 3.1: "predicates appearing in the  */
/* query pipeline")                                                          */
/* ------------------------------------------------------------------------ */
static int contains_seq(const uint8_t* s, int64_t n, const uint8_t* w1, int32_t n1,
                        const uint8_t* w2, int32_t n2) {
    /* The leftmost occurrence of w1 leaves the most room for w2, so testing
     * only it is exact for LIKE '%w1%w2%'. */
    const uint8_t* p = memmem(s, (size_t)n, w1, (size_t)n1);
    if (!p) return 0;
    const uint8_t* rest = p + n1;
    int64_t left = n - (rest - s);
    return memmem(rest, (size_t)left, w2, (size_t)n2) != NULL;
}

static int eval_pred(const orc_pred* p, const orc_column* cols, int64_t row) {
    const orc_column* c = &cols[p->col];
    if (p->op == ORC_STR_CONTAINS_SEQ) {
        int64_t a = c->str_off[row], b = c->str_off[row + 1];
        return contains_seq(c->str_bytes + a, b - a, p->s1, p->n1, p->s2, p->n2);
    }
    int64_t x = c->ival[row];
    switch (p->op) {
        case ORC_LT: return x < p->a;
        case ORC_LE: return x <= p->a;
        case ORC_GT: return x > p->a;
        case ORC_GE: return x >= p->a;
        case ORC_EQ: return x == p->a;
        case ORC_NE: return x != p->a;
        case ORC_BETWEEN: return x >= p->a && x <= p->b;
        case ORC_IN:
            for (int32_t i = 0; i < p->nin; ++i)
                if (p->in[i] == x) return 1;
            return 0;
        default: return 0;
    }
}

static int check_preds(const orc_pred* preds, int32_t n, const orc_column* cols, int32_t ncols) {
    for (int32_t i = 0; i < n; ++i) {
        const orc_pred* p = &preds[i];
        if (p->col < 0 || p->col >= ncols) return ORC_ERR_INVALID;
        int is_str = p->op == ORC_STR_CONTAINS_SEQ;
        if (is_str != (cols[p->col].str_off != NULL)) return ORC_ERR_INVALID;
        if (is_str && (p->n1 <= 0 || p->n2 <= 0 || !p->s1 || !p->s2)) return ORC_ERR_INVALID;
        if (p->op < ORC_LT || p->op > ORC_STR_CONTAINS_SEQ) return ORC_ERR_INVALID;
        if (p->op == ORC_IN && p->nin > 0 && !p->in) return ORC_ERR_INVALID;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Build side: the filtered dimension, sorted by key (Section 3.1, Kernel #1 */
/* "builds a hash table"; a sorted array searched by key is the same map).   */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t key, pay[ORC_MAX_PAYLOADS]; } dim_entry;

static int cmp_entry(const void* a, const void* b) {
    int64_t x = ((const dim_entry*)a)->key, y = ((const dim_entry*)b)->key;
    return (x > y) - (x < y);
}

typedef struct { dim_entry* e; int64_t n; } dim_map;

static const dim_entry* probe_dim(const dim_map* m, int64_t key) {
    dim_entry k;
    k.key = key;
    return (const dim_entry*)bsearch(&k, m->e, (size_t)m->n, sizeof(dim_entry), cmp_entry);
}

#define ORC_MAX_DEPTH 4  /* nesting of joined build sides */

/* The qualifying rows of a (possibly joined) dimension, sorted by key: a row
 * qualifies if it passes the dimension's predicates and, for each of its own
 * probes, its foreign key is a key of that probe's qualifying rows (built
 * first, the same way: a filtered inner join, Section 3.1's Kernel #2). */
static int build_dim_at(const orc_probe* pr, dim_map* out, int depth) {
    const orc_column* cols = pr->cols;
    if (depth > ORC_MAX_DEPTH || pr->nsub < 0 || pr->nsub > ORC_MAX_PROBES || (pr->nsub && !pr->sub))
        return ORC_ERR_INVALID;
    if (pr->key_col < 0 || pr->key_col >= pr->ncols || !cols[pr->key_col].ival) return ORC_ERR_INVALID;
    if (pr->npay < 0 || pr->npay > ORC_MAX_PAYLOADS) return ORC_ERR_INVALID;
    for (int32_t k = 0; k < pr->npay; ++k) {
        const int32_t src = pr->nsub ? pr->pay_src[k] : -1;
        if (src < 0 && (pr->pay_col[k] < 0 || pr->pay_col[k] >= pr->ncols || !cols[pr->pay_col[k]].ival))
            return ORC_ERR_INVALID;
        if (src >= 0 && (src >= pr->nsub || pr->pay_col[k] < 0 || pr->pay_col[k] >= pr->sub[src].npay))
            return ORC_ERR_INVALID;
    }
    for (int32_t j = 0; j < pr->nsub; ++j)
        if (pr->sub[j].fact_fk_col < 0 || pr->sub[j].fact_fk_col >= pr->ncols || !cols[pr->sub[j].fact_fk_col].ival)
            return ORC_ERR_INVALID;
    int rc = check_preds(pr->preds, pr->npreds, cols, pr->ncols);
    if (rc) return rc;
    dim_map sub[ORC_MAX_PROBES];
    memset(sub, 0, sizeof sub);
    for (int32_t j = 0; j < pr->nsub && !rc; ++j) rc = build_dim_at(&pr->sub[j], &sub[j], depth + 1);
    int64_t nrows = cols[pr->key_col].nrows;
    dim_entry* e = rc ? NULL : (dim_entry*)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(dim_entry));
    if (!rc && !e) rc = ORC_ERR_OOM;
    int64_t n = 0;
    const dim_entry* hit[ORC_MAX_PROBES];
    for (int64_t r = 0; r < nrows && !rc; ++r) {
        int ok = 1;
        for (int32_t i = 0; i < pr->npreds && ok; ++i) ok = eval_pred(&pr->preds[i], cols, r);
        for (int32_t j = 0; j < pr->nsub && ok; ++j) {
            hit[j] = probe_dim(&sub[j], cols[pr->sub[j].fact_fk_col].ival[r]);
            ok = hit[j] != NULL;
        }
        if (!ok) continue;
        e[n].key = cols[pr->key_col].ival[r];
        for (int32_t k = 0; k < ORC_MAX_PAYLOADS; ++k) {
            if (k < pr->npay && pr->nsub && pr->pay_src[k] >= 0) {
                e[n].pay[k] = hit[pr->pay_src[k]]->pay[pr->pay_col[k]];
                continue;
            }
            e[n].pay[k] = k < pr->npay ? cols[pr->pay_col[k]].ival[r] : 0;
        }
        ++n;
    }
    for (int32_t j = 0; j < pr->nsub; ++j) free(sub[j].e);
    if (rc) { free(e); return rc; }
    qsort(e, (size_t)n, sizeof(dim_entry), cmp_entry);
    for (int64_t i = 1; i < n; ++i)
        if (e[i].key == e[i - 1].key) { free(e); return ORC_ERR_DUPLICATE; }
    out->e = e;
    out->n = n;
    return ORC_OK;
}

static int build_dim(const orc_probe* pr, dim_map* out) { return build_dim_at(pr, out, 0); }

/* ------------------------------------------------------------------------ */
/* Group store: records [key_0 .. key_{nk-1}, acc_0 .. acc_{na-1}] kept in    */
/* ascending key order; found by binary search, inserted by shifting.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t* rec;
    int64_t n, cap;
    int32_t nk, width;
} group_store;

static int cmp_keys(const int64_t* a, const int64_t* b, int32_t nk) {
    for (int32_t i = 0; i < nk; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

/* Returns the record for key tuple k, inserting a zeroed one if absent. */
static int64_t* group_find(group_store* g, const int64_t* k) {
    int64_t lo = 0, hi = g->n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_keys(g->rec + mid * g->width, k, g->nk);
        if (c == 0) return g->rec + mid * g->width;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    if (g->n == g->cap) {
        int64_t nc = g->cap ? 2 * g->cap : 64;
        int64_t* nr = (int64_t*)realloc(g->rec, (size_t)(nc * g->width) * sizeof(int64_t));
        if (!nr) return NULL;
        g->rec = nr;
        g->cap = nc;
    }
    int64_t* at = g->rec + lo * g->width;
    memmove(at + g->width, at, (size_t)((g->n - lo) * g->width) * sizeof(int64_t));
    memset(at, 0, (size_t)g->width * sizeof(int64_t));
    memcpy(at, k, (size_t)g->nk * sizeof(int64_t));
    g->n += 1;
    return at;
}

/* ------------------------------------------------------------------------ */
/* The query                                                                 */
/* ------------------------------------------------------------------------ */
static int ref_ok(const orc_ref* r, const orc_query* q) {
    if (r->src < 0) return r->idx >= 0 && r->idx < q->nfact && q->fact[r->idx].ival != NULL;
    return r->src < q->nprobes && r->idx >= 0 && r->idx < q->probes[r->src].npay;
}

static int64_t ref_value(const orc_ref* r, const orc_column* fact, int64_t row,
                         const dim_entry* const* hit) {
    if (r->src < 0) return fact[r->idx].ival[row];
    return hit[r->src]->pay[r->idx];
}

/* Rows [r0, r1) of the fact table into the group store g (one row at a
 * time: the predicate atoms, then every probe, then the key tuple and the
 * checked products and sums). */
static int scan_rows(const orc_query* q, const dim_map* dims, int64_t r0, int64_t r1, group_store* g) {
    int rc = ORC_OK;
    const dim_entry* hit[ORC_MAX_PROBES];
    int64_t key[ORC_MAX_KEYS + 1];
    for (int64_t r = r0; r < r1; ++r) {
        int ok = 1;
        for (int32_t i = 0; i < q->npreds && ok; ++i) ok = eval_pred(&q->preds[i], q->fact, r);
        for (int32_t j = 0; j < q->nprobes && ok; ++j) {
            hit[j] = probe_dim(&dims[j], q->fact[q->probes[j].fact_fk_col].ival[r]);
            ok = hit[j] != NULL;
        }
        if (!ok) continue;
        for (int32_t i = 0; i < q->nkeys; ++i) key[i] = ref_value(&q->keys[i], q->fact, r, hit);
        int64_t* rec = group_find(g, key);
        if (!rec) { rc = ORC_ERR_OOM; break; }
        int64_t* acc = rec + q->nkeys;
        if (__builtin_add_overflow(acc[0], (int64_t)1, &acc[0])) { rc = ORC_ERR_OVERFLOW; break; }
        int32_t s = 1;
        for (int32_t a = 0; a < q->naggs && !rc; ++a) {
            const orc_agg* ag = &q->aggs[a];
            if (ag->kind == ORC_AGG_COUNT) continue;
            int64_t prod = 1;
            for (int32_t t = 0; t < ag->nterms && !rc; ++t) {
                const orc_term* tm = &ag->terms[t];
                int64_t v = tm->add;
                if (tm->has_ref) {
                    int64_t x = ref_value(&tm->ref, q->fact, r, hit), mx;
                    if (__builtin_mul_overflow(tm->mul, x, &mx) || __builtin_add_overflow(mx, tm->add, &v))
                        rc = ORC_ERR_OVERFLOW;
                }
                if (!rc && __builtin_mul_overflow(prod, v, &prod)) rc = ORC_ERR_OVERFLOW;
            }
            if (!rc && __builtin_add_overflow(acc[s], prod, &acc[s])) rc = ORC_ERR_OVERFLOW;
            ++s;
        }
        if (rc) break;
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Timing-only variant: the rows are cut into nthreads contiguous ranges,    */
/* each scanned by scan_rows into a group store of its own, and the stores   */
/* are merged by key with checked adds.  It exists to time the oracle on all */
/* host cores; the tests check that its records equal the single-thread     */
/* ones.  (A partial sum that overflows int64 where the whole does not would */
/* be reported as an overflow here; exact int64 results are unaffected.)    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_query* q;
    const dim_map* dims;
    int64_t r0, r1;
    group_store g;
    int rc;
} scan_job;

static void* scan_job_run(void* arg) {
    scan_job* j = (scan_job*)arg;
    j->rc = scan_rows(j->q, j->dims, j->r0, j->r1, &j->g);
    return NULL;
}

static int merge_store(group_store* into, const group_store* from) {
    for (int64_t i = 0; i < from->n; ++i) {
        const int64_t* src = from->rec + i * from->width;
        int64_t* dst = group_find(into, src);
        if (!dst) return ORC_ERR_OOM;
        for (int32_t c = into->nk; c < into->width; ++c)
            if (__builtin_add_overflow(dst[c], src[c], &dst[c])) return ORC_ERR_OVERFLOW;
    }
    return ORC_OK;
}

static int scan_threaded(const orc_query* q, const dim_map* dims, int64_t nrows, int32_t nthreads,
                         group_store* g) {
    if (nthreads > 256) nthreads = 256;
    scan_job* jobs = (scan_job*)calloc((size_t)nthreads, sizeof(scan_job));
    pthread_t* tid = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    char* started = (char*)calloc((size_t)nthreads, 1);
    int rc = (jobs && tid && started) ? ORC_OK : ORC_ERR_OOM;
    for (int32_t t = 0; t < nthreads && !rc; ++t) {
        jobs[t].q = q;
        jobs[t].dims = dims;
        jobs[t].r0 = nrows * t / nthreads;
        jobs[t].r1 = nrows * (t + 1) / nthreads;
        jobs[t].g = *g;  /* empty store of the same shape */
        if (pthread_create(&tid[t], NULL, scan_job_run, &jobs[t]) == 0) started[t] = 1;
        else scan_job_run(&jobs[t]);
    }
    for (int32_t t = 0; jobs && tid && started && t < nthreads; ++t) {
        if (started[t]) pthread_join(tid[t], NULL);
        if (!rc) rc = jobs[t].rc;
        if (!rc) rc = merge_store(g, &jobs[t].g);
        free(jobs[t].g.rec);
    }
    free(jobs);
    free(tid);
    free(started);
    return rc;
}

static int run_query(const orc_query* q, int32_t nthreads, int64_t** out_rows, int64_t* out_ngroups,
                     int32_t* out_ncols) {
    if (!q || !out_rows || !out_ngroups || !out_ncols) return ORC_ERR_INVALID;
    if (q->nfact <= 0 || !q->fact || q->nprobes < 0 || q->nprobes > ORC_MAX_PROBES) return ORC_ERR_INVALID;
    if (q->nkeys < 0 || q->nkeys > ORC_MAX_KEYS || q->naggs < 0 || q->naggs > ORC_MAX_AGGS) return ORC_ERR_INVALID;
    int64_t nrows = q->fact[0].nrows;
    for (int32_t c = 0; c < q->nfact; ++c) {
        if (q->fact[c].nrows != nrows) return ORC_ERR_INVALID;
        if (!q->fact[c].ival && !q->fact[c].str_off) return ORC_ERR_INVALID;
    }
    int rc = check_preds(q->preds, q->npreds, q->fact, q->nfact);
    if (rc) return rc;
    for (int32_t j = 0; j < q->nprobes; ++j) {
        const orc_probe* pr = &q->probes[j];
        if (pr->fact_fk_col < 0 || pr->fact_fk_col >= q->nfact || !q->fact[pr->fact_fk_col].ival)
            return ORC_ERR_INVALID;
    }
    for (int32_t i = 0; i < q->nkeys; ++i)
        if (!ref_ok(&q->keys[i], q)) return ORC_ERR_INVALID;
    /* Output columns: COUNT -> 1, SUM -> 1, AVG -> 2 (sum, count).  Internal
     * accumulators: [count, sum of each SUM/AVG]. */
    int32_t ncols_out = q->nkeys, nsums = 0;
    for (int32_t a = 0; a < q->naggs; ++a) {
        const orc_agg* ag = &q->aggs[a];
        if (ag->kind == ORC_AGG_COUNT) { ncols_out += 1; continue; }
        if (ag->kind != ORC_AGG_SUM && ag->kind != ORC_AGG_AVG) return ORC_ERR_INVALID;
        if (ag->nterms < 1 || ag->nterms > ORC_MAX_TERMS) return ORC_ERR_INVALID;
        for (int32_t t = 0; t < ag->nterms; ++t)
            if (ag->terms[t].has_ref && !ref_ok(&ag->terms[t].ref, q)) return ORC_ERR_INVALID;
        ncols_out += ag->kind == ORC_AGG_AVG ? 2 : 1;
        nsums += 1;
    }

    dim_map dims[ORC_MAX_PROBES];
    memset(dims, 0, sizeof dims);
    for (int32_t j = 0; j < q->nprobes; ++j) {
        rc = build_dim(&q->probes[j], &dims[j]);
        if (rc) goto done;
    }

    group_store g = {NULL, 0, 0, q->nkeys, q->nkeys + 1 + nsums};
    rc = nthreads > 1 ? scan_threaded(q, dims, nrows, nthreads, &g) : scan_rows(q, dims, 0, nrows, &g);

    if (!rc) {
        int64_t* out = (int64_t*)malloc((size_t)((g.n ? g.n : 1) * ncols_out) * sizeof(int64_t));
        if (!out) {
            rc = ORC_ERR_OOM;
        } else {
            for (int64_t i = 0; i < g.n; ++i) {
                const int64_t* rec = g.rec + i * g.width;
                int64_t* o = out + i * ncols_out;
                int32_t c = 0, s = 1;
                for (int32_t k = 0; k < q->nkeys; ++k) o[c++] = rec[k];
                const int64_t* acc = rec + q->nkeys;
                for (int32_t a = 0; a < q->naggs; ++a) {
                    int32_t kind = q->aggs[a].kind;
                    if (kind == ORC_AGG_COUNT) { o[c++] = acc[0]; continue; }
                    o[c++] = acc[s++];
                    if (kind == ORC_AGG_AVG) o[c++] = acc[0];
                }
            }
            *out_rows = out;
            *out_ngroups = g.n;
            *out_ncols = ncols_out;
        }
    }
    free(g.rec);
done:
    for (int32_t j = 0; j < q->nprobes; ++j) free(dims[j].e);
    return rc;
}

int orc_run(const orc_query* q, int64_t** out_rows, int64_t* out_ngroups, int32_t* out_ncols) {
    return run_query(q, 1, out_rows, out_ngroups, out_ncols);
}

int orc_run_threads(const orc_query* q, int32_t nthreads, int64_t** out_rows, int64_t* out_ngroups,
                    int32_t* out_ncols) {
    return run_query(q, nthreads, out_rows, out_ngroups, out_ncols);
}

void orc_free(int64_t* p) { free(p); }

/* Row count of the conjunctive fact filter alone (used by tests as an
 * invariant: the sum of group counts never exceeds it). */
int64_t orc_count_filter(const orc_column* cols, int32_t ncols, const orc_pred* preds, int32_t npreds) {
    if (ncols <= 0 || check_preds(preds, npreds, cols, ncols)) return -1;
    int64_t n = 0;
    for (int64_t r = 0; r < cols[0].nrows; ++r) {
        int ok = 1;
        for (int32_t i = 0; i < npreds && ok; ++i) ok = eval_pred(&preds[i], cols, r);
        n += ok;
    }
    return n;
}

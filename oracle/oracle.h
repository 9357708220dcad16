/*
 * oracle.h -- plain CPU reference for the scan -> filter -> probe -> aggregate
 * query path.  TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke
 * check and the benchmark's CPU-baseline leg, never by the library.
 */
#ifndef DPF_ORACLE_H
#define DPF_ORACLE_H
#include <stdint.h>

#define ORC_MAX_PROBES 8
#define ORC_MAX_KEYS 8
#define ORC_MAX_AGGS 16
#define ORC_MAX_TERMS 3
#define ORC_MAX_PAYLOADS 2

enum { ORC_OK = 0, ORC_ERR_INVALID = 1, ORC_ERR_OVERFLOW = 2, ORC_ERR_DUPLICATE = 3, ORC_ERR_OOM = 4 };
enum { ORC_LT = 1, ORC_LE, ORC_GT, ORC_GE, ORC_EQ, ORC_NE, ORC_BETWEEN, ORC_IN, ORC_STR_CONTAINS_SEQ };
enum { ORC_AGG_COUNT = 0, ORC_AGG_SUM = 1, ORC_AGG_AVG = 2 };

/* An uncompressed column: integers widened to int64, or a string column as
 * nrows + 1 offsets into a byte array. */
typedef struct {
    int64_t nrows;
    const int64_t* ival;
    const int64_t* str_off;
    const uint8_t* str_bytes;
} orc_column;

/* One conjunctive atom.  LT..NE compare with a; BETWEEN is a <= x <= b;
 * IN tests membership in in[0..nin); STR_CONTAINS_SEQ is LIKE '%s1%s2%'. */
typedef struct {
    int32_t col;
    int32_t op;
    int64_t a, b;
    int32_t nin;
    const int64_t* in;
    const uint8_t* s1;
    int32_t n1;
    const uint8_t* s2;
    int32_t n2;
} orc_pred;

/* An inner join of fact column fact_fk_col with the key of a filtered
 * dimension; the dimension's keys must be unique among qualifying rows.
 * The dimension may itself be joined (a build side that is a pipeline, as
 * in the paper's Section 3.1 running example): its rows qualify only if they
 * pass preds and find a match in every one of its nsub own probes sub[]
 * (whose fact_fk_col names a column of this dimension).  Payload k is column
 * pay_col[k] of this dimension when pay_src[k] < 0, else payload pay_col[k]
 * of sub-probe pay_src[k]. */
typedef struct orc_probe_s {
    const orc_column* cols;
    int32_t ncols;
    int32_t key_col;
    const orc_pred* preds;
    int32_t npreds;
    int32_t npay;
    int32_t pay_col[ORC_MAX_PAYLOADS];
    int32_t fact_fk_col;
    int32_t pay_src[ORC_MAX_PAYLOADS];
    const struct orc_probe_s* sub;
    int32_t nsub;
} orc_probe;

/* A value reference: src < 0 -> fact column idx; src = j -> payload idx of
 * probe j. */
typedef struct {
    int32_t src;
    int32_t idx;
} orc_ref;

/* A factor of an aggregate product: mul * ref + add, or add alone. */
typedef struct {
    int32_t has_ref;
    orc_ref ref;
    int64_t mul, add;
} orc_term;

typedef struct {
    int32_t kind;
    int32_t nterms;
    orc_term terms[ORC_MAX_TERMS];
} orc_agg;

typedef struct {
    const orc_column* fact;
    int32_t nfact;
    const orc_pred* preds;
    int32_t npreds;
    const orc_probe* probes;
    int32_t nprobes;
    const orc_ref* keys;
    int32_t nkeys;
    const orc_agg* aggs;
    int32_t naggs;
} orc_query;

/* Evaluates q.  On success *out_rows holds *out_ngroups records of *out_ncols
 * int64 (group keys, then COUNT -> count, SUM -> sum, AVG -> sum, count),
 * ascending by key; free with orc_free.  Returns ORC_OK or an ORC_ERR_*. */
int orc_run(const orc_query* q, int64_t** out_rows, int64_t* out_ngroups, int32_t* out_ncols);
/* The same query with the fact rows split over nthreads threads (timing
 * only: each thread keeps its own groups, merged by key at the end); the
 * records equal orc_run's. */
int orc_run_threads(const orc_query* q, int32_t nthreads, int64_t** out_rows, int64_t* out_ngroups,
                    int32_t* out_ncols);
void orc_free(int64_t* p);
int64_t orc_count_filter(const orc_column* cols, int32_t ncols, const orc_pred* preds, int32_t npreds);

#endif

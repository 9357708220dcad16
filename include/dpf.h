/*
 * dpf.h -- C ABI of the data-path-fusion query library for MI355X (gfx950).
 *
 * One query pipeline = scan compressed column chunks -> decode -> filter ->
 * hash-join probes -> group-by aggregation, run by ONE persistent HIP kernel
 * with no intermediate results materialised (paper Section 3.1, the fused
 * kernels #1..#3; Section 3.2, kernel fusion; Section 4.1, fused kernel
 * composition).  A multi-kernel ("fragmented") execution of the same plan,
 * the form the paper argues against (Section 5.1, the GiDP baseline), is kept
 * beside it.
 *
 * Conventions for every call:
 *  - Returns dpf_status: DPF_OK (0) or a negative DPF_ERR_* code.  On error,
 *    out-parameters are left untouched and dpf_last_error() describes it.
 *  - Nothing throws across this ABI and the library never aborts.
 *  - Host arrays passed in are borrowed for the duration of the call only.
 *  - Handles are reference counted: a plan retains its columns and hashes, a
 *    result retains its plans; *_release drops one reference.
 *  - A context is used by one host thread at a time.
 *  - Device work is enqueued on the caller's stream (a hipStream_t passed as
 *    dpf_stream; NULL is the null stream) and never synchronised inside the
 *    call, except where a call's description says it synchronises.
 *  - Device memory (HBM) and pinned, device-mapped host memory come from the
 *    context's allocator (hipMalloc / hipHostMalloc when none is given).
 *    Blocks of up to 64 MB are recycled inside the context through
 *    power-of-two size classes instead of being freed (hipFree synchronises
 *    the device); they return to the allocator in dpf_ctx_destroy.
 */
#ifndef DPF_H
#define DPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dpf_status;
enum {
    DPF_OK = 0,
    DPF_ERR_INVALID_ARG = -1,   /* bad handle, size, index or combination            */
    DPF_ERR_OOM = -2,           /* an allocation failed                               */
    DPF_ERR_HIP = -3,           /* a HIP runtime call failed                          */
    DPF_ERR_UNSUPPORTED = -4,   /* valid, but outside what this build implements      */
    DPF_ERR_OVERFLOW = -5,      /* an aggregate could exceed int64 (static bound)     */
    DPF_ERR_CAPACITY = -6,      /* a device table ran out of room (reported by kernel) */
    DPF_ERR_DUPLICATE_KEY = -7, /* a hash build met the same key twice                */
    DPF_ERR_CORRUPT = -8,       /* a chunk or mini-block header is inconsistent        */
    DPF_ERR_NOT_READY = -9      /* result read before its work was issued              */
};

typedef struct dpf_ctx_s* dpf_ctx;
typedef struct dpf_column_s* dpf_column;
typedef struct dpf_hash_s* dpf_hash;
typedef struct dpf_plan_s* dpf_plan;
typedef struct dpf_result_s* dpf_result;
typedef void* dpf_stream; /* a hipStream_t */

/* Thread-local description of the last error on this thread; valid until the
 * next call on the thread. */
const char* dpf_last_error(void);

/* ---------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------ */
enum { DPF_MEM_HBM = 0, DPF_MEM_HOST_MAPPED = 1 };

/* Optional allocator.  alloc returns memory of the given kind (HBM, or pinned
 * host memory that the device can address) or NULL; free releases it.  For
 * DPF_MEM_HOST_MAPPED the returned pointer must be a host pointer that
 * hipHostGetDevicePointer accepts.  The library synchronises the device
 * before it hands a block back through free (it does not track which
 * streams used the block). */
typedef struct {
    void* user;
    void* (*alloc)(void* user, size_t bytes, int32_t kind);
    void (*free)(void* user, void* p, int32_t kind);
} dpf_allocator;

/* device >= 0 selects a GPU; device == -1 makes a host-only context in which
 * only encoding, column inspection and host decoding work (placement must be
 * DPF_PLACE_HOST).  allocator may be NULL. */
dpf_status dpf_ctx_create(int32_t device, const dpf_allocator* allocator, dpf_ctx* out);
/* Synchronises the device, then frees everything the context still holds. */
void dpf_ctx_destroy(dpf_ctx ctx);

typedef struct {
    int32_t device;
    int32_t num_cus;           /* compute units                          */
    int64_t lds_per_block;     /* bytes of LDS one workgroup may use     */
    int64_t hbm_bytes;         /* device memory                          */
    int64_t launches;          /* kernels this context has launched      */
} dpf_ctx_info;
dpf_status dpf_ctx_get_info(dpf_ctx ctx, dpf_ctx_info* out);

/* ---------------------------------------------------------------------------
 * Columns: type-specific compression into chunks of mini blocks (paper
 * Section 3.4.1: mini blocks each preceded by a frame-of-reference base, bit
 * width and offset; Section 3.4.2 and Figure 4: variable-length values and
 * the row-id index; Section 4.2: the loader's page-offset, page-size and
 * row-count side arrays).
 *
 * A column is split into chunks of chunk_rows rows (a multiple of 256; the
 * paper's page) and each chunk into mini blocks of 256 values.  Encodings:
 *   FOR    value = base + (packed bits), width per mini block 0..64 bits;
 *   DELTA  value_i = anchor + sum over j <= i of (dmin + packed_j);
 *   DICT   codes (ranks in the sorted distinct values) packed as FOR;
 *   VARLEN string lengths packed as FOR + a contiguous byte heap;
 *   FSST   strings compressed with FSST (paper Sections 3.4.2 and 4.1): one
 *          table of up to 255 symbols of 1..8 bytes per chunk, each string a
 *          run of one-byte codes (code 255 escapes the literal byte after
 *          it), code lengths packed as FOR + a contiguous code heap.
 * AUTO picks VARLEN for strings, DELTA for non-decreasing integers, else FOR.
 * ------------------------------------------------------------------------ */
enum { DPF_TYPE_I32 = 1, DPF_TYPE_I64 = 2, DPF_TYPE_STR = 3 };
enum {
    DPF_ENC_AUTO = 0,
    DPF_ENC_FOR = 1,
    DPF_ENC_DELTA = 2,
    DPF_ENC_DICT = 3,
    DPF_ENC_VARLEN = 4,
    DPF_ENC_PLAIN = 5,
    DPF_ENC_FSST = 6
};
/* PLAIN (integers only) stores every value at full width, 32 bits for I32
 * and 64 for I64, in FOR's layout with a fixed base (INT32_MIN / INT64_MIN):
 * the uncompressed reference that separates the gain of fusion from that of
 * compression (paper Section 5's breakdown).  AUTO never picks it. */
enum { DPF_PLACE_HBM = 0, DPF_PLACE_HOST_MAPPED = 1, DPF_PLACE_HOST = 2 };

/* I32/I64: values points to nrows int32_t / int64_t.  STR: str_offsets has
 * nrows + 1 non-decreasing entries starting at 0 into str_bytes. */
typedef struct {
    int32_t type;
    int64_t nrows;
    const void* values;
    const int64_t* str_offsets;
    const uint8_t* str_bytes;
} dpf_column_src;

/* chunk_rows 0 means 65536.  placement HBM copies the encoded column to
 * device memory; HOST_MAPPED keeps it in pinned host memory that kernels read
 * directly over the host link; HOST keeps it on the host only (tests). */
typedef struct {
    int32_t encoding;
    int32_t chunk_rows;
    int32_t placement;
    int32_t threads; /* encoder threads, 0 = hardware concurrency */
} dpf_encode_opts;

/* Encodes src into a new column.  Copies what it needs from src.  For HBM the
 * upload is complete when the call returns. */
dpf_status dpf_column_encode(dpf_ctx ctx, const dpf_column_src* src, const dpf_encode_opts* opts,
                             dpf_column* out);

typedef struct {
    int32_t type, encoding, placement;
    int32_t chunk_rows;
    int64_t nrows;
    int64_t nchunks;
    int64_t nminiblocks;
    int64_t compressed_bytes; /* bytes a full scan reads: packed data + mini-block headers
                                 (+ dictionary, + string heap) */
    int64_t min, max;         /* integer columns: value range (0, 0 when empty) */
    int64_t ndict;            /* DICT: distinct values                          */
    int64_t str_bytes;        /* strings: decoded bytes (the decode capacity)   */
} dpf_column_stats;
dpf_status dpf_column_info(dpf_column col, dpf_column_stats* out);

/* Per-chunk directory entry: the row-id index (row_start is the prefix sum of
 * row counts) and the zone map (min/max of the chunk's values). */
typedef struct {
    int64_t row_start;
    int64_t nrows;
    int64_t byte_offset, byte_length; /* of the chunk's packed data (or heap, for strings) */
    int64_t min, max;
} dpf_chunk_info;
dpf_status dpf_column_chunk(dpf_column col, int64_t chunk, dpf_chunk_info* out);

/* Host-side decode of the whole column (round-trip checks).  I32/I64: values
 * receives nrows values of the column's type.  STR: str_offsets receives
 * nrows + 1 offsets and str_bytes at most cap bytes.  Returns
 * DPF_ERR_INVALID_ARG if cap is too small. */
dpf_status dpf_column_decode(dpf_column col, void* values, int64_t* str_offsets, uint8_t* str_bytes,
                             size_t cap);

/* For tests of corruption handling: a host pointer to the column's array of
 * mini-block word offsets (nminiblocks + 1 uint32), valid for HOST and
 * HOST_MAPPED placement; writing to it is visible to later kernels. */
dpf_status dpf_column_debug_offsets(dpf_column col, uint32_t** offsets);
void dpf_column_release(dpf_column col);

/* ---------------------------------------------------------------------------
 * Predicates (conjunctive atoms; paper Section 3.1 and Section 4.1: filters
 * and a LIKE-style string matcher evaluated inside the fused kernel)
 * ------------------------------------------------------------------------ */
enum {
    DPF_OP_LT = 1, DPF_OP_LE, DPF_OP_GT, DPF_OP_GE, DPF_OP_EQ, DPF_OP_NE,
    DPF_OP_BETWEEN,         /* a <= x <= b                                        */
    DPF_OP_IN,              /* x equals one of in_values[0..n_in), n_in <= 64      */
    DPF_OP_STR_CONTAINS_SEQ /* s1 occurs and s2 occurs at or after its end
                               (LIKE '%s1%s2%'); 1 <= n1, n2 <= 32 bytes; on a
                               VARLEN or FSST column.  A plan takes at most one
                               such atom on an FSST column (DPF_ERR_UNSUPPORTED
                               otherwise): the fused kernel keeps one code
                               table of (2 (n1 + n2 + 1) + 1) x 256 bytes per
                               workgroup in LDS (paper Sections 3.4.2, 4.1)   */
};
typedef struct {
    int32_t col; /* index into the column array of the enclosing description */
    int32_t op;
    int64_t a, b;
    int32_t n_in;
    const int64_t* in_values;
    const uint8_t* s1;
    int32_t n1;
    const uint8_t* s2;
    int32_t n2;
} dpf_pred;

/* ---------------------------------------------------------------------------
 * Dimension hash tables (paper Section 3.1, Kernel #1: scan a dimension,
 * filter it and build the hash table a later pipeline probes; Section 4.3:
 * the build side must fit in GPU memory).
 * ------------------------------------------------------------------------ */
enum { DPF_HASH_AUTO = 0, DPF_HASH_LDS = 1, DPF_HASH_HBM = 2 };
typedef struct {
    int32_t fk_col;
    dpf_hash hash;
} dpf_probe;

typedef struct {
    int32_t ncols;
    const dpf_column* cols;     /* dimension columns (same row count)          */
    int32_t key_col;            /* unique among qualifying rows; values must fit
                                   int32 and differ from INT32_MIN              */
    int32_t npreds;
    const dpf_pred* preds;      /* integer predicates over cols                */
    int32_t npayloads;          /* 0..2 payloads                                */
    int32_t payload_cols[2];    /* payload k: integer column payload_cols[k], or
                                   (payload_probe[k] >= 0) payload number
                                   payload_cols[k] of probe payload_probe[k]     */
    int32_t placement;          /* where probes keep the table (AUTO: LDS when
                                   it fits the per-workgroup LDS budget)       */
    /* A joined build side (paper Section 3.1, Kernel #2: a scan that probes an
     * earlier table and builds the next): 0..2 probes of tables already built,
     * each by an integer column fk_col of cols.  A row enters the table only
     * if it passes preds and every probe finds its foreign key; the probed
     * tables are read during the call only. */
    int32_t nprobes;
    const dpf_probe* probes;
    int32_t payload_probe[2];   /* -1: payload k is a column of cols           */
} dpf_hash_desc;

/* Builds an open-addressing table (power-of-two capacity, load <= 1/2) in HBM
 * from the qualifying rows.  Synchronises the stream (the entry count sizes
 * the table).  DPF_ERR_DUPLICATE_KEY if a key repeats. */
dpf_status dpf_hash_build(dpf_ctx ctx, const dpf_hash_desc* desc, dpf_stream stream, dpf_hash* out);

typedef struct {
    int64_t entries, capacity, bytes;  /* bytes: keys and payloads (what an LDS copy takes) */
    int32_t lds_eligible, placement;
    int32_t npayloads;
    int64_t key_min, key_max;
    int64_t payload_min[2], payload_max[2];
    int64_t device_bytes;              /* the table's device allocation: keys, payloads,
                                          membership bitmap and bit filter */
} dpf_hash_stats;
dpf_status dpf_hash_info(dpf_hash h, dpf_hash_stats* out);
void dpf_hash_release(dpf_hash h);

/* ---------------------------------------------------------------------------
 * Plans: scan(cols) -> filter(preds) -> probe(fk, hash)* -> group by keys ->
 * aggregates (paper Section 3.1: the host generates the plan; Kernel #3
 * probes and aggregates; the result returns in record form).
 * ------------------------------------------------------------------------ */
enum { DPF_REF_COL = 0, DPF_REF_PAYLOAD = 1 };
typedef struct {
    int32_t kind;  /* DPF_REF_COL: fact column idx; DPF_REF_PAYLOAD: payload idx of probe */
    int32_t idx;
    int32_t probe;
} dpf_ref;

/* A factor mul * ref + add (or add alone when has_ref is 0). */
typedef struct {
    int32_t has_ref;
    dpf_ref ref;
    int64_t mul, add;
} dpf_term;

enum { DPF_AGG_COUNT = 0, DPF_AGG_SUM = 1, DPF_AGG_AVG = 2 };
/* COUNT -> one output column; SUM(product of terms) -> one; AVG -> two (sum,
 * count): an exact average as a pair. */
typedef struct {
    int32_t op;
    int32_t nterms; /* 1..3 for SUM and AVG */
    dpf_term terms[3];
} dpf_agg;

typedef struct {
    int32_t ncols;
    const dpf_column* cols;  /* fact columns, all of the same table */
    int32_t npreds;
    const dpf_pred* preds;
    int32_t nprobes;         /* probed in this order (put the most selective first) */
    const dpf_probe* probes;
    int32_t nkeys;
    const dpf_ref* keys;
    int32_t naggs;
    const dpf_agg* aggs;
} dpf_plan_desc;

/* Validates the plan, proves every aggregate stays within int64 over the
 * table (else DPF_ERR_OVERFLOW), sizes the group table and pre-allocates the
 * per-plan device workspace and pinned result buffer (paper Section 3.1,
 * Kernels #3 and #4).  The group table is indexed by the group keys'
 * combined value range (the product of each key's max - min + 1): directly
 * up to 2^22 slots; above that it is an open-addressing hash table in
 * device memory whose slot count is a power of two at least twice
 * min(range, table rows), at most 2^22 slots, as the direct table (else
 * DPF_ERR_UNSUPPORTED, as for a range above 2^62): the workgroup that
 * finishes last scans the table to emit the records.  Executing the plan then allocates nothing and
 * can be captured in a HIP graph.  The device
 * copy of the plan (its descriptor, the surviving-block list and the zeroed
 * workspace) is enqueued on the context's own upload stream from pinned
 * staging, and the call returns without waiting for it: every execution
 * orders itself after that upload (a stream wait on its event, or a host
 * wait when the execution is being captured into a graph). */
dpf_status dpf_plan_build(dpf_ctx ctx, const dpf_plan_desc* desc, dpf_plan* out);

/* Device memory the plan itself holds, for admission control: its workspace
 * (descriptor, group table, status word, queue counters, surviving-block
 * list) and, once it has run fragmented, that path's intermediate buffers.
 * The dimension hash tables it probes belong to their own handles and are
 * not counted (dpf_hash_stats.device_bytes gives them), so that a table many
 * plans share is charged once. */
dpf_status dpf_plan_footprint(dpf_plan plan, size_t* hbm_bytes);

/* Chunk pruning (paper Section 3.1.1: predicates checked against zone maps
 * before the scan).  At plan build, a mini block is excluded when the
 * min/max its column recorded for the chunk holding it rules out one fact
 * atom for every row (string columns record lengths: rows shorter than
 * |s1| + |s2| cannot match), or when one probe's foreign keys all fall
 * outside the qualifying keys' range.  The fused execution then scans only
 * the blocks (the smallest chunk of the plan's columns) that keep a mini
 * block; the fragmented one scans everything, with the same result.
 * *total_blocks receives the plan's blocks, *scanned_blocks those it scans. */
dpf_status dpf_plan_blocks(dpf_plan plan, int64_t* scanned_blocks, int64_t* total_blocks);
void dpf_plan_release(dpf_plan plan);

/* ---------------------------------------------------------------------------
 * Execution
 * ------------------------------------------------------------------------ */
enum { DPF_MODE_FUSED = 0, DPF_MODE_FRAGMENTED = 1 };
typedef struct {
    int32_t mode;
    int32_t wg_per_cu;       /* FUSED: workgroups per compute unit (0 = auto)          */
    int32_t rows_per_item;   /* FUSED: rows per work item, multiple of 256 (0 = auto:   */
                             /* at most 16384, about three items per workgroup; even   */
                             /* slices of a pruned plan's blocks)                       */
    int32_t lds_hash_bytes;  /* FUSED: LDS budget for dimension tables (-1 = auto:     */
                             /* 72 KB, none for batches of more than 8 plans)          */
    int32_t waves_per_wg;    /* FUSED: 4, 8 or 16 waves per workgroup (0 = auto)       */
    int32_t max_workgroups;  /* FUSED: cap on the grid (0 = none).  A scan bound by the
                                host link needs few workgroups; a small grid leaves the
                                other CUs' slots and memory queues to concurrent work */
} dpf_exec_opts;

/* Enqueues n >= 1 plans on stream.  FUSED runs them all in ONE launch of the
 * persistent kernel, which claims (plan, row range) work items from a device
 * queue; FRAGMENTED runs each plan as a sequence of separate kernels with
 * materialised intermediates (it allocates on first use and is not meant for
 * graph capture).  FUSED with n <= 64 allocates no device memory and is
 * graph-capturable.  Outside stream capture the call records a completion
 * event on the stream for dpf_result_release.  A plan must not be in two
 * executions at once.  *out receives a result handle that is readable after
 * the stream has synchronised. */
dpf_status dpf_execute(dpf_ctx ctx, int32_t n, const dpf_plan* plans, const dpf_exec_opts* opts,
                       dpf_stream stream, dpf_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the fused
 * execution of dpf_execute with the same arguments and results, except that
 * the launch's scratch state -- the work-queue counters and each plan's group
 * table and status word, which dpf_execute keeps in the plans' workspaces --
 * lives in one static device array of 8 MiB per GPU (held by the library
 * until the process ends).  The call allocates no device or pinned memory
 * and creates no event.  mode must be DPF_MODE_FUSED (else
 * DPF_ERR_UNSUPPORTED).  The scratch needed is 2,304 bytes of counters plus,
 * per plan, 256 bytes of status and the group table (slots x accumulators
 * x 8 bytes, plus slots x 8 bytes of keys for a hash table), each rounded up
 * to 256 bytes; a batch needing more than
 * 8 MiB is refused with DPF_ERR_UNSUPPORTED before anything is enqueued.  The
 * call zeroes the part of the array it uses on the stream before its launch
 * (the array keeps the previous call's contents).  Every call on one GPU
 * shares that GPU's array: calls whose work overlaps on the device race and
 * give wrong results, so order them (one stream, or events).  The records
 * still go to each plan's pinned result buffer: synchronise the stream, then
 * read them with dpf_result_get; release the result only after that
 * synchronisation (it holds no completion event to wait for). */
dpf_status dpf_execute_noalloc(dpf_ctx ctx, int32_t n, const dpf_plan* plans, const dpf_exec_opts* opts,
                               dpf_stream stream, dpf_result* out);

/* Reads plan i's records after the work has completed (the caller
 * synchronises the stream).  Rows are int64: group key values, then the
 * aggregate columns, one row per non-empty group, ascending by key.  Returns
 * the device-reported status (e.g. DPF_ERR_CAPACITY, DPF_ERR_CORRUPT) and no
 * rows when the kernel reported an error.  The records live in the plan's
 * one pinned result buffer, which every execution of that plan overwrites:
 * read a result before the plan runs again.  Each call decodes the buffer
 * anew (so a result captured in a graph can be read after every replay);
 * *rows stays valid until the next call on the same result or its release. */
dpf_status dpf_result_get(dpf_result res, int32_t i, int64_t* ngroups, int32_t* ncols,
                          const int64_t** rows);
/* Waits for the execution to finish (its completion event; a captured
 * execution has none, and its replays are the caller's to order), then drops
 * the result's references to its plans, whose memory may be recycled. */
void dpf_result_release(dpf_result res);

/* ---------------------------------------------------------------------------
 * Measurement helper (not part of a query; the bandwidth ceilings the scan
 * is compared against, paper Section 5.1 measures its IO path the same way)
 * ------------------------------------------------------------------------ */
/* Read bandwidth that kernels reach from memory of one kind (DPF_MEM_HBM, or
 * DPF_MEM_HOST_MAPPED: pinned host memory read over the host link).
 * Allocates bytes (a positive multiple of 16) from the context's allocator,
 * fills it, then enqueues reps (1..1000) launches of a streaming kernel on
 * stream -- grid workgroups of 256 lanes (0: 8 per CU), 16-byte loads, four
 * in flight per lane -- each bracketed by HIP events.  ms[0..reps) receives
 * each launch's time.  Synchronises the stream and frees the buffer before
 * returning. */
dpf_status dpf_measure_read(dpf_ctx ctx, int32_t kind, size_t bytes, int32_t grid, int32_t reps,
                            dpf_stream stream, float* ms);

#ifdef __cplusplus
}
#endif
#endif /* DPF_H */

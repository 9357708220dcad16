// dpf_internal.h -- descriptors shared by the host runtime and the gfx950
// kernels.  A plan is flattened into one DevQuery in device memory; the
// persistent kernel reads it with scalar (wave-uniform) loads.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dpf {

constexpr int kMB = 256;          // values per mini block
constexpr int kWave = 64;         // CDNA wavefront
constexpr int kWaves = 4;         // waves per workgroup
constexpr int kBlock = kWave * kWaves;
constexpr int kMaxCols = 16;      // fact columns per plan
constexpr int kMaxPreds = 12;     // predicate atoms per plan
constexpr int kMaxProbes = 4;     // probes per plan
constexpr int kMaxSlots = 8;      // values carried per surviving row
constexpr int kMaxKeys = 4;       // group-by keys
constexpr int kMaxAccs = 12;      // accumulators (count + sums)
constexpr int kMaxTerms = 3;      // factors per aggregate product
constexpr int kMaxIn = 64;        // IN-list values per plan
constexpr int kMaxWord = 32;      // bytes per string-predicate word
constexpr int kMaxBatch = 64;     // plans per fused launch
constexpr int kMaxHashCols = 8;   // dimension columns per hash build
constexpr int kMaxHashPreds = 8;  // dimension predicates per hash build
constexpr int64_t kMaxGroups = int64_t(1) << 22;  // direct-indexed group table limit
constexpr int64_t kMaxHashSlots = int64_t(1) << 22;  // hash group table limit (slots; one workgroup emits it)
constexpr int64_t kMaxGroupDomain = int64_t(1) << 62;  // group index + 1 fits int64
constexpr int32_t kEmptyKey = INT32_MIN;
constexpr int kXcds = 8;             // XCDs per device; workgroup i is dispatched to XCD i % 8
constexpr int kCounterStride = 32;   // 32-bit words between work-queue counters (128-byte lines)
constexpr int kCounterWords = (2 * kXcds + 1) * kCounterStride;

enum : int32_t { ENC_FOR = 1, ENC_DELTA = 2, ENC_DICT = 3, ENC_VARLEN = 4, ENC_FSST = 6 };

// Device view of one encoded column (all arrays indexed by global mini block).
struct DevCol {
    const int64_t* base;    // [nmb] FOR base | DELTA anchor | DICT code base | VARLEN min length
    const uint32_t* woff;   // [nmb + 1] first word of each mini block's packed data
    const uint32_t* words;  // packed values, LSB first, value i at bit i * width
    const int64_t* dmin;    // DELTA: [nmb] minimum first difference
    const uint64_t* hoff;   // VARLEN, FSST: [nmb + 1] byte offset of the mini block's strings (codes)
    const uint8_t* heap;    // VARLEN: string bytes; FSST: codes (padded)
    const int64_t* dict;    // DICT: [ndict] sorted distinct values
    const uint64_t* doff;   // FSST: [nmb + 1] decoded byte offset of each mini block
    const uint8_t* symtab;  // FSST: per chunk, sym[256] (uint64) then len[256] (uint8)
    int64_t nrows;
    uint64_t heap_bytes;
    uint64_t str_bytes;     // VARLEN, FSST: decoded string bytes
    uint32_t nwords;
    int32_t nmb;
    int32_t enc;
    int32_t ndict;
    int32_t mbpc;           // mini blocks per chunk (FSST: mini block m uses table m / mbpc)
    int32_t pad;
};

enum : int32_t { PK_RANGE = 1, PK_NE = 2, PK_INMASK = 3, PK_INLIST = 4, PK_STR = 5, PK_FALSE = 6 };

// One conjunctive atom, already rewritten into the column's code space
// (dictionary columns compare codes).
struct DevPred {
    int32_t col;
    int32_t kind;
    int64_t lo, hi;     // RANGE: lo <= x <= hi; NE: x != lo
    uint64_t mask;      // INMASK: bit c set -> code c qualifies (codes < 64)
    int32_t in_off;     // INLIST: values in_vals[in_off .. in_off + n_in)
    int32_t n_in;
    int32_t n1, n2;     // STR: word lengths
    uint8_t s1[kMaxWord];
    uint8_t s2[kMaxWord];
    // STR with both words of at least 7 bytes: lookup table of the aligned-
    // word test.  The eight 4-byte shifts (bytes [j, j + 4), j < 4) of s1
    // and s2 sit at slot str_slot(x, tab_rot); a free slot i holds a word
    // whose slot is not i, so a word x is a shift iff tab[str_slot(x)] == x.
    // tab_rot = 0: no rotation separates the shifts (no table).
    uint32_t tab_rot;
    uint32_t tab[32];
};

// Slot of a 4-byte word in DevPred::tab: bits 2..6 of x ^ rotr(x, r).
__host__ __device__ inline uint32_t str_slot(uint32_t x, uint32_t r) {
    return ((x ^ ((x >> r) | (x << ((32u - r) & 31u)))) & 0x7Cu) >> 2;
}

// Workgroup LDS of the fused kernel: the string-scan table (DevPred::tab of
// the plan's last atom, static LDS), then, dynamic, control words, the
// shared area and the per-wave areas.
constexpr size_t kLdsCtrlBytes = 64;
constexpr size_t kLdsStrTabBytes = 128;
constexpr size_t kLdsHeadBytes = kLdsCtrlBytes + kLdsStrTabBytes;  // counted against the CU's LDS

// Open-addressing table: int32 keys (kEmptyKey = free), payload arrays
// follow the key array in the same allocation.  When the qualifying keys
// span at most kMaxBitmapBits values, a membership bitmap over [bmin, bmin +
// bspan) follows as well: a probe that needs no payload tests one bit.
constexpr uint64_t kMaxBitmapBits = uint64_t(1) << 25;  // 4 MB
struct DevHash {
    const int32_t* keys;
    const void* pay[2];
    const uint32_t* bits;  // nullptr: no bitmap
    int64_t bmin;
    uint64_t bspan;
    uint32_t cap_mask;
    int32_t log2cap;
    int32_t npay;
    int32_t pay64[2];   // payload k stored as int64 (else int32)
    int32_t lds_off;    // >= 0: byte offset of the workgroup's LDS copy
    uint32_t bytes;     // keys + payloads
    // Two-hash bit filter over the keys (small tables only): a probe of a
    // table left in HBM first tests the workgroup's LDS copy of the filter.
    const uint32_t* filt;  // nullptr: none
    int32_t flog2;         // filter bits = 2^flog2
    int32_t filt_lds_off;  // >= 0: byte offset of the LDS copy
    int32_t bits_lds_off;  // >= 0: byte offset of an LDS copy of the bitmap
};
constexpr int kMaxFilterLog2 = 18;  // 32 KB
// The filter's two bit positions, both in one 32-bit word (a blocked
// filter: one LDS read a probe): top bits of 24-bit products, a full-rate
// multiply on the GPU where a 32-bit one issues at quarter rate.  Keys that
// differ only above bit 23 share their bits: more false positives, never a
// missed key.
__host__ __device__ inline uint32_t filter_bit(int32_t key, int flog2) {
    return (((uint32_t)key & 0xFFFFFFu) * 0x2545F5u) >> (32 - flog2);
}
__host__ __device__ inline uint32_t filter_bit2(int32_t key, int flog2) {
    return (filter_bit(key, flog2) & ~31u) | (((((uint32_t)key & 0xFFFFFFu) * 0x9E3779u) + 0x7F4A7C15u) >> 27);
}

struct DevProbe {
    int32_t fk_col;
    int32_t pay_slot[2];  // value slot receiving payload k (-1: unused)
    DevHash h;
};

struct DevLoad { int32_t col, slot, dict_val, pad; };  // fact column -> value slot (DICT: code or value)
struct DevKey { int32_t slot; int32_t pad; int64_t min, card, stride; };
struct DevTerm { int32_t slot; int32_t pad; int64_t mul, add; };  // slot < 0: constant add
struct DevAcc { int32_t nterms; int32_t pad; DevTerm t[kMaxTerms]; };

enum : uint32_t { ST_CORRUPT = 1u, ST_CAPACITY = 2u, ST_UNSUPPORTED = 4u, ST_DUPLICATE = 8u };

struct DevQuery {
    int64_t nrows;
    int32_t nmb;
    int32_t ncols;
    DevCol cols[kMaxCols];
    int32_t npreds;  // integer atoms first, then string atoms
    int32_t nint_preds;
    DevPred preds[kMaxPreds];
    int64_t in_vals[kMaxIn];
    int32_t nprobes;
    int32_t nloads;
    DevProbe probes[kMaxProbes];
    DevLoad loads[kMaxSlots];
    int32_t nkeys;
    int32_t nacc;    // accumulator 0 is the row count
    DevKey keys[kMaxKeys];
    DevAcc accs[kMaxAccs];
    // Group table: ngroups rows of nacc accumulators, zero between
    // executions.  Direct (agg_hash 0): row g is group index g.  Hash
    // (agg_hash 1, a group-key domain above kMaxGroups): ngroups is a power
    // of two at least twice the groups the table can receive, and ngroups
    // keys follow the accumulators (group index + 1; 0: empty slot), placed
    // by linear probing.
    int64_t ngroups;
    int64_t* agg;
    int32_t agg_lds;     // accumulate in the workgroup's LDS table first
    int32_t agg_lds_off; // byte offset of that table
    int32_t lds_shared;  // LDS bytes of this plan's shared area (hashes + table)
    int32_t has_str;
    int32_t agg_hash;
    int32_t agg_pad;
    // The string atom on an FSST column (index into preds, -1: none): its
    // byte automaton (fs_states rows of 256 next states, device memory) and
    // the byte offset of its code table ((2 fs_states + 1) rows of 256) in
    // the shared area.
    int32_t fs_pred;
    int32_t fs_lds_off;
    int32_t fs_states;
    int32_t fs_pad;
    const uint8_t* fs_dfa;
    uint32_t* status;    // device status bits (ST_*)
    int64_t* host_out;   // device address of the pinned output: [status, nrec, records...]
    // Chunk pruning: null, or the ascending indices of the blocks of
    // prune_mb mini blocks that the zone maps do not exclude; the fused
    // kernel's work items then cover those blocks only.
    const int32_t* live;
    int32_t nlive;
    int32_t prune_mb;
};

// Bytes of a plan's group table: the accumulators, and the keys of a hash
// table.
inline size_t agg_table_bytes(const DevQuery& q) {
    return (size_t)q.ngroups * (size_t)(q.nacc + (q.agg_hash ? 1 : 0)) * 8;
}

struct BatchArgs {
    const DevQuery* q[kMaxBatch];
    // Per plan: its group table (agg_table_bytes, zero between
    // executions) and its status word, in the plan's workspace or in the
    // library's static scratch area.
    int64_t* agg[kMaxBatch];
    uint32_t* status[kMaxBatch];
    int32_t item_start[kMaxBatch + 1];
    int32_t nq;
    int32_t mb_per_item;
    uint32_t* counters;   // kCounterWords: per XCD x, the claim head of item range x (line x) and
                          // its finished workgroups (line 8 + x); finished XCDs (line 16)
    int32_t lds_shared;   // max lds_shared over the batch
    int32_t str_stage;    // per-wave string staging present (2: some plan has an FSST atom)
    int32_t pend_stage;   // per-wave survivor queue present (some plan has a fact predicate or a probe)
    int32_t agg_hash;     // some plan aggregates into a hash group table
};

// Hash build over a dimension table (optionally joined: the rows must find
// their foreign keys in the tables of sub[], probed from device memory).
struct HashBuildArgs {
    DevCol cols[kMaxHashCols];
    int32_t ncols;
    int32_t npreds;
    DevPred preds[kMaxHashPreds];
    int64_t in_vals[kMaxIn];
    int32_t key_col;
    int32_t npay;
    int32_t pay_col[2];   // column, or (pay_src >= 0) payload index of sub[pay_src]
    int32_t pay_src[2];   // -1: a column of cols
    int32_t nsub;
    DevProbe sub[2];
    int32_t nmb;
    int32_t pad;
    int64_t nrows;
    // outputs
    unsigned long long* count;  // qualifying rows
    long long* mm;              // [0..1] key min/max, [2..5] payload min/max
    uint32_t* status;
    // insert pass
    int32_t* keys;
    void* pay[2];
    int32_t pay64[2];
    uint32_t cap_mask;
    int32_t log2cap;
    uint32_t* bits;     // membership bitmap (nullptr: none)
    int64_t bmin;
    uint32_t* filt;     // bit filter (nullptr: none)
    int32_t flog2;
    int32_t pad2;
};

// Launchers (kernels.hip).  Each returns the hipError_t of the launch.
// waves: 4, 8 or 16 waves per workgroup.
hipError_t launch_fused(const BatchArgs& a, int waves, int grid, size_t lds_bytes, hipStream_t s);
// Per-wave LDS the fused kernel needs (survivor queue, string row offsets).
size_t fused_wave_area_bytes(bool str, bool pend);
hipError_t launch_hash_count(const HashBuildArgs* d_args, int grid, hipStream_t s);
hipError_t launch_hash_insert(const HashBuildArgs* d_args, int grid, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// Bandwidth probe: grid x 256 lanes read bytes (a multiple of 16) at p.
hipError_t launch_stream_read(const void* p, uint64_t bytes, uint32_t key, uint32_t* sink, int grid,
                              hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);

// Fragmented (multi-kernel) execution of one plan.  Row lists hold row ids
// as uint32: plans cover at most 2^32 - 1 rows, and every decoded array is
// indexed with the id widened to 64 bits.
typedef uint32_t FragRow;
static_assert(sizeof(FragRow) == 4 && FragRow(-1) == UINT32_MAX, "row ids must reach 2^32 - 1");
struct FragBuffers {
    int64_t* dec[kMaxCols];      // decoded integer columns (codes for DICT)
    int64_t* str_off[kMaxCols];  // decoded string offsets [nrows + 1]
    uint8_t* str_bytes[kMaxCols];
    const DevCol* str_col[kMaxCols];  // the column's descriptor with its heap at str_bytes
    uint8_t* flags;              // [nrows]
    FragRow* rows[2];            // ping-pong row lists [nrows]
    int64_t* pay[2][2 * kMaxProbes];  // payload arrays aligned with the row lists
    unsigned long long* counts;  // [kMaxProbes + 2] list lengths
};
// Returns the number of kernels launched, or -1 on a launch error.
int run_fragmented(const DevQuery* d_q, const DevQuery& h_q, const FragBuffers& fb, hipStream_t s);

}  // namespace dpf

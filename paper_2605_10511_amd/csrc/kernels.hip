// kernels.hip -- gfx950 kernels of the data-path-fusion query library.
//
//  * fused_kernel: ONE persistent kernel per launch runs whole query
//    pipelines (paper Section 3.2 and Section 4.1 "Fused kernel
//    composition"): each workgroup claims (plan, mini-block range) work
//    items from a device queue; its waves each take one 256-row mini block at
//    a time, decode the referenced columns straight from where the chunks
//    rest (HBM or pinned host memory mapped into the device), filter, and
//    queue the surviving row ids in LDS; full batches of 64 survivors are
//    probed against the dimension hash tables (LDS copies for small ones) and
//    aggregated into a per-workgroup LDS table.  The last workgroup to finish
//    writes the records to the host buffer -- nothing is materialised in
//    between.
//  * hash_count / hash_insert: the build side (Section 3.1, Kernel #1).
//  * frag_*: the same plan as separate kernels with materialised
//    intermediates (Section 5.1, the multi-kernel baseline).
//
// Work mapping inside a mini block: lane l of a wave owns rows l, l+64,
// l+128, l+192, so every load instruction of the wave covers a contiguous
// run of packed bits (row i sits at bit i * width).
#include <hip/hip_runtime.h>

#include "dpf_internal.h"

namespace dpf {
namespace {

// Descriptors and encoded columns are read-only during a launch, so the
// kernels read them through the constant address space: wave-uniform reads
// (headers, descriptor fields) become scalar loads and per-lane reads become
// global loads, never flat ones.
#define DPF_AS_CONST __attribute__((address_space(4)))
template <class T>
using cptr = const DPF_AS_CONST T*;
template <class T>
__device__ __forceinline__ cptr<T> ro(const T* p) { return (cptr<T>)p; }
using CQ = const DPF_AS_CONST DevQuery;
using CC = const DPF_AS_CONST DevCol;
using CP = const DPF_AS_CONST DevPred;
using CH = const DPF_AS_CONST DevHash;
using CPR = const DPF_AS_CONST DevProbe;
using CL = const DPF_AS_CONST DevLoad;
using CK = const DPF_AS_CONST DevKey;
using CT = const DPF_AS_CONST DevTerm;
using CA = const DPF_AS_CONST DevAcc;
using CHB = const DPF_AS_CONST HashBuildArgs;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld4(cptr<uint4> g, uint32_t i) {
    const u32x4 t = ((cptr<u32x4>)g)[i];
    return make_uint4(t.x, t.y, t.z, t.w);
}

constexpr int kPendCap = 320;   // per-wave survivor queue (64 pending + one mini block)
constexpr int kSegIters = 2;    // 16-byte string loads per lane per segment (2 KB per wave, double-buffered)
constexpr int kRecCap = 64;     // per-wave queue of string words with a prefix hit (16 B each)

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t bits_below(uint64_t b) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ __forceinline__ int32_t uniform_i32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Cross-lane moves through DPP (GFX9 data-parallel primitives): no address
// registers, no LDS.  A lane whose source is outside the pattern, or whose
// row is masked off, receives 0.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppWaveShl1 = 0x130;  // lane i receives lane i + 1
constexpr int kDppWaveShr1 = 0x138;  // lane i receives lane i - 1
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, kRowMask, 0xf, false);
}

template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    const uint32_t lo = dpp_u32<kCtrl, kRowMask>((uint32_t)x);
    const uint32_t hi = dpp_u32<kCtrl, kRowMask>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive wave scans: shifts 1, 2, 4, 8 inside each 16-lane row, then lane
// 15 of a row is added to the next row and lane 31 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += dpp_u32<kDppRowShr1>(x);
    x += dpp_u32<kDppRowShr2>(x);
    x += dpp_u32<kDppRowShr4>(x);
    x += dpp_u32<kDppRowShr8>(x);
    x += dpp_u32<kDppRowBcast15, 0xa>(x);
    x += dpp_u32<kDppRowBcast31, 0xc>(x);
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    x += dpp_u64<kDppRowShr1>(x);
    x += dpp_u64<kDppRowShr2>(x);
    x += dpp_u64<kDppRowShr4>(x);
    x += dpp_u64<kDppRowShr8>(x);
    x += dpp_u64<kDppRowBcast15, 0xa>(x);
    x += dpp_u64<kDppRowBcast31, 0xc>(x);
    return x;
}

// Orders this wave's LDS accesses (a wave's LDS operations complete in issue
// order; the fence keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Bit unpacking (paper Section 3.4.1 and 4.1: FOR with a per-mini-block base
// and bit width; the 64-bit variant reads through a wider window)
// ---------------------------------------------------------------------------
typedef uint64_t u64_a4 __attribute__((aligned(4)));

__device__ __forceinline__ uint64_t bits_at(cptr<uint32_t> w, uint32_t bitpos, int b) {
    cptr<uint32_t> p = w + (bitpos >> 5);
    uint32_t sh = bitpos & 31u;
    uint64_t x = *(cptr<u64_a4>)p >> sh;
    if (b > 32) {
        uint64_t hi = p[2];
        if (sh) x |= hi << (64 - sh);
    }
    return b >= 64 ? x : (x & ((uint64_t(1) << b) - 1));
}

struct MbHdr {
    int64_t base;
    cptr<uint32_t> w;
    int b;
    bool ok;
};

// Mini-block header with consistency checks (a corrupt header must not
// steer a load out of bounds).
__device__ __forceinline__ MbHdr mb_hdr(CC& c, int m) {
    MbHdr h;
    uint32_t w0 = ro(c.woff)[m], w1 = ro(c.woff)[m + 1];
    uint32_t nw = w1 - w0;
    h.ok = (w0 <= w1) && (w1 <= c.nwords) && ((nw & 7u) == 0) && (nw <= 512u);
    h.b = (int)(nw >> 3);
    h.base = ro(c.base)[m];
    h.w = ro(c.words) + (h.ok ? w0 : 0);
    if (!h.ok) h.b = 0;
    return h;
}

// Dense decode of the wave's four rows (64k + lane) of mini block m.
// DICT columns yield codes; VARLEN yields lengths.  Returns false on a
// corrupt header.
// Dense decode in two steps, so that a wave can have the loads of several
// mini blocks in flight: issue_dense reads the header and the packed words
// (raw 64-bit windows, or the full values for widths above 32), and
// finish_dense unpacks them (DELTA: a wave scan).
struct RawDense {
    MbHdr h;
    int64_t dmin;
    uint64_t raw[4];
    uint32_t sh[4];
};

__device__ __forceinline__ void issue_dense(CC& c, int m, int lane, RawDense& R) {
    R.h = mb_hdr(c, m);
    R.dmin = c.enc == ENC_DELTA ? ro(c.dmin)[m] : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t bitpos = (uint32_t)(64 * k + lane) * (uint32_t)R.h.b;
        R.sh[k] = bitpos & 31u;
        if (R.h.b == 0) {
            R.raw[k] = 0;
        } else if (R.h.b <= 32) {
            R.raw[k] = *(cptr<u64_a4>)(R.h.w + (bitpos >> 5));
        } else {
            R.raw[k] = bits_at(R.h.w, bitpos, R.h.b);
            R.sh[k] = 0;
        }
    }
}

__device__ __forceinline__ bool finish_dense(CC& c, const RawDense& R, int lane, int64_t v[4]) {
    const MbHdr& h = R.h;
    uint64_t u[4];
    const uint64_t mask = h.b >= 64 ? ~uint64_t(0) : ((uint64_t(1) << h.b) - 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = h.b == 0 ? 0 : ((R.raw[k] >> R.sh[k]) & mask);
    if (c.enc == ENC_DELTA) {
        // value_i = anchor + i * dmin + sum_{j <= i} packed_j  (packed_0 = 0)
        const uint64_t dmin = (uint64_t)R.dmin;
        uint64_t carry = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint64_t s = h.b ? wave_incl_scan_u64(u[k]) : 0;
            uint32_t i = 64 * k + lane;
            v[k] = (int64_t)((uint64_t)h.base + (uint64_t)i * dmin + carry + s);
            if (h.b) carry += readlane_u64(s, 63);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (int64_t)((uint64_t)h.base + u[k]);
    }
    return h.ok;
}

// An empty use of R's packed words: their loads must be complete here.
__device__ __forceinline__ void dense_ready(const RawDense& R) {
#pragma unroll
    for (int k = 0; k < 4; ++k) asm volatile("" ::"v"(R.raw[k]));
}

__device__ __forceinline__ bool decode_dense(CC& c, int m, int lane, int64_t v[4]) {
    RawDense R;
    issue_dense(c, m, lane, R);
    return finish_dense(c, R, lane, v);
}

// Value of row i of mini block m (random access).  DELTA sums the packed
// differences up to i.
__device__ __forceinline__ int64_t decode_at(CC& c, int m, int i, bool& ok) {
    MbHdr h = mb_hdr(c, m);
    ok = ok && h.ok;
    if (c.enc == ENC_DELTA) {
        uint64_t s = 0;
        if (h.b)
            for (int j = 1; j <= i; ++j) s += bits_at(h.w, (uint32_t)j * (uint32_t)h.b, h.b);
        return (int64_t)((uint64_t)h.base + (uint64_t)i * (uint64_t)ro(c.dmin)[m] + s);
    }
    uint64_t u = h.b ? bits_at(h.w, (uint32_t)i * (uint32_t)h.b, h.b) : 0;
    return (int64_t)((uint64_t)h.base + u);
}

// DICT code -> value (bounds-checked).
__device__ __forceinline__ int64_t dict_value(CC& c, int64_t code, bool& ok) {
    if (code < 0 || code >= c.ndict) { ok = false; return 0; }
    return ro(c.dict)[code];
}

// ---------------------------------------------------------------------------
// Zone test from the mini-block header alone.  A FOR mini block holds values
// in [base, base + 2^b - 1]; a DELTA one, anchor + i * dmin + (a sum of i
// packed differences in [0, 2^b - 1]) for i < 256.  When that interval lies
// inside a range atom every row passes, when it misses the atom none does,
// and the column need not be decoded (the paper's zone maps, Section 3.4,
// at mini-block granularity and with no bytes beyond the header).
// Returns 1: all rows pass, 0: none, -1: undecided.  Wave-uniform (scalar).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int zone_test(CC& c, CP& p, int m) {
    if (p.kind != PK_RANGE && p.kind != PK_NE) return -1;
    const MbHdr h = mb_hdr(c, m);
    // int64 is exact here: |base| < 2^61, width <= 32, |dmin| < 2^31, so the
    // interval ends stay below 2^62 in magnitude.  Otherwise: undecided.
    const int64_t kLim = int64_t(1) << 61;
    if (!h.ok || h.b > 32 || h.base >= kLim || h.base <= -kLim) return -1;
    const int64_t span = h.b ? (int64_t)((uint64_t(1) << h.b) - 1) : 0;
    int64_t lo = h.base, hi = h.base;
    if (c.enc == ENC_DELTA) {
        const int64_t dmin = ro(c.dmin)[m];
        if (dmin >= (int64_t(1) << 31) || dmin <= -(int64_t(1) << 31)) return -1;
        const int64_t d = dmin * (kMB - 1);
        if (d < 0) lo += d; else hi += d;
        hi += span * (kMB - 1);
    } else {
        hi += span;
    }
    if (p.kind == PK_RANGE) {
        if (lo >= p.lo && hi <= p.hi) return 1;
        if (hi < p.lo || lo > p.hi) return 0;
        return -1;
    }
    if (hi < p.lo || lo > p.lo) return 1;  // NE: the excluded value is outside
    if (lo == hi) return 0;                // every row equals it
    return -1;
}

// ---------------------------------------------------------------------------
// Integer predicates on four dense values -> 4-bit mask
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t eval_int_pred(CP& p, cptr<int64_t> in_vals,
                                                  const int64_t v[4]) {
    uint32_t mk = 0;
    const int kind = p.kind;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool t;
        if (kind == PK_RANGE) {
            t = v[k] >= p.lo && v[k] <= p.hi;
        } else if (kind == PK_NE) {
            t = v[k] != p.lo;
        } else if (kind == PK_INMASK) {
            t = v[k] >= 0 && v[k] < 64 && ((p.mask >> (uint64_t)v[k]) & 1u);
        } else if (kind == PK_INLIST) {
            t = false;
            for (int j = 0; j < p.n_in; ++j) t |= v[k] == in_vals[p.in_off + j];
        } else {
            t = false;
        }
        mk |= (uint32_t)t << k;
    }
    return mk;
}

// ---------------------------------------------------------------------------
// String predicate "s1 then s2" (LIKE '%s1%s2%', paper Section 4.1) over one
// mini block, byte-parallel.
//
// The mini block's heap is read into registers in 2 KB segments of 16-byte
// loads, two segments in turn (the next one loads while the current one is
// compared): each lane holds four consecutive words, and the two words after
// them come from the next lane by a DPP lane shift.  At every byte position
// the 4-byte window is compared with the first 4 bytes of s1 and of s2
// (three byte-aligns and eight compares per word; the hit masks combine in
// scalar registers), so a chance match costs nothing until a whole 4-byte
// prefix agrees.  A word with such a hit is queued in LDS with its two
// successors; after the last segment the queued words are checked together,
// one per lane, against 8-byte windows (the rest of a longer pattern from
// memory), mapped to their row by binary search over the row offsets (LDS),
// and kept as the row's leftmost s1 start and rightmost s2 start.  A row
// contains s1 then s2 iff some s2 start b and s1 start a satisfy b >= a +
// |s1|, that is iff rightmost s2 >= leftmost s1 + |s1|.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int row_of(const uint32_t* offs, uint32_t p) {
    int lo = 0, hi = 255;  // largest r with offs[r] <= p
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class S, class Wp>
__device__ __forceinline__ bool bytes_eq(S s, Wp w, int from, int n) {
    for (int i = from; i < n; ++i)
        if (s[i] != w[i]) return false;
    return true;
}

struct StrPattern {
    uint64_t p8, m8;  // first min(n, 8) bytes, little endian, and their mask
};

__device__ __forceinline__ StrPattern make_pattern(cptr<uint8_t> w, int n) {
    StrPattern P;
    P.p8 = *(cptr<uint64_t>)w;  // bytes past n are zero
    P.m8 = n >= 8 ? ~uint64_t(0) : ((uint64_t(1) << (8 * n)) - 1);
    P.p8 &= P.m8;
    return P;
}

struct StrLds {
    const uint32_t* tab;  // [32] the workgroup's copy of DevPred::tab (kStrTable)
    uint32_t* offs;    // [257] row start offsets within the mini block's heap
    uint32_t* first1;  // [256] leftmost s1 start (0xffffffff: none)
    uint32_t* last2;   // [256] rightmost s2 start + 1 (0: none)
    uint4* recs;       // [kRecCap] words with a prefix hit: {byte offset, word, next, the one after}
};

// Records an s1 and/or s2 start at heap position pos of the mini block: the
// row comes from a binary search over the row offsets; a word longer than 8
// bytes is checked in full where it rests.
__device__ __forceinline__ void note_start(const StrLds& L, uint32_t pos, bool m1, bool m2, CP& p,
                                           cptr<uint8_t> hs) {
    const int r = row_of(L.offs, pos);
    const uint32_t rend = L.offs[r + 1];
    if (m1 && pos + (uint32_t)p.n1 <= rend && (p.n1 <= 8 || bytes_eq(hs + pos, p.s1, 8, p.n1)))
        atomicMin(&L.first1[r], pos);
    if (m2 && pos + (uint32_t)p.n2 <= rend && (p.n2 <= 8 || bytes_eq(hs + pos, p.s2, 8, p.n2)))
        atomicMax(&L.last2[r], pos + 1);
}

// Tests 4 byte positions with 8-byte windows: q is the byte offset of word
// e0 from the 16-byte-aligned start, e1/e2 the two words after it, and the
// positions are q + kFirst .. q + kFirst + 3.
template <int kFirst>
__device__ __forceinline__ void check_word(const StrLds& L, uint32_t q, uint32_t e0, uint32_t e1, uint32_t e2,
                                           uint32_t s0, uint32_t total, const StrPattern& P1, const StrPattern& P2,
                                           CP& p, cptr<uint8_t> hs) {
    uint32_t k1 = 0, k2 = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int sh = kFirst + t;  // 0..4
        const uint32_t lo = sh == 0 ? e0 : sh == 4 ? e1 : __builtin_amdgcn_alignbit(e1, e0, 8 * (sh & 3));
        const uint32_t hi = sh == 0 ? e1 : sh == 4 ? e2 : __builtin_amdgcn_alignbit(e2, e1, 8 * (sh & 3));
        const uint64_t win8 = (uint64_t)lo | ((uint64_t)hi << 32);
        const uint32_t qt = q + (uint32_t)sh;
        const bool inr = qt >= s0 && qt - s0 < total;
        k1 |= (uint32_t)(inr && (win8 & P1.m8) == P1.p8) << t;
        k2 |= (uint32_t)(inr && (win8 & P2.m8) == P2.p8) << t;
    }
    for (uint32_t k = k1 | k2; k; k &= k - 1) {
        const int t = __builtin_ctz(k);
        note_start(L, q + (uint32_t)(kFirst + t) - s0, (k1 >> t) & 1u, (k2 >> t) & 1u, p, hs);
    }
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// One mini block's string test between issuing its loads and using them.
// One heap segment in registers: lane l holds bytes [16 (base + it * 64 + l),
// +16) in W[it]; tx, ty are the two words after the segment (for lane 63).
struct Seg {
    uint4 W[kSegIters];
    uint32_t tx, ty;
};

struct StrTile {
    Seg cur;               // the segment being compared (the first, after str_begin)
    uint64_t lraw[4];      // packed lengths of rows 4 lane .. 4 lane + 3, unshifted
    cptr<uint4> g;         // 16-byte-aligned start of the heap bytes
    const uint8_t* gp;     // the same address, generic
    uint64_t h0, h1;       // heap byte range of the mini block
    int64_t lbase;         // minimum length
    uint32_t lsh;          // bit offset of row 4 lane's length in lraw[0]
    int b;                 // length bit width
    bool ok;
};

// Buffer resource over [p, p + nbytes): raw (stride 0) 32-bit words; a load
// whose VGPR offset + immediate offset lies past nbytes returns zeros.
constexpr int kRawBufferWord3 = 0x00020000;

// Loads heap vectors base .. base + 511 of the tile (vector v = bytes
// [16 v, 16 v + 16) from the 16-byte-aligned start) into W; vectors past
// nvec read as zero through the buffer range check.  The per-lane offset is
// the only VGPR address; the slots differ by immediate offsets.
__device__ __forceinline__ void load_segment(Seg& G, const StrTile& S, uint32_t base, uint32_t nvec, int lane) {
    const uint32_t nbytes = (nvec + 1u - base) * 16u;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(S.gp + (uint64_t)base * 16u), 0, (int)nbytes, kRawBufferWord3);
    // The empty asm keeps the compiler from hoisting one offset register per
    // slot out of the loops: the slot offsets must stay immediates.
    int vo = lane * 16;
    asm volatile("" : "+v"(vo));
    const int vo2 = vo + 4096;
#pragma unroll
    for (int it = 0; it < kSegIters; ++it) {
        const int off = it * kWave * 16;  // below 4096: immediate on vo; else on vo2
        const u32x4 t = off < 4096 ? __builtin_amdgcn_raw_buffer_load_b128(r, vo + off, 0, 0)
                                   : __builtin_amdgcn_raw_buffer_load_b128(r, vo2 + (off - 4096), 0, 0);
        G.W[it] = make_uint4(t.x, t.y, t.z, t.w);
    }
    const uint32_t vt = base + kSegIters * kWave;  // wave-uniform: scalar load
    G.tx = G.ty = 0;
    if (vt <= nvec) {
        const u32x2 t = ((cptr<u32x2>)S.g)[2 * vt];
        G.tx = t.x;
        G.ty = t.y;
    }
}

// Issues the loads of mini block m's lengths and first heap segment.
__device__ __forceinline__ void str_begin(CC& c, int m, int lane, StrTile& S) {
    const MbHdr h = mb_hdr(c, m);
    S.h0 = ro(c.hoff)[m];
    S.h1 = ro(c.hoff)[m + 1];
    S.ok = h.ok && h.b <= 32 && S.h0 <= S.h1 && S.h1 <= c.heap_bytes && (S.h1 - S.h0) < (uint64_t(1) << 30);
    S.b = S.ok ? h.b : 0;
    S.lbase = h.base;
    const uint64_t a0 = S.h0 & ~uint64_t(15);
    S.g = (cptr<uint4>)(c.heap + a0);
    S.gp = c.heap + a0;
    const uint32_t nvec = S.ok ? (uint32_t)((S.h1 - a0 + 15u) >> 4) : 0u;
    // lengths: row 4 lane + j at bit (4 lane + j) b; one 8-byte window per row
    const uint32_t bp = 4u * (uint32_t)lane * (uint32_t)S.b;
    S.lsh = bp & 31u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t pj = bp + (uint32_t)j * (uint32_t)S.b;
        S.lraw[j] = S.b ? *(cptr<u64_a4>)(h.w + (pj >> 5)) : 0;
    }
    if (S.ok) {
        load_segment(S.cur, S, 0, nvec, lane);
    } else {
#pragma unroll
        for (int it = 0; it < kSegIters; ++it) S.cur.W[it] = make_uint4(0u, 0u, 0u, 0u);
        S.cur.tx = S.cur.ty = 0;
    }
}

// An empty use of every word of G: the loads that fill G must be complete
// here, so the compares that follow need no wait of their own.
__device__ __forceinline__ void seg_ready(const Seg& G) {
#pragma unroll
    for (int it = 0; it < kSegIters; ++it)
        asm volatile("" ::"v"(G.W[it].x), "v"(G.W[it].y), "v"(G.W[it].z), "v"(G.W[it].w));
}

// Neighbour words of lane's segment slot it: the next lane's first two words
// (for lane 63, those of the next slot's lane 0, or the words after the
// segment).
__device__ __forceinline__ void next_words(const Seg& S, int it, int lane, uint32_t& nx, uint32_t& nx2) {
    nx = dpp_u32<kDppWaveShl1>(S.W[it].x);
    nx2 = dpp_u32<kDppWaveShl1>(S.W[it].y);
    uint32_t lx = S.tx, ly = S.ty;
    if (it + 1 < kSegIters) {
        lx = __builtin_amdgcn_readlane(S.W[it + 1 < kSegIters ? it + 1 : it].x, 0);
        ly = __builtin_amdgcn_readlane(S.W[it + 1 < kSegIters ? it + 1 : it].y, 0);
    }
    if (lane == kWave - 1) { nx = lx; nx2 = ly; }
}

// Checks queued hit words, one per lane (all lanes at once: a wave pays
// for the check once per batch of hits, not once per hit).
// A record {q, e0, e1, e2} stands for the starts q + kFirst .. + 3.
template <int kFirst>
__device__ __forceinline__ void drain_records(const StrLds& L, int nrec, uint32_t s0, uint32_t total,
                                              const StrPattern& P1, const StrPattern& P2, CP& p,
                                              cptr<uint8_t> hs, int lane) {
    wave_lds_sync();
    for (int j = lane; j < nrec; j += kWave) {
        const uint4 r = L.recs[j];
        check_word<kFirst>(L, r.x, r.y, r.z, r.w, s0, total, P1, P2, p, hs);
    }
    wave_lds_sync();
}

// Scan modes of the string test:
//   kStrMasked  (a word under 4 bytes): 4-byte windows at every byte, masked;
//   kStrShifted (words of 4 bytes or more): 4-byte windows at every byte
//               (a word and its three byte-aligns);
//   kStrTable   (both words of 7 bytes or more, with a table): every
//               occurrence covers a whole 4-byte-aligned word, which then
//               equals one of the word's four 4-byte shifts; each aligned
//               word is looked up in the 32-slot LDS table of the eight
//               shifts (DevPred::tab), one read and one compare a word, and
//               the neighbour words are gathered only on a hit.
enum : int { kStrMasked = 0, kStrShifted = 1, kStrTable = 2 };

__device__ __forceinline__ int str_mode(int n1, int n2) { return (n1 < 4 || n2 < 4) ? kStrMasked : kStrShifted; }

// Returns the 4-bit match mask of the lane's rows (row 64 k + lane -> bit k)
// for the mini block whose loads str_begin issued; clears ok on corruption.
// kOffsReady: the caller has written the row offsets (L.offs[0..256]) from
// materialised string offsets, and S carries no packed lengths.
template <int kMode, bool kOffsReady = false>
__device__ __forceinline__ uint32_t str_finish(CC& c, CP& p, int lane, int nvalid, StrTile& S,
                                               const StrLds& L, bool& ok) {
    if (!S.ok) { ok = false; return 0; }
    uint32_t* const offs = L.offs;
    const uint32_t s0 = (uint32_t)(S.h0 & 15u);
    const uint32_t nvec = (uint32_t)((S.h1 - (S.h0 - s0) + 15u) >> 4);
    if (kOffsReady) {
        reinterpret_cast<uint4*>(L.first1)[lane] = make_uint4(~0u, ~0u, ~0u, ~0u);
        reinterpret_cast<uint4*>(L.last2)[lane] = make_uint4(0u, 0u, 0u, 0u);
    } else {
    // Row offsets: lane l takes rows 4l..4l+3, so one wave scan suffices.
    uint32_t len[4], lsum = 0;
    const uint64_t lmask = (uint64_t(1) << S.b) - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t sh = (S.lsh + (uint32_t)j * (uint32_t)S.b) & 31u;
        const uint32_t u = (uint32_t)((S.lraw[j] >> sh) & lmask);
        len[j] = 4 * lane + j < nvalid ? (uint32_t)S.lbase + u : 0u;
        lsum += len[j];
    }
    const uint32_t incl = wave_incl_scan_u32(lsum);
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    {
        uint32_t o = incl - lsum;
        uint4 ov;
        ov.x = o;
        ov.y = o + len[0];
        ov.z = ov.y + len[1];
        ov.w = ov.z + len[2];
        reinterpret_cast<uint4*>(offs)[lane] = ov;
        // Materialised here (the empty asm keeps the compiler from hoisting
        // the constant registers out of the tile loop, where they spilled).
        uint32_t ones = ~0u, zero = 0u;
        asm volatile("" : "+v"(ones), "+v"(zero));
        reinterpret_cast<uint4*>(L.first1)[lane] = make_uint4(ones, ones, ones, ones);
        reinterpret_cast<uint4*>(L.last2)[lane] = make_uint4(zero, zero, zero, zero);
    }
    if (lane == 0) offs[256] = total;
    if ((uint64_t)total != S.h1 - S.h0) { ok = false; return 0; }
    }

    const StrPattern P1 = make_pattern(p.s1, p.n1), P2 = make_pattern(p.s2, p.n2);
    // The first 4 bytes of each word (masked for kStrMasked).
    const uint32_t k1 = (uint32_t)P1.m8, k2 = (uint32_t)P2.m8;
    const uint32_t q1 = (uint32_t)P1.p8, q2 = (uint32_t)P2.p8;
    cptr<uint8_t> hs = ro(c.heap + S.h0);
    const uint32_t total_b = (uint32_t)(S.h1 - S.h0);
    int nrec = 0;
    // Window modes: does a word's 4-byte prefix start in x (x1: the word
    // after it), at x or one of its three byte-aligns?
    auto word_hit = [&](uint32_t x, uint32_t x1) -> bool {
        const uint32_t w1 = __builtin_amdgcn_alignbit(x1, x, 8);
        const uint32_t w2 = __builtin_amdgcn_alignbit(x1, x, 16);
        const uint32_t w3 = __builtin_amdgcn_alignbit(x1, x, 24);
        if (kMode == kStrMasked)
            return ((x & k1) == q1) | ((w1 & k1) == q1) | ((w2 & k1) == q1) | ((w3 & k1) == q1) |
                   ((x & k2) == q2) | ((w1 & k2) == q2) | ((w2 & k2) == q2) | ((w3 & k2) == q2);
        return (x == q1) | (w1 == q1) | (w2 == q1) | (w3 == q1) | (x == q2) | (w1 == q2) | (w2 == q2) | (w3 == q2);
    };
    // A record {q, x, y, z} holds the 12 bytes from offset q and stands for
    // 4 starts: q .. q + 3 in the window modes; q + 1 .. q + 4 for kStrTable,
    // whose hit on the aligned word y means a start in the 3 bytes before y
    // or at y itself.
    constexpr int kFirst = kMode == kStrTable ? 1 : 0;
    auto push = [&](bool cnd, uint32_t q, uint32_t x, uint32_t y, uint32_t z) {
        const uint64_t hb = __builtin_amdgcn_ballot_w64(cnd);
        if (hb) {
            const int nh = (int)__popcll(hb);
            if (nrec + nh > kRecCap) {
                drain_records<kFirst>(L, nrec, s0, total_b, P1, P2, p, hs, lane);
                nrec = 0;
            }
            if (cnd) L.recs[nrec + bits_below(hb)] = make_uint4(q, x, y, z);
            nrec += nh;
        }
    };
    uint32_t tail = 0;  // last word of the previous segment (lane 63's fourth)
    // Hot loop over one segment.  A word with a prefix hit queues its record
    // in LDS (a rare, wave-uniform branch); kStrTable gathers the
    // neighbouring words only then.
    const uint32_t rot = p.tab_rot;
    auto scan = [&](const Seg& G, uint32_t base) {
#pragma unroll
        for (int it = 0; it < kSegIters; ++it) {
            if (base + (uint32_t)it * kWave > nvec) break;  // slots past the mini block hold zeros
            const uint4 w = G.W[it];
            const uint32_t q0 = (base + (uint32_t)it * kWave + (uint32_t)lane) * 16u;
            uint32_t nx = 0, nx2 = 0;
            if (kMode != kStrTable) next_words(G, it, lane, nx, nx2);
            const uint32_t e[6] = {w.x, w.y, w.z, w.w, nx, nx2};
            if (kMode != kStrTable) {
#pragma unroll
                for (int wd = 0; wd < 4; ++wd) {
                    const bool h = word_hit(e[wd], e[wd + 1]);
                    if (__builtin_amdgcn_ballot_w64(h)) push(h, q0 + 4u * (uint32_t)wd, e[wd], e[wd + 1], e[wd + 2]);
                }
                continue;
            }
            // kStrTable: the four table reads first, so that they wait together.
            uint32_t t[4];
#pragma unroll
            for (int wd = 0; wd < 4; ++wd) {
                const uint32_t y = e[wd] ^ __builtin_amdgcn_alignbit(e[wd], e[wd], rot);
                t[wd] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(L.tab) + (y & 0x7Cu));
            }
            // one wave vote for the four words: hits are rare
            if (!__builtin_amdgcn_ballot_w64((t[0] == e[0]) | (t[1] == e[1]) | (t[2] == e[2]) | (t[3] == e[3])))
                continue;
#pragma unroll
            for (int wd = 0; wd < 4; ++wd) {
                const bool h = t[wd] == e[wd];
                if (!__builtin_amdgcn_ballot_w64(h)) continue;
                // The word before: the previous lane's last (lane 0: the
                // previous slot's lane 63, or the segment before's); the word
                // after: the next lane's first for the lane's last word.
                uint32_t xp, y1;
                if (wd) {
                    xp = e[wd - 1];
                } else {
                    const uint32_t prev = it ? __builtin_amdgcn_readlane(G.W[it ? it - 1 : 0].w, 63) : tail;
                    xp = (uint32_t)__builtin_amdgcn_update_dpp((int)prev, (int)w.w, kDppWaveShr1, 0xf, 0xf, false);
                }
                if (wd < 3) {
                    y1 = e[wd + 1];
                } else {
                    uint32_t b;
                    next_words(G, it, lane, y1, b);
                }
                push(h, q0 + 4u * (uint32_t)wd - 4u, xp, e[wd], y1);
            }
        }
        if (kMode == kStrTable) tail = __builtin_amdgcn_readlane(G.W[kSegIters - 1].w, 63);
    };
    // Two segment buffers in turn: the next segment's loads are in flight
    // while the current one is compared.  seg_ready makes the wait for the
    // current buffer explicit before the next loads are issued: left to the
    // compiler, the join after a conditional load merges the two paths'
    // outstanding-load counts, and the wait before the compares would then
    // also cover the loads just issued.
    constexpr uint32_t kSeg = kSegIters * kWave;
    Seg other;
    for (uint32_t base = 0;; base += 2 * kSeg) {
        const bool more1 = base + kSeg < nvec;
        seg_ready(S.cur);
        if (more1) load_segment(other, S, base + kSeg, nvec, lane);
        scan(S.cur, base);
        if (!more1) break;
        const bool more2 = base + 2 * kSeg < nvec;
        seg_ready(other);
        if (more2) load_segment(S.cur, S, base + 2 * kSeg, nvec, lane);
        scan(other, base + kSeg);
        if (!more2) break;
    }
    if (nrec) drain_records<kFirst>(L, nrec, s0, total_b, P1, P2, p, hs, lane);
    wave_lds_sync();
    uint32_t res = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int i = 64 * k + lane;
        uint32_t f = L.first1[i], e = L.last2[i];
        bool hit = i < nvalid && f != 0xFFFFFFFFu && e != 0u && (uint64_t)(e - 1) >= (uint64_t)f + p.n1;
        res |= (uint32_t)hit << k;
    }
    return res;
}

template <int kMode>
__device__ __forceinline__ uint32_t str_pred(CC& c, CP& p, int m, int lane, int nvalid, const StrLds& L,
                                             bool& ok) {
    StrTile S;
    str_begin(c, m, lane, S);
    return str_finish<kMode>(c, p, lane, nvalid, S, L, ok);
}

// ---------------------------------------------------------------------------
// FSST strings (Sections 3.4.2 and 4.1): each chunk carries a table of up to
// 255 symbols of 1..8 bytes; a record is a run of one-byte codes, code 255
// escaping the literal byte after it.  The string test never writes a
// decoded byte: LIKE '%s1%s2%' is a byte automaton D with S = |s1| + |s2|
// + 1 states (the two words' Knuth-Morris-Pratt automata in sequence, built
// with the plan), and the workgroup lifts it to the chunk's codes,
//     T[q][c] = the state D reaches from q over the bytes of symbol c,
// so that a lane steps one code per LDS byte read.  The escape joins the
// same table: T[q][255] = S + q, whose row is D itself (the literal byte's
// step), and codes the chunk does not define lead to a sink row 2S.  T has
// 2S + 1 rows of 256 bytes (DevQuery::fs_lds_off); rows S .. 2S are loaded
// with the plan, rows 0 .. S-1 for every chunk.
// ---------------------------------------------------------------------------

// Rows S .. 2S of the plan's code table: the byte automaton and the sink.
__device__ void fsst_load_dfa(CQ& Q, uint8_t* smem_shared) {
    if (Q.fs_pred < 0) return;
    const uint32_t S = (uint32_t)Q.fs_states;
    uint8_t* T = smem_shared + Q.fs_lds_off;
    cptr<uint4> src = (cptr<uint4>)Q.fs_dfa;
    uint4* dst = reinterpret_cast<uint4*>(T + S * 256);
    for (uint32_t e = threadIdx.x; e < S * 16; e += blockDim.x) dst[e] = ld4(src, e);
    for (uint32_t e = threadIdx.x; e < 256; e += blockDim.x) T[2 * S * 256 + e] = (uint8_t)(2 * S);
}

// Rows 0 .. S-1 of the code table for chunk k (rows S .. 2S in place).
__device__ void fsst_load_chunk(CQ& Q, uint8_t* smem_shared, int k) {
    CP& P = Q.preds[Q.fs_pred];
    CC& c = Q.cols[P.col];
    const uint32_t S = (uint32_t)Q.fs_states;
    uint8_t* T = smem_shared + Q.fs_lds_off;
    const uint8_t* D = T + S * 256;
    cptr<uint8_t> tab = ro(c.symtab) + (size_t)k * (256 * 8 + 256);
    for (uint32_t code = threadIdx.x; code < 256; code += blockDim.x) {
        const uint64_t sv = ((cptr<uint64_t>)tab)[code];
        const uint32_t L = code < 255 ? (uint32_t)tab[256 * 8 + code] : 0u;
        for (uint32_t q = 0; q < S; ++q) {
            uint32_t st;
            if (code == 255) {
                st = S + q;
            } else if (L == 0 || L > 8) {
                st = 2 * S;
            } else {
                st = q;
                for (uint32_t b = 0; b < L; ++b) st = D[st * 256 + (uint32_t)((sv >> (8 * b)) & 0xFF)];
            }
            T[q * 256 + code] = (uint8_t)st;
        }
    }
}

// A lane's run of codes through a 48-byte register window x:y:z of the
// heap (x at byte offset A from base, 16-byte aligned, A <= pos < A + 16):
// a peek reads x and y only, so the load that refills z has the 16 bytes of
// y to work through before it is waited for.  Offsets are 32-bit, relative
// to the 16-byte-aligned start of the mini block's codes; the heap is
// padded, so the window's loads stay inside it while pos is at most the
// mini block's end.
struct CodeReader {
    cptr<uint4> base;
    uint32_t pos, A;
    uint4 x, y, z;
    __device__ __forceinline__ void init(const uint8_t* heap, uint64_t h0, uint32_t p) {
        const uint64_t a0 = h0 & ~uint64_t(15);
        base = (cptr<uint4>)(heap + a0);
        pos = (uint32_t)(h0 - a0) + p;
        A = pos & ~15u;
        x = ld4(base, A >> 4);
        y = ld4(base, (A >> 4) + 1u);
        z = ld4(base, (A >> 4) + 2u);
    }
    // the next 4 code bytes, first in the low byte
    // (two-way selects: a four-way pick by o >> 2 compiles to a stack copy
    // of the window and an indexed load)
    __device__ __forceinline__ uint32_t peek4() const {
        const uint32_t o = pos - A;
        const bool half = (o & 8u) != 0;
        const uint32_t a0 = half ? x.z : x.x, a1 = half ? x.w : x.y, b0 = half ? y.x : x.z;
        const uint32_t lo = __builtin_amdgcn_alignbyte(a1, a0, o & 3u);
        const uint32_t hi = __builtin_amdgcn_alignbyte(b0, a1, o & 3u);
        return (o & 4u) ? hi : lo;
    }
    // the next 16 code bytes, four per word (a: the first four)
    __device__ __forceinline__ void peek16(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) const {
        const uint32_t o = pos - A;
        const bool half = (o & 8u) != 0, q = (o & 4u) != 0;
        const uint32_t B0 = half ? x.z : x.x, B1 = half ? x.w : x.y, B2 = half ? y.x : x.z, B3 = half ? y.y : x.w;
        const uint32_t B4 = half ? y.z : y.x, B5 = half ? y.w : y.y;
        const uint32_t c0 = q ? B1 : B0, c1 = q ? B2 : B1, c2 = q ? B3 : B2, c3 = q ? B4 : B3, c4 = q ? B5 : B4;
        a = __builtin_amdgcn_alignbyte(c1, c0, o & 3u);
        b = __builtin_amdgcn_alignbyte(c2, c1, o & 3u);
        c = __builtin_amdgcn_alignbyte(c3, c2, o & 3u);
        d = __builtin_amdgcn_alignbyte(c4, c3, o & 3u);
    }
    // the next 8 code bytes (a: the first four)
    __device__ __forceinline__ void peek8(uint32_t& a, uint32_t& b) const {
        const uint32_t o = pos - A;
        const bool half = (o & 8u) != 0, q = (o & 4u) != 0;
        const uint32_t B0 = half ? x.z : x.x, B1 = half ? x.w : x.y, B2 = half ? y.x : x.z, B3 = half ? y.y : x.w;
        const uint32_t c0 = q ? B1 : B0, c1 = q ? B2 : B1, c2 = q ? B3 : B2;
        a = __builtin_amdgcn_alignbyte(c1, c0, o & 3u);
        b = __builtin_amdgcn_alignbyte(c2, c1, o & 3u);
    }
    __device__ __forceinline__ void advance(uint32_t n) {
        pos += n;
        if (pos - A < 16) return;
        if (pos - A < 32) {
            x = y;
            y = z;
            A += 16;
            z = ld4(base, (A >> 4) + 2u);
        } else {
            A = pos & ~15u;
            x = ld4(base, A >> 4);
            y = ld4(base, (A >> 4) + 1u);
            z = ld4(base, (A >> 4) + 2u);
        }
    }
};

// Code lengths of rows 4 lane .. 4 lane + 3 of FSST mini block m (rows from
// nvalid on: 0) and the mini block's code range; false on a corrupt header.
__device__ __forceinline__ bool fsst_lengths(CC& c, int m, int lane, int nvalid, uint32_t rl[4], uint32_t& lsum,
                                             uint32_t& incl, uint64_t& h0) {
    const MbHdr h = mb_hdr(c, m);
    h0 = ro(c.hoff)[m];
    const uint64_t h1 = ro(c.hoff)[m + 1];
    if (!(h.ok && h.b <= 32 && h0 <= h1 && h1 <= c.heap_bytes && (h1 - h0) < (uint64_t(1) << 30))) return false;
    lsum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = 4 * lane + j;
        rl[j] = r < nvalid ? (uint32_t)h.base + (uint32_t)(h.b ? bits_at(h.w, (uint32_t)r * (uint32_t)h.b, h.b) : 0) : 0u;
        lsum += rl[j];
    }
    incl = wave_incl_scan_u32(lsum);
    return (uint64_t)__builtin_amdgcn_readlane(incl, 63) == h1 - h0;
}

// The string atom on FSST mini block m: returns the mask of rows that
// contain s1 and, after its leftmost end, s2 (row 64 k + lane -> bit k).
// Lane l takes rows 4 l .. 4 l + 3, whose codes are contiguous in the heap,
// sixteen codes per step.  fl: 256 bytes of the wave's LDS for the
// transposition.
__device__ __forceinline__ uint32_t fsst_pred(CQ& Q, CC& c, int m, int lane, int nvalid, uint8_t* fl,
                                              const uint8_t* smem_shared, bool& ok) {
    // The table is the first thing in the shared area (fs_lds_off == 0), so
    // its address is a constant and a step's LDS address is one byte
    // permute: {code, state, 0, 0}.
    const uint8_t* T = smem_shared;
    const uint32_t S = (uint32_t)Q.fs_states, acc = S - 1;
    uint32_t rl[4], lsum, incl;
    uint64_t h0;
    if (!fsst_lengths(c, m, lane, nvalid, rl, lsum, incl, h0)) { ok = false; return 0; }
    CodeReader R;
    R.init(c.heap, h0, incl - lsum);
    uint32_t res = 0;
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        // (a select, not rl[r]: a dynamic index would put rl in scratch)
        uint32_t rem = r == 0 ? rl[0] : r == 1 ? rl[1] : r == 2 ? rl[2] : rl[3];
        uint32_t st = 0;
        while (rem) {
            // sixteen codes a step (most records take one or two): the
            // states after 1 .. 16 codes, then the one after nq of them
            uint32_t qa, qb, qc, qd;
            R.peek16(qa, qb, qc, qd);
            const uint32_t nq = min(rem, 16u);
            auto step = [&](uint32_t s, uint32_t w, uint32_t sel) -> uint32_t {
                return T[__builtin_amdgcn_perm(s, w, sel)];
            };
            const uint32_t x0 = step(st, qa, 0x0c0c0400u), x1 = step(x0, qa, 0x0c0c0401u);
            const uint32_t x2 = step(x1, qa, 0x0c0c0402u), x3 = step(x2, qa, 0x0c0c0403u);
            const uint32_t x4 = step(x3, qb, 0x0c0c0400u), x5 = step(x4, qb, 0x0c0c0401u);
            const uint32_t x6 = step(x5, qb, 0x0c0c0402u), x7 = step(x6, qb, 0x0c0c0403u);
            const uint32_t x8 = step(x7, qc, 0x0c0c0400u), x9 = step(x8, qc, 0x0c0c0401u);
            const uint32_t x10 = step(x9, qc, 0x0c0c0402u), x11 = step(x10, qc, 0x0c0c0403u);
            const uint32_t x12 = step(x11, qd, 0x0c0c0400u), x13 = step(x12, qd, 0x0c0c0401u);
            const uint32_t x14 = step(x13, qd, 0x0c0c0402u);
            uint32_t x15 = step(x14, qd, 0x0c0c0403u);
            // (an empty use keeps the last reads unconditional: the compiler
            // otherwise branches on nq around them)
            asm volatile("" : "+v"(x15));
            {
                // a select tree on the bits of nq - 1
                const uint32_t i = nq - 1u;
                const bool b0 = (i & 1u) != 0, b1 = (i & 2u) != 0, b2 = (i & 4u) != 0, b3 = (i & 8u) != 0;
                const uint32_t t0 = b0 ? x1 : x0, t1 = b0 ? x3 : x2, t2 = b0 ? x5 : x4, t3 = b0 ? x7 : x6;
                const uint32_t t4 = b0 ? x9 : x8, t5 = b0 ? x11 : x10, t6 = b0 ? x13 : x12, t7 = b0 ? x15 : x14;
                const uint32_t u0 = b1 ? t1 : t0, u1 = b1 ? t3 : t2, u2 = b1 ? t5 : t4, u3 = b1 ? t7 : t6;
                const uint32_t v0 = b2 ? u1 : u0, v1 = b2 ? u3 : u2;
                st = b3 ? v1 : v0;
            }
            // matched: the rest of the record is skipped
            const uint32_t adv = st == acc ? rem : nq;
            rem -= adv;
            R.advance(adv);
        }
        if (st >= S) ok = false;  // an escape without its byte, or a code the table does not define
        res |= (uint32_t)(st == acc) << r;
    }
    // rows 4 lane + j -> rows 64 k + lane, through LDS
    reinterpret_cast<uint32_t*>(fl)[lane] =
        (res & 1u) | ((res >> 1) & 1u) << 8 | ((res >> 2) & 1u) << 16 | ((res >> 3) & 1u) << 24;
    wave_lds_sync();
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(fl[64 * k + lane] != 0) << k;
    wave_lds_sync();
    return mask;
}

// ---------------------------------------------------------------------------
// Value slots carried by a surviving row.  Fact-column loads occupy slots
// 0..nloads-1, probe payloads the slots after them.  In the fused kernel the
// slots live in the wave's LDS area (one int64 column per lane, so runtime
// slot ids cost nothing); the fragmented kernels keep them in registers.
// ---------------------------------------------------------------------------
struct LdsSlots {
    int64_t* p;  // this lane's slot 0; slot s at p[s * kWave]
    __device__ __forceinline__ void set(int id, int64_t x) const { p[id * kWave] = x; }
    __device__ __forceinline__ int64_t get(int id) const { return p[id * kWave]; }
};

struct RegSlots {
    int64_t v[kMaxSlots];
    __device__ __forceinline__ void set(int id, int64_t x) {
#pragma unroll
        for (int i = 0; i < kMaxSlots; ++i)
            if (i == id) v[i] = x;
    }
    __device__ __forceinline__ int64_t get(int id) const {
        int64_t x = 0;
#pragma unroll
        for (int i = 0; i < kMaxSlots; ++i)
            if (i == id) x = v[i];
        return x;
    }
};

__device__ __forceinline__ uint32_t hash32(int32_t key, int log2cap) {
    return log2cap ? ((uint32_t)key * 0x9E3779B1u) >> (32 - log2cap) : 0u;
}

// Linear-probing lookup; returns the slot or -1.
template <bool kLds>
__device__ __forceinline__ int hash_find(CH& h, const uint8_t* smem_shared, int64_t key) {
    if (key < INT32_MIN || key > INT32_MAX || key == kEmptyKey) return -1;
    const int32_t k = (int32_t)key;
    const int32_t* lkeys = reinterpret_cast<const int32_t*>(smem_shared + h.lds_off);
    cptr<int32_t> gkeys = ro(h.keys);
    uint32_t s = hash32(k, h.log2cap);
    for (uint32_t n = 0; n <= h.cap_mask; ++n) {
        int32_t x = kLds ? lkeys[s] : gkeys[s];
        if (x == k) return (int)s;
        if (x == kEmptyKey) return -1;
        s = (s + 1) & h.cap_mask;
    }
    return -1;
}

// LDS filter test: false means the key is certainly absent.
__device__ __forceinline__ bool filter_maybe(CH& h, const uint8_t* smem_shared, int64_t key) {
    if (h.filt_lds_off < 0) return true;
    const uint32_t b = filter_bit((int32_t)key, h.flog2), b2 = filter_bit2((int32_t)key, h.flog2);
    const uint32_t* f = reinterpret_cast<const uint32_t*>(smem_shared + h.filt_lds_off);
    const uint32_t w = f[b >> 5];  // b2 lies in the same word
    return ((w >> (b & 31)) & (w >> (b2 & 31)) & 1u) != 0;
}

// Key-range bitmap test (the table has one: h.bits != nullptr).
__device__ __forceinline__ bool bitmap_has(CH& h, const uint8_t* smem_shared, int64_t key) {
    const uint64_t d = (uint64_t)key - (uint64_t)h.bmin;
    if (d >= h.bspan) return false;
    const uint32_t w = h.bits_lds_off >= 0
                           ? reinterpret_cast<const uint32_t*>(smem_shared + h.bits_lds_off)[d >> 5]
                           : ro(h.bits)[d >> 5];
    return (w >> (d & 31)) & 1u;
}

// The same test on the bitmap in device memory (kernels without the fused
// kernel's LDS copies).
__device__ __forceinline__ bool bitmap_has_global(CH& h, int64_t key) {
    const uint64_t d = (uint64_t)key - (uint64_t)h.bmin;
    return d < h.bspan && ((ro(h.bits)[d >> 5] >> (d & 31)) & 1u);
}

// Membership of the lane's four keys (mask bit k: row 64 k + lane is live):
// four independent bit tests when the table has a bitmap, else the hash
// chains probed in lockstep so that their loads are in flight together.
template <bool kLds>
__device__ __forceinline__ uint32_t hash_member4(CH& h, const uint8_t* smem_shared, const int64_t key[4],
                                                 uint32_t live) {
    if (h.filt_lds_off >= 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (key[k] < INT32_MIN || key[k] > INT32_MAX || !filter_maybe(h, smem_shared, key[k])) live &= ~(1u << k);
        if (__ballot(live != 0) == 0) return 0;
    }
    if (h.bits) {
        uint32_t found = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            found |= (uint32_t)(((live >> k) & 1u) && bitmap_has(h, smem_shared, key[k])) << k;
        return found;
    }
    const int32_t* lkeys = reinterpret_cast<const int32_t*>(smem_shared + h.lds_off);
    cptr<int32_t> gkeys = ro(h.keys);
    uint32_t slot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (key[k] < INT32_MIN || key[k] > INT32_MAX || key[k] == kEmptyKey) live &= ~(1u << k);
        slot[k] = hash32((int32_t)key[k], h.log2cap);
    }
    uint32_t found = 0;
    for (uint32_t n = 0; n <= h.cap_mask && __ballot(live != 0); ++n) {
        int32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = (live >> k) & 1u ? (kLds ? lkeys[slot[k]] : gkeys[slot[k]]) : kEmptyKey;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((live >> k) & 1u)) continue;
            if (x[k] == (int32_t)key[k]) {
                found |= 1u << k;
                live &= ~(1u << k);
            } else if (x[k] == kEmptyKey) {
                live &= ~(1u << k);
            } else {
                slot[k] = (slot[k] + 1) & h.cap_mask;
            }
        }
    }
    return found;
}

template <bool kLds>
__device__ __forceinline__ int64_t hash_payload(CH& h, const uint8_t* smem_shared, int k,
                                                int slot) {
    if (kLds) {
        // payload arrays follow the keys at the same relative offsets
        const uint8_t* base = smem_shared + h.lds_off + ((const uint8_t*)h.pay[k] - (const uint8_t*)h.keys);
        return h.pay64[k] ? reinterpret_cast<const int64_t*>(base)[slot]
                          : (int64_t)reinterpret_cast<const int32_t*>(base)[slot];
    }
    cptr<uint8_t> base = ro((const uint8_t*)h.pay[k]);
    return h.pay64[k] ? ((cptr<int64_t>)base)[slot] : (int64_t)((cptr<int32_t>)base)[slot];
}

// ---------------------------------------------------------------------------
// Aggregation of one surviving row into the (LDS or global) group table
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ bool group_index(CQ& Q, const S& sv, int64_t& g) {
    g = 0;
    for (int k = 0; k < Q.nkeys; ++k) {
        CK& K = Q.keys[k];
        int64_t d = sv.get(K.slot) - K.min;
        if (d < 0 || d >= K.card) return false;
        g += d * K.stride;
    }
    return true;
}

template <class S>
__device__ __forceinline__ int64_t acc_value(CA& A, const S& sv) {
    int64_t prod = 1;
    for (int t = 0; t < A.nterms; ++t) {
        CT& T = A.t[t];
        int64_t x = T.slot >= 0 ? T.mul * sv.get(T.slot) + T.add : T.add;
        prod *= x;
    }
    return prod;
}

// Row of group g in the group table T: g itself (direct table), or the
// slot that g holds in the hash table, claimed with a compare-and-swap on
// the first free slot of its linear probe sequence (-1: no slot free, which
// the table's size rules out).
__device__ __forceinline__ int64_t agg_row(CQ& Q, unsigned long long* T, int64_t g) {
    if (!Q.agg_hash) return g;
    const uint64_t n = (uint64_t)Q.ngroups, mask = n - 1;
    unsigned long long* K = T + n * (uint64_t)Q.nacc;
    const unsigned long long key = (unsigned long long)g + 1ull;
    uint64_t h = ((uint64_t)key * 0x9E3779B97F4A7C15ull) >> 17;
    for (uint64_t t = 0; t < n; ++t) {
        h &= mask;
        unsigned long long k = __hip_atomic_load(&K[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == 0ull) k = atomicCAS(&K[h], 0ull, key);
        if (k == 0ull || k == key) return (int64_t)h;
        ++h;
    }
    return -1;
}

// false: the hash group table had no free slot.  kHash: the batch has a
// plan with a hash group table (only those instantiations carry its code).
template <bool kHash, class S>
__device__ __forceinline__ bool aggregate_row(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const S& sv,
                                              int64_t g) {
    const int nacc = Q.nacc;
    unsigned long long* T = Q.agg_lds
        ? reinterpret_cast<unsigned long long*>(smem_shared + Q.agg_lds_off) + g * nacc
        : gagg + g * nacc;
    if constexpr (kHash) {
        if (Q.agg_hash) {
            const int64_t r = agg_row(Q, gagg, g);
            if (r < 0) return false;
            T = gagg + r * nacc;
        }
    }
    atomicAdd(&T[0], 1ull);
    for (int a = 1; a < nacc; ++a) atomicAdd(&T[a], (unsigned long long)acc_value(Q.accs[a], sv));
    return true;
}

// ---------------------------------------------------------------------------
// Stage B: probes, value loads and aggregation of one row per lane.  m and i
// may differ between lanes (rows queued from several mini blocks).  gagg is
// the plan's group table in device memory.
// ---------------------------------------------------------------------------
template <bool kHash>
__device__ __forceinline__ void stage_b(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, LdsSlots sv, int m,
                                        int i, bool active, bool& ok_hdr) {
    bool ok = active;
    const int nprobes = Q.nprobes;
    for (int j = 0; j < nprobes; ++j) {
        if (__ballot(ok) == 0) return;
        CPR& P = Q.probes[j];
        if (ok) {
            CC& fc = Q.cols[P.fk_col];
            int64_t fk = decode_at(fc, m, i, ok_hdr);
            if (fc.enc == ENC_DICT) fk = dict_value(fc, fk, ok_hdr);
            if (fk < INT32_MIN || fk > INT32_MAX || !filter_maybe(P.h, smem_shared, fk)) {
                ok = false;  // certainly absent
                continue;
            }
            // The key-range bitmap answers membership exactly: it settles a
            // probe that needs no payload, and keeps non-members (most rows
            // of a selective join) away from the hash table's random reads.
            if (P.h.bits) {
                if (!bitmap_has(P.h, smem_shared, fk)) {
                    ok = false;
                    continue;
                }
                if (P.pay_slot[0] < 0 && P.pay_slot[1] < 0) continue;
            }
            const bool lds = P.h.lds_off >= 0;
            int slot = lds ? hash_find<true>(P.h, smem_shared, fk) : hash_find<false>(P.h, smem_shared, fk);
            ok = slot >= 0;
            if (ok) {
                for (int k = 0; k < P.h.npay; ++k) {
                    if (P.pay_slot[k] < 0) continue;
                    int64_t pv = lds ? hash_payload<true>(P.h, smem_shared, k, slot)
                                     : hash_payload<false>(P.h, smem_shared, k, slot);
                    sv.set(P.pay_slot[k], pv);
                }
            }
        }
    }
    if (!ok) return;
    // Fact values for slots 0..nloads-1, two slots at a time: the group's
    // loads go out in three rounds (mini-block headers, packed words,
    // dictionary entries), so that a flush waits for memory three times a
    // group rather than three times a slot; a DELTA column (a running sum)
    // decodes on its own.
    const int nloads = Q.nloads;
    constexpr int kGrp = 2;
#pragma unroll 1
    for (int g0 = 0; g0 < nloads; g0 += kGrp) {
        uint32_t w0[kGrp], w1[kGrp];
        int64_t base[kGrp];
#pragma unroll
        for (int k = 0; k < kGrp; ++k) {
            if (g0 + k < nloads) {
                CC& c = Q.cols[Q.loads[g0 + k].col];
                w0[k] = ro(c.woff)[m];
                w1[k] = ro(c.woff)[m + 1];
                base[k] = ro(c.base)[m];
            }
        }
        uint64_t u[kGrp];
#pragma unroll
        for (int k = 0; k < kGrp; ++k) {
            if (g0 + k < nloads) {
                CC& c = Q.cols[Q.loads[g0 + k].col];
                if (c.enc == ENC_DELTA) {
                    u[k] = (uint64_t)decode_at(c, m, i, ok_hdr);
                } else {
                    // the checks of mb_hdr: a corrupt header must not steer a load
                    const uint32_t nw = w1[k] - w0[k];
                    const bool hok = (w0[k] <= w1[k]) && (w1[k] <= c.nwords) && ((nw & 7u) == 0) && (nw <= 512u);
                    ok_hdr = ok_hdr && hok;
                    const int b = hok ? (int)(nw >> 3) : 0;
                    u[k] = (uint64_t)base[k] +
                           (b ? bits_at(ro(c.words) + (hok ? w0[k] : 0u), (uint32_t)i * (uint32_t)b, b) : 0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kGrp; ++k) {
            if (g0 + k < nloads) {
                CL& Ld = Q.loads[g0 + k];
                int64_t x = (int64_t)u[k];
                if (Ld.dict_val) x = dict_value(Q.cols[Ld.col], x, ok_hdr);
                sv.set(g0 + k, x);
            }
        }
    }
    int64_t g;
    if (!group_index(Q, sv, g)) { ok_hdr = false; return; }
    if (!aggregate_row<kHash>(Q, smem_shared, gagg, sv, g)) ok_hdr = false;
}

// ---------------------------------------------------------------------------
// One mini block of one plan, by one wave (stage A), survivors queued
// ---------------------------------------------------------------------------
struct WaveArea {
    const uint32_t* tab;  // [32] the workgroup's string-scan table
    uint32_t* pend;    // [kPendCap] queued surviving row ids
    int64_t* slots;    // [kMaxSlots][kWave] stage-B values
    uint32_t* offs;    // [260] string row offsets
    uint32_t* first1;  // [256] leftmost s1 start per row
    uint32_t* last2;   // [256] rightmost s2 start + 1 per row
    uint4* recs;       // [kRecCap] string words with a prefix hit
};

template <bool kHash>
__device__ __forceinline__ void flush_pending(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const WaveArea& W,
                                              int& npend, int lane, bool& ok_hdr) {
    wave_lds_sync();
    for (int base = 0; base < npend; base += kWave) {
        int idx = base + lane;
        bool act = idx < npend;
        uint32_t row = W.pend[act ? idx : 0];
        stage_b<kHash>(Q, smem_shared, gagg, LdsSlots{W.slots + lane}, (int)(row >> 8), (int)(row & 255u), act,
                       ok_hdr);
    }
    npend = 0;
    wave_lds_sync();
}

template <bool kHash>
__device__ __forceinline__ void queue_survivors(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const WaveArea& W,
                                                int64_t row0, uint32_t mask, int lane, int& npend, bool& ok_hdr) {
    if (__ballot(mask != 0) == 0) return;
    // Queue survivors (wave ballot + mbcnt compaction).
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool bit = (mask >> k) & 1u;
        uint64_t b = __ballot(bit);
        if (bit) W.pend[npend + bits_below(b)] = (uint32_t)(row0 + 64 * k + lane);
        npend += (int)__popcll(b);
    }
    if (npend >= kWave) flush_pending<kHash>(Q, smem_shared, gagg, W, npend, lane, ok_hdr);
}

// Stage A of mini block m: returns the mask of rows passing every atom (row
// 64 k + lane -> bit k).  kEager: the plan's one string atom comes last and
// its loads are issued before the integer atoms run, so both wait for memory
// once, together.
template <bool kEager, int kStr>
__device__ __forceinline__ uint32_t filter_tile(CQ& Q, const uint8_t* smem_shared, const WaveArea& W, int m, int lane,
                                                int nvalid, bool& ok_hdr) {
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(64 * k + lane < nvalid) << k;
    const StrLds L{W.tab, W.offs, W.first1, W.last2, W.recs};
    const int npreds = Q.npreds;
    CP& PL = Q.preds[npreds - 1];
    StrTile S;
    if (kEager) str_begin(Q.cols[PL.col], m, lane, S);
    int64_t v[4];
    int last_col = -1;
    for (int a = 0; a < (kEager ? npreds - 1 : npreds); ++a) {
        CP& P = Q.preds[a];
        if (!kEager && P.kind == PK_STR) {
            if (!kStr) {
                ok_hdr = false;  // unreachable: the launch picks the string instantiation
                return 0;
            } else if (kStr == 2 && Q.cols[P.col].enc == ENC_FSST) {
                mask &= fsst_pred(Q, Q.cols[P.col], m, lane, nvalid, reinterpret_cast<uint8_t*>(W.offs), smem_shared,
                                  ok_hdr);
            } else {
                // (the table is loaded for the plan's last atom only)
                if (str_mode(P.n1, P.n2) == kStrShifted)
                    mask &= str_pred<kStrShifted>(Q.cols[P.col], P, m, lane, nvalid, L, ok_hdr);
                else
                    mask &= str_pred<kStrMasked>(Q.cols[P.col], P, m, lane, nvalid, L, ok_hdr);
            }
        } else {
            const int z = zone_test(Q.cols[P.col], P, m);
            if (z == 1) continue;
            if (z == 0) return 0;
            if (P.col != last_col) {
                ok_hdr &= decode_dense(Q.cols[P.col], m, lane, v);
                last_col = P.col;
            }
            mask &= eval_int_pred(P, Q.in_vals, v);
        }
        if (__ballot(mask != 0) == 0) return 0;  // no survivor in this mini block
    }
    if (kEager) {
        const int mode = PL.tab_rot ? kStrTable : str_mode(PL.n1, PL.n2);
        if (mode == kStrTable)
            mask &= str_finish<kStrTable>(Q.cols[PL.col], PL, lane, nvalid, S, L, ok_hdr);
        else if (mode == kStrShifted)
            mask &= str_finish<kStrShifted>(Q.cols[PL.col], PL, lane, nvalid, S, L, ok_hdr);
        else
            mask &= str_finish<kStrMasked>(Q.cols[PL.col], PL, lane, nvalid, S, L, ok_hdr);
    }
    return mask;
}

// Rows of mask (row 64 k + lane -> bit k) of mini block m whose first
// probe finds its key.
__device__ __forceinline__ uint32_t member_tile(CQ& Q, const uint8_t* smem_shared, int m, int lane, uint32_t mask,
                                                bool& ok_hdr) {
    CPR& P0 = Q.probes[0];
    CC& fc = Q.cols[P0.fk_col];
    int64_t fk[4];
    ok_hdr &= decode_dense(fc, m, lane, fk);
    if (fc.enc == ENC_DICT)
#pragma unroll
        for (int k = 0; k < 4; ++k) fk[k] = (mask >> k) & 1u ? dict_value(fc, fk[k], ok_hdr) : 0;
    return P0.h.lds_off >= 0 ? hash_member4<true>(P0.h, smem_shared, fk, mask)
                             : hash_member4<false>(P0.h, smem_shared, fk, mask);
}

template <int kStr, bool kHash>
__device__ __forceinline__ void process_tile(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const WaveArea& W,
                                             int m, int lane, int& npend, bool& ok_hdr) {
    const int64_t row0 = (int64_t)m * kMB;
    const int nvalid = (int)min((int64_t)kMB, Q.nrows - row0);
    const int npreds = Q.npreds;

    if (npreds == 0 && Q.nprobes == 0) {
        // Neither a fact predicate nor a join: every valid row goes straight
        // to stage B.
        for (int k = 0; k < 4; ++k) {
            if (64 * k >= nvalid) break;
            int i = 64 * k + lane;
            stage_b<kHash>(Q, smem_shared, gagg, LdsSlots{W.slots + lane}, m, i, i < nvalid, ok_hdr);
        }
        return;
    }
    if (npreds == 0) return;  // probes without predicates: semi_tiles handles those plans
    // (an FSST atom is never the eager one: its plan has fs_pred >= 0)
    uint32_t mask =
        Q.nint_preds == npreds - 1 && Q.preds[npreds - 1].kind == PK_STR && Q.fs_pred < 0
            ? (kStr ? filter_tile<true, kStr>(Q, smem_shared, W, m, lane, nvalid, ok_hdr) : (ok_hdr = false, 0u))
            : filter_tile<false, kStr>(Q, smem_shared, W, m, lane, nvalid, ok_hdr);
    // The first (most selective) probe's membership test joins stage A: its
    // foreign keys are decoded for the whole mini block with coalesced
    // loads, so stage B gets only the rows that find their key (and probes
    // them again for payloads), not every row that passed the filters.
    if (Q.nprobes > 0 && __ballot(mask != 0)) mask = member_tile(Q, smem_shared, m, lane, mask, ok_hdr);
    queue_survivors<kHash>(Q, smem_shared, gagg, W, row0, mask, lane, npend, ok_hdr);
}

// Semi-join stage A of one mini block whose foreign keys issue_dense read:
// the first (most selective) probe filters; its survivors are probed again,
// with payloads, in stage B.
template <bool kHash>
__device__ __forceinline__ void semi_tile(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const WaveArea& W,
                                          int m, int lane, const RawDense& R, int& npend, bool& ok_hdr) {
    const int64_t row0 = (int64_t)m * kMB;
    const int nvalid = (int)min((int64_t)kMB, Q.nrows - row0);
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(64 * k + lane < nvalid) << k;
    CPR& P0 = Q.probes[0];
    CC& fc = Q.cols[P0.fk_col];
    int64_t fk[4];
    ok_hdr &= finish_dense(fc, R, lane, fk);
    if (fc.enc == ENC_DICT)
#pragma unroll
        for (int k = 0; k < 4; ++k) fk[k] = (mask >> k) & 1u ? dict_value(fc, fk[k], ok_hdr) : 0;
    mask = P0.h.lds_off >= 0 ? hash_member4<true>(P0.h, smem_shared, fk, mask)
                             : hash_member4<false>(P0.h, smem_shared, fk, mask);
    queue_survivors<kHash>(Q, smem_shared, gagg, W, row0, mask, lane, npend, ok_hdr);
}

// The semi-join tiles m0, m0 + NW, ... < m1 of one wave, two in flight: the
// next tile's keys are loaded while the current one is probed.
template <int NW, bool kHash>
__device__ __forceinline__ void semi_tiles(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg, const WaveArea& W,
                                           int m0, int m1, int lane, int& npend, bool& ok_hdr) {
    CC& fc = Q.cols[Q.probes[0].fk_col];
    RawDense A, B;
    if (m0 < m1) issue_dense(fc, m0, lane, A);
    for (int m = m0; m < m1; m += 2 * NW) {
        const int m2 = m + NW;
        dense_ready(A);  // as seg_ready: wait for A before B's loads are issued
        if (m2 < m1) issue_dense(fc, m2, lane, B);
        semi_tile<kHash>(Q, smem_shared, gagg, W, m, lane, A, npend, ok_hdr);
        if (m2 >= m1) break;
        dense_ready(B);
        if (m2 + NW < m1) issue_dense(fc, m2 + NW, lane, A);
        semi_tile<kHash>(Q, smem_shared, gagg, W, m2, lane, B, npend, ok_hdr);
    }
}


// Per-wave LDS: (plans with fact predicates) the survivor queue, then one
// region shared by the stage-B value slots and the string predicate's row
// offsets, s1 / s2 starts and hit queue -- a wave never uses both at once
// (a mini block's string test finishes before its survivors are queued).
constexpr size_t kSlotBytes = kMaxSlots * kWave * 8;
constexpr size_t kStrBytes = 260 * 4 + 2 * 256 * 4 + kRecCap * 16;

__host__ __device__ constexpr size_t wave_area_bytes(bool str_stage, bool pend_stage) {
    return (pend_stage ? kPendCap * 4 : 0) + (str_stage && kStrBytes > kSlotBytes ? kStrBytes : kSlotBytes);
}

__device__ __forceinline__ WaveArea wave_area(uint8_t* p, const uint32_t* tab, bool pend_stage) {
    WaveArea W;
    W.tab = tab;
    W.pend = reinterpret_cast<uint32_t*>(p);
    uint8_t* shared = p + (pend_stage ? kPendCap * 4 : 0);
    W.slots = reinterpret_cast<int64_t*>(shared);
    W.offs = reinterpret_cast<uint32_t*>(shared);
    W.first1 = W.offs + 260;
    W.last2 = W.first1 + 256;
    W.recs = reinterpret_cast<uint4*>(W.last2 + 256);
    return W;
}

// Merge the workgroup's LDS group table into the plan's global table.  The
// device-scope adds return their old values, which the caller folds into a
// sink: once the sink is known the adds have been performed.
__device__ unsigned long long flush_lds_agg(CQ& Q, uint8_t* smem_shared, unsigned long long* gagg) {
    if (!Q.agg_lds) return 0;
    const int64_t n = Q.ngroups * Q.nacc;
    unsigned long long* T = reinterpret_cast<unsigned long long*>(smem_shared + Q.agg_lds_off);
    unsigned long long sink = 0;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        unsigned long long x = T[e];
        if (x) sink += atomicAdd(gagg + e, x);
        T[e] = 0;
    }
    return sink;
}

// Load a plan's LDS-resident dimension tables and clear its LDS group table.
__device__ void load_lds_state(CQ& Q, uint8_t* smem_shared, uint32_t* str_tab) {
    if (Q.npreds > 0 && threadIdx.x < 32) {
        CP& PL = Q.preds[Q.npreds - 1];
        if (PL.kind == PK_STR && PL.tab_rot) str_tab[threadIdx.x] = PL.tab[threadIdx.x];
    }
    for (int j = 0; j < Q.nprobes; ++j) {
        CH& h = Q.probes[j].h;
        if (h.bits_lds_off >= 0) {
            cptr<uint4> src = (cptr<uint4>)h.bits;
            uint4* dst = reinterpret_cast<uint4*>(smem_shared + h.bits_lds_off);
            const uint32_t n = (uint32_t)((h.bspan + 127) / 128);  // 16-byte units
            for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = ld4(src, e);
        }
        if (h.filt_lds_off >= 0) {
            cptr<uint4> src = (cptr<uint4>)h.filt;
            uint4* dst = reinterpret_cast<uint4*>(smem_shared + h.filt_lds_off);
            const uint32_t n = (1u << h.flog2) / 128u;  // 16-byte units
            for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = ld4(src, e);
        }
        if (h.lds_off < 0) continue;
        cptr<uint4> src = (cptr<uint4>)h.keys;
        uint4* dst = reinterpret_cast<uint4*>(smem_shared + h.lds_off);
        for (uint32_t e = threadIdx.x; e < h.bytes / 16u; e += blockDim.x) dst[e] = ld4(src, e);
    }
    if (Q.agg_lds) {
        const int64_t n = Q.ngroups * Q.nacc;
        unsigned long long* T = reinterpret_cast<unsigned long long*>(smem_shared + Q.agg_lds_off);
        for (int64_t e = threadIdx.x; e < n; e += blockDim.x) T[e] = 0;
    }
}

__device__ __forceinline__ unsigned long long ld_acq(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Write a plan's non-empty groups as records [group, acc...] into its pinned
// host buffer (paper Section 3.1: the aggregate is converted into a record
// format and returned to the host), then clear the device table T (and a
// hash table's keys) and the status word for the next execution.  Run by
// one workgroup after every other one has finished.
__device__ void emit_records(CQ& Q, int32_t* ctrl, unsigned long long* T, uint32_t* status) {
    const int nacc = Q.nacc;
    const int64_t G = Q.ngroups;
    unsigned long long* K = Q.agg_hash ? T + G * nacc : nullptr;
    if (threadIdx.x == 0) ctrl[2] = 0;
    __syncthreads();
    for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
        unsigned long long key = 0;
        if (K) {
            key = ld_acq(&K[g]);
            if (key == 0) continue;
            K[g] = 0;
        }
        unsigned long long cnt = ld_acq(&T[g * nacc]);
        if (cnt == 0) continue;
        int pos = atomicAdd(&ctrl[2], 1);
        int64_t* rec = Q.host_out + 2 + (int64_t)pos * (1 + nacc);
        rec[0] = K ? (int64_t)(key - 1ull) : g;
        rec[1] = (int64_t)cnt;
        T[g * nacc] = 0;
        for (int a = 1; a < nacc; ++a) {
            rec[1 + a] = (int64_t)ld_acq(&T[g * nacc + a]);
            T[g * nacc + a] = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t st = __hip_atomic_exchange(status, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.host_out[0] = (int64_t)st;
        Q.host_out[1] = (int64_t)ctrl[2];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Work queue.  Workgroup i runs on XCD i % 8 (round-robin dispatch), and each
// XCD has its own L2, so a single queue head would serialise every claim of
// the grid on one device-coherent atomic.  Instead the items are split into
// eight contiguous ranges with one head each: a workgroup claims from its
// XCD's range, then steals from the others, skipping a drained range after a
// plain load of its head.  Completion counts per XCD and then across XCDs.
// The dispatch rule only affects speed: any workgroup may take any item.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t* ctr(const BatchArgs& a, int i) { return a.counters + i * kCounterStride; }

__device__ __forceinline__ int claim_item(const BatchArgs& a, int home, uint32_t& drained, int total) {
    for (int k = 0; k < kXcds; ++k) {
        const int x = (home + k) & (kXcds - 1);
        if ((drained >> x) & 1u) continue;
        const uint32_t lo = (uint32_t)((int64_t)total * x / kXcds);
        const uint32_t n = (uint32_t)((int64_t)total * (x + 1) / kXcds) - lo;
        uint32_t* head = ctr(a, x);
        if (k > 0 && __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) {
            drained |= 1u << x;
            continue;
        }
        const uint32_t j = atomicAdd(head, 1u);
        if (j < n) return (int)(lo + j);
        drained |= 1u << x;
    }
    return -1;
}

// True for the workgroup that finishes last (call after a fence).
__device__ __forceinline__ bool finish_last(const BatchArgs& a, int home) {
    const uint32_t nhome = (gridDim.x - 1u - (uint32_t)home) / kXcds + 1u;  // workgroups homed on this XCD
    if (atomicAdd(ctr(a, kXcds + home), 1u) != nhome - 1u) return false;
    __threadfence();
    const uint32_t nx = gridDim.x < (uint32_t)kXcds ? gridDim.x : (uint32_t)kXcds;
    return atomicAdd(ctr(a, 2 * kXcds), 1u) == nx - 1u;
}

// ---------------------------------------------------------------------------
// The persistent fused kernel (NW waves per workgroup)
// ---------------------------------------------------------------------------
// kStr: 0 no string atom in the batch, 1 string atoms on VARLEN columns, 2
// also an FSST atom.  kHash: some plan aggregates into a hash group table.
template <int NW, int kStr, bool kHash>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(kStr == 2 ? 5 : kStr ? 6 : 4, 8))) void fused_kernel(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    // Static LDS: its address is known when the kernel is compiled, so the
    // string scan's table reads take it as an immediate offset.
    __shared__ __align__(16) uint32_t str_tab[kLdsStrTabBytes / 4];
    int32_t* ctrl = reinterpret_cast<int32_t*>(smem);
    uint8_t* shared_area = smem + kLdsCtrlBytes;
    const bool str_stage = a.str_stage != 0;
    const int lane = lane_id();
    const int wave = uniform_i32(threadIdx.x >> 6);  // uniform: mini-block headers become scalar loads
    const bool pend_stage = a.pend_stage != 0;
    const WaveArea W =
        wave_area(shared_area + a.lds_shared + (size_t)wave * wave_area_bytes(str_stage, pend_stage), str_tab,
                  pend_stage);
    const int total_items = a.item_start[a.nq];

    const int home = (int)(blockIdx.x % kXcds);
    uint32_t drained = 0;  // thread 0: item ranges found empty
    unsigned long long sink = 0;  // old values of this thread's device-scope atomics
    bool direct = false;          // some plan aggregated straight into global memory
    int cur = -1;
    int fs_chunk = -1;  // chunk whose FSST code tables are in LDS
    bool ok_hdr = true;
    int npend = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) ctrl[0] = claim_item(a, home, drained, total_items);
        __syncthreads();
        const int item = uniform_i32(ctrl[0]);
        if (item < 0) break;
        int qi = 0;
        while (qi + 1 < a.nq && a.item_start[qi + 1] <= item) ++qi;
        qi = uniform_i32(qi);
        CQ& Q = *ro(a.q[qi]);
        unsigned long long* const gagg = reinterpret_cast<unsigned long long*>(a.agg[qi]);
        if (qi != cur) {
            if (cur >= 0) {
                unsigned long long* const cagg = reinterpret_cast<unsigned long long*>(a.agg[cur]);
                // Queued survivors stay valid across the items of one plan:
                // they go to stage B when the queue fills, at a plan switch
                // (before the plan's LDS state is replaced) and at the end.
                // The string instantiation also flushes at every item's end:
                // its survivors are few, and a full flush in the middle of an
                // item keeps the workgroup's other waves waiting at the next
                // item's barrier (measured: without string atoms, deferring
                // is faster; with them, flushing per item).
                if (npend) flush_pending<kHash>(*ro(a.q[cur]), shared_area, cagg, W, npend, lane, ok_hdr);
                __syncthreads();
                sink += flush_lds_agg(*ro(a.q[cur]), shared_area, cagg);
                if (!ok_hdr) sink += atomicOr(a.status[cur], ST_CORRUPT);
                ok_hdr = true;
            }
            __syncthreads();
            load_lds_state(Q, shared_area, str_tab);
            if (kStr == 2) fsst_load_dfa(Q, shared_area);
            fs_chunk = -1;
            __syncthreads();
            cur = qi;
            direct |= Q.agg_lds == 0;
        }
        // The item's mini blocks: a slice of the plan, or, after chunk
        // pruning, a slice of one surviving block.
        const int t = item - a.item_start[qi];
        int mb0, mb1;
        if (Q.live) {
            const int ipc = (Q.prune_mb + a.mb_per_item - 1) / a.mb_per_item;  // items per block
            const int j = t / ipc;
            const int blk = ro(Q.live)[j];
            mb0 = blk * Q.prune_mb + (t - j * ipc) * a.mb_per_item;
            mb1 = min(min(mb0 + a.mb_per_item, (blk + 1) * Q.prune_mb), Q.nmb);
        } else {
            mb0 = t * a.mb_per_item;
            mb1 = min(mb0 + a.mb_per_item, Q.nmb);
        }
        if (Q.npreds == 0 && Q.nprobes > 0) {
            semi_tiles<NW, kHash>(Q, shared_area, gagg, W, mb0 + wave, mb1, lane, npend, ok_hdr);
        } else if (kStr == 2 && Q.fs_pred >= 0) {
            // FSST: the item's mini blocks chunk by chunk, each chunk's code
            // tables built once by the workgroup
            const int mbpc = max(Q.cols[Q.preds[Q.fs_pred].col].mbpc, 1);
            for (int s0 = mb0; s0 < mb1;) {
                const int k = s0 / mbpc;
                const int s1 = min(mb1, (k + 1) * mbpc);
                if (k != fs_chunk) {
                    __syncthreads();
                    fsst_load_chunk(Q, shared_area, k);
                    __syncthreads();
                    fs_chunk = k;
                }
                for (int m = s0 + wave; m < s1; m += NW)
                    process_tile<kStr, kHash>(Q, shared_area, gagg, W, m, lane, npend, ok_hdr);
                s0 = s1;
            }
        } else {
            for (int m = mb0 + wave; m < mb1; m += NW)
                process_tile<kStr, kHash>(Q, shared_area, gagg, W, m, lane, npend, ok_hdr);
        }
        if (kStr && npend) flush_pending<kHash>(Q, shared_area, gagg, W, npend, lane, ok_hdr);
    }
    if (cur >= 0) {
        unsigned long long* const cagg = reinterpret_cast<unsigned long long*>(a.agg[cur]);
        if (npend) flush_pending<kHash>(*ro(a.q[cur]), shared_area, cagg, W, npend, lane, ok_hdr);
        __syncthreads();
        sink += flush_lds_agg(*ro(a.q[cur]), shared_area, cagg);
        if (!ok_hdr) sink += atomicOr(a.status[cur], ST_CORRUPT);
    }
    // Last workgroup out emits every plan's records and resets the queue.
    // Publishing: the workgroup's global effects are device-scope atomics,
    // which are coherent across XCDs; waiting for their returned values
    // (the sink) orders them before the completion count, so the costly
    // agent-scope release fence (an L2 writeback) is needed only where rows
    // were aggregated straight into global memory with plain-result atomics.
    if (direct) __threadfence();
    if (sink == ~0ull) ctrl[3] = 1;  // consumes every returned value
    __syncthreads();
    if (threadIdx.x == 0) ctrl[1] = finish_last(a, home) ? 1 : 0;
    __syncthreads();
    if (!ctrl[1]) return;
    __threadfence();
    for (int qi = 0; qi < a.nq; ++qi)
        emit_records(*ro(a.q[qi]), ctrl, reinterpret_cast<unsigned long long*>(a.agg[qi]), a.status[qi]);
    if (threadIdx.x < 2 * kXcds + 1)  // every other workgroup has left: reset for the next launch
        __hip_atomic_store(ctr(a, threadIdx.x), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence_system();
}

// ---------------------------------------------------------------------------
// Hash build (dimension scan -> filter -> insert)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hash_tile_mask(CHB& A, int m, int lane, int nvalid,
                                                   int64_t key[4], int64_t pay[2][4], bool& ok) {
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(64 * k + lane < nvalid) << k;
    int64_t v[4];
    for (int p = 0; p < A.npreds; ++p) {
        CP& P = A.preds[p];
        ok &= decode_dense(A.cols[P.col], m, lane, v);
        mask &= eval_int_pred(P, A.in_vals, v);
    }
    CC& kc = A.cols[A.key_col];
    ok &= decode_dense(kc, m, lane, key);
    if (kc.enc == ENC_DICT)
        for (int k = 0; k < 4; ++k) key[k] = dict_value(kc, key[k], ok);
    for (int j = 0; j < A.npay; ++j) {
        if (A.pay_src[j] >= 0) continue;  // taken from a probe below
        CC& pc = A.cols[A.pay_col[j]];
        ok &= decode_dense(pc, m, lane, pay[j]);
        if (pc.enc == ENC_DICT)
            for (int k = 0; k < 4; ++k) pay[j][k] = dict_value(pc, pay[j][k], ok);
    }
    // A joined build side (Section 3.1, Kernel #2): each row must find its
    // foreign key in every probed table; payloads may come from those tables.
    for (int s = 0; s < A.nsub; ++s) {
        if (__ballot(mask != 0) == 0) break;
        CPR& P = A.sub[s];
        CC& fc = A.cols[P.fk_col];
        int64_t fk[4];
        ok &= decode_dense(fc, m, lane, fk);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((mask >> k) & 1u)) continue;
            if (fc.enc == ENC_DICT) fk[k] = dict_value(fc, fk[k], ok);
            const bool maybe = !P.h.bits || bitmap_has_global(P.h, fk[k]);
            const int slot = maybe ? hash_find<false>(P.h, nullptr, fk[k]) : -1;
            if (slot < 0) {
                mask &= ~(1u << k);
                continue;
            }
            for (int j = 0; j < A.npay; ++j)
                if (A.pay_src[j] == s) pay[j][k] = hash_payload<false>(P.h, nullptr, A.pay_col[j], slot);
        }
    }
    return mask;
}

__global__ __launch_bounds__(kBlock) void hash_count_kernel(const HashBuildArgs* __restrict__ args) {
    CHB& A = *ro(args);
    const int lane = lane_id();
    const int gw = uniform_i32((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));  // wave-uniform
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    unsigned long long cnt = 0;
    long long mn0 = INT64_MAX, mx0 = INT64_MIN, mn1 = INT64_MAX, mx1 = INT64_MIN, mn2 = INT64_MAX, mx2 = INT64_MIN;
    for (int m = gw; m < A.nmb; m += nw) {
        const int nvalid = (int)min((int64_t)kMB, A.nrows - (int64_t)m * kMB);
        int64_t key[4], pay[2][4];
        uint32_t mask = hash_tile_mask(A, m, lane, nvalid, key, pay, ok);
        for (int k = 0; k < 4; ++k) {
            if (!((mask >> k) & 1u)) continue;
            cnt += 1;
            mn0 = min(mn0, (long long)key[k]);
            mx0 = max(mx0, (long long)key[k]);
            if (A.npay > 0) { mn1 = min(mn1, (long long)pay[0][k]); mx1 = max(mx1, (long long)pay[0][k]); }
            if (A.npay > 1) { mn2 = min(mn2, (long long)pay[1][k]); mx2 = max(mx2, (long long)pay[1][k]); }
        }
    }
    if (cnt) {
        atomicAdd(A.count, cnt);
        atomicMin(&A.mm[0], mn0);
        atomicMax(&A.mm[1], mx0);
        if (A.npay > 0) { atomicMin(&A.mm[2], mn1); atomicMax(&A.mm[3], mx1); }
        if (A.npay > 1) { atomicMin(&A.mm[4], mn2); atomicMax(&A.mm[5], mx2); }
    }
    if (!ok) atomicOr(A.status, ST_CORRUPT);
}

__global__ __launch_bounds__(kBlock) void hash_insert_kernel(const HashBuildArgs* __restrict__ args) {
    CHB& A = *ro(args);
    const int lane = lane_id();
    const int gw = uniform_i32((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));  // wave-uniform
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    uint32_t flags = 0;
    for (int m = gw; m < A.nmb; m += nw) {
        const int nvalid = (int)min((int64_t)kMB, A.nrows - (int64_t)m * kMB);
        int64_t key[4], pay[2][4];
        uint32_t mask = hash_tile_mask(A, m, lane, nvalid, key, pay, ok);
        for (int k = 0; k < 4; ++k) {
            if (!((mask >> k) & 1u)) continue;
            if (key[k] < INT32_MIN || key[k] > INT32_MAX || key[k] == kEmptyKey) {
                flags |= ST_UNSUPPORTED;
                continue;
            }
            const int32_t kk = (int32_t)key[k];
            uint32_t s = hash32(kk, A.log2cap);
            for (uint32_t n = 0;; ++n) {
                if (n > A.cap_mask) { flags |= ST_CAPACITY; break; }
                int32_t prev = atomicCAS(&A.keys[s], kEmptyKey, kk);
                if (prev == kEmptyKey) {
                    if (A.bits) {
                        const uint64_t d = (uint64_t)(key[k] - A.bmin);
                        atomicOr(&A.bits[d >> 5], 1u << (d & 31));
                    }
                    if (A.filt) {
                        const uint32_t fb = filter_bit(kk, A.flog2), fb2 = filter_bit2(kk, A.flog2);
                        atomicOr(&A.filt[fb >> 5], 1u << (fb & 31));
                        atomicOr(&A.filt[fb2 >> 5], 1u << (fb2 & 31));
                    }
                    for (int j = 0; j < A.npay; ++j) {
                        if (A.pay64[j]) reinterpret_cast<int64_t*>(A.pay[j])[s] = pay[j][k];
                        else reinterpret_cast<int32_t*>(A.pay[j])[s] = (int32_t)pay[j][k];
                    }
                    break;
                }
                if (prev == kk) { flags |= ST_DUPLICATE; break; }
                s = (s + 1) & A.cap_mask;
            }
        }
    }
    if (!ok) flags |= ST_CORRUPT;
    if (flags) atomicOr(A.status, flags);
}

// Bandwidth probe (measurement only, not on the query path): every lane
// streams 16-byte loads over [p, p + n16 * 16) in a grid-stride loop, four
// loads in flight, and folds them into one word that is stored only when it
// equals the caller's value `key`, so that no load can be dropped.
__global__ __launch_bounds__(256) void stream_read_kernel(const uint4* __restrict__ p, uint64_t n16,
                                                           uint32_t key, uint32_t* __restrict__ sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    cptr<u32x4> v = (cptr<u32x4>)p;
    uint32_t acc = 0;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 x0 = v[i], x1 = v[i + stride], x2 = v[i + 2 * stride], x3 = v[i + 3 * stride];
        acc ^= (x0.x ^ x0.y ^ x0.z ^ x0.w) + (x1.x ^ x1.y ^ x1.z ^ x1.w) + (x2.x ^ x2.y ^ x2.z ^ x2.w) +
               (x3.x ^ x3.y ^ x3.z ^ x3.w);
    }
    for (; i < n16; i += stride) {
        const u32x4 x = v[i];
        acc ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    if (acc == key) sink[0] = acc;
}

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Fragmented execution: one kernel per step, intermediates in HBM.  Each
// kernel is the straightforward data-parallel form of its step, with
// workgroup-level aggregation of its atomics.
// ---------------------------------------------------------------------------
// Decode one integer column to int64 (codes for DICT).
__global__ __launch_bounds__(kBlock) void frag_decode_int(const DevQuery* __restrict__ q, int c, int64_t* out) {
    CQ& Q = *ro(q);
    CC& C = Q.cols[c];
    const int lane = lane_id();
    const int gw = uniform_i32((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));  // wave-uniform
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    for (int m = gw; m < Q.nmb; m += nw) {
        int64_t v[4];
        ok &= decode_dense(C, m, lane, v);
        for (int k = 0; k < 4; ++k) {
            int64_t r = (int64_t)m * kMB + 64 * k + lane;
            if (r < Q.nrows) out[r] = v[k];
        }
    }
    if (!ok) atomicOr(Q.status, ST_CORRUPT);
}

// Decode a string column: offsets [nrows + 1] and a copy of the bytes.
__global__ __launch_bounds__(kBlock) void frag_decode_str(const DevQuery* __restrict__ q, int c, int64_t* off,
                                                           uint8_t* bytes) {
    CQ& Q = *ro(q);
    CC& C = Q.cols[c];
    const int lane = lane_id();
    const int gw = uniform_i32((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));  // wave-uniform
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    for (int m = gw; m < Q.nmb; m += nw) {
        const int nvalid = (int)min((int64_t)kMB, Q.nrows - (int64_t)m * kMB);
        MbHdr h = mb_hdr(C, m);
        ok &= h.ok;
        uint64_t h0 = ro(C.hoff)[m], h1 = ro(C.hoff)[m + 1];
        if (!(h0 <= h1 && h1 <= C.heap_bytes)) { ok = false; continue; }
        uint64_t carry = h0;
        for (int k = 0; k < 4; ++k) {
            int i = 64 * k + lane;
            uint64_t len = (i < nvalid) ? (uint64_t)h.base + (h.b ? bits_at(h.w, (uint32_t)i * h.b, h.b) : 0) : 0;
            uint64_t s = wave_incl_scan_u64(len);
            if (i < nvalid) off[(int64_t)m * kMB + i] = (int64_t)(carry + s - len);
            carry += readlane_u64(s, 63);
        }
        if (carry != h1) ok = false;
        // copy the bytes: 16-byte pieces where both sides are aligned
        uint64_t b = h0;
        while (b < h1 && (b & 15)) {
            if (b + lane < h1 && ((b + lane) & ~uint64_t(15)) == (b & ~uint64_t(15))) bytes[b + lane] = ro(C.heap)[b + lane];
            b = (b | 15) + 1;
        }
        for (uint64_t v = b + 16 * (uint64_t)lane; v + 16 <= h1; v += 16 * kWave)
            *reinterpret_cast<uint4*>(bytes + v) = ld4((cptr<uint4>)(C.heap + v), 0);
        uint64_t tail = b + ((h1 > b ? h1 - b : 0) & ~uint64_t(15));
        if (tail + lane < h1) bytes[tail + lane] = ro(C.heap)[tail + lane];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[Q.nrows] = (int64_t)Q.cols[c].heap_bytes;
    if (!ok) atomicOr(Q.status, ST_CORRUPT);
}

// FSST record decode (Section 4.1): one wave per mini block, lane l on rows
// 4 l .. 4 l + 3.  Pass 1 walks the codes for the decoded record lengths and
// a wave prefix sum gives every row's output offset; pass 2 decodes the
// records in parallel into an LDS staging window, copied out with
// coalesced stores (a mini block larger than the window takes several
// windows).  Each wave takes a contiguous run of mini blocks and keeps the
// symbol table of the current chunk in its LDS.  Both passes take eight
// codes a step, so that their table reads are issued together.  The window
// (7.5 KiB, above the 6.8 KiB that 256 rows of the string workload's
// comments decode to) lets four workgroups share a CU's LDS.
constexpr int kFsstStage = 7680;
// + 16: the spill of the last 8-byte symbol write, and the copy-out's
// read-ahead dword
constexpr size_t kFsstDecodeWaveBytes = 256 * 8 + 256 + kFsstStage + 16;
// an 8-byte store at any byte address (gfx950's LDS takes unaligned access)
typedef uint64_t u64_ua __attribute__((aligned(1)));

__global__ __launch_bounds__(kBlock) void frag_decode_fsst(const DevQuery* __restrict__ q, int c, int64_t* off,
                                                           uint8_t* bytes) {
    extern __shared__ __align__(16) uint8_t smem[];
    CQ& Q = *ro(q);
    CC& C = Q.cols[c];
    const int lane = lane_id();
    const int wave = uniform_i32(threadIdx.x >> 6);
    uint8_t* wa = smem + (size_t)wave * kFsstDecodeWaveBytes;
    uint64_t* sym = reinterpret_cast<uint64_t*>(wa);
    uint8_t* len = wa + 256 * 8;
    uint8_t* stage = wa + 256 * 8 + 256;
    const int nw = gridDim.x * kWaves;
    const int gw = blockIdx.x * kWaves + wave;
    const int per = (Q.nmb + nw - 1) / nw;
    const int m0 = gw * per, m1 = min(Q.nmb, m0 + per);
    const int mbpc = max(C.mbpc, 1);
    int chunk = -1;
    bool ok = true;
    for (int m = m0; m < m1; ++m) {
        const int nvalid = (int)min((int64_t)kMB, Q.nrows - (int64_t)m * kMB);
        if (m / mbpc != chunk) {
            chunk = m / mbpc;
            cptr<uint8_t> tab = ro(C.symtab) + (size_t)chunk * (256 * 8 + 256);
            wave_lds_sync();
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = 64 * j + lane;
                const uint32_t le = e < 255 ? min((uint32_t)tab[256 * 8 + e], 8u) : 0u;
                // bytes past a symbol's length are zero in LDS (code 255: none)
                sym[e] = ((cptr<uint64_t>)tab)[e] & (le >= 8u ? ~0ull : (1ull << (8 * le)) - 1ull);
                len[e] = (uint8_t)le;
            }
            wave_lds_sync();
        }
        uint32_t rl[4], lsum, incl;
        uint64_t h0;
        if (!fsst_lengths(C, m, lane, nvalid, rl, lsum, incl, h0)) { ok = false; continue; }
        const uint64_t d0 = ro(C.doff)[m], d1 = ro(C.doff)[m + 1];
        if (!(d0 <= d1 && d1 <= C.str_bytes)) { ok = false; continue; }
        // pass 1: decoded lengths, the lane's four rows' codes as one run,
        // eight codes a step (a literal counts 1 byte; the bytes before each
        // row boundary are summed on the side).  A code of length 0 and an
        // escape as the lane's last code mark the column corrupt.
        CodeReader R;
        R.init(C.heap, h0, incl - lsum);
        bool esc = false;
        const uint32_t c1 = rl[0], c2 = c1 + rl[1], c3 = c2 + rl[2];
        uint32_t n = 0, n1 = 0, n2 = 0, n3 = 0;
        for (uint32_t i = 0; i < lsum;) {
            uint32_t qa, qb;
            R.peek8(qa, qb);
            const uint32_t nq = min(lsum - i, 8u);
            uint32_t l[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) l[j] = len[((j < 4 ? qa : qb) >> (8 * (j & 3))) & 0xFFu];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t cd = ((j < 4 ? qa : qb) >> (8 * (j & 3))) & 0xFFu;
                const bool act = (uint32_t)j < nq;
                const bool lit = esc;
                ok = ok && !(act && !lit && cd != 255u && l[j] == 0);
                const uint32_t cb = act ? (lit ? 1u : l[j]) : 0u;
                const uint32_t k = i + j;
                n += cb;
                n1 += k < c1 ? cb : 0u;
                n2 += k < c2 ? cb : 0u;
                n3 += k < c3 ? cb : 0u;
                esc = act ? (!lit && cd == 255u) : esc;
            }
            i += nq;
            R.advance(nq);
        }
        if (esc) { ok = false; esc = false; }
        const uint32_t dl[4] = {n1, n2 - n1, n3 - n2, n - n3};
        const uint32_t dsum = n;
        const uint32_t dincl = wave_incl_scan_u32(dsum);
        const uint32_t dtotal = __builtin_amdgcn_readlane(dincl, 63);
        if ((uint64_t)dtotal != d1 - d0) { ok = false; continue; }
        uint32_t start = dincl - dsum;
        {
            uint32_t o = start;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * lane + j;
                if (r < nvalid) off[(int64_t)m * kMB + r] = (int64_t)(d0 + o);
                o += dl[j];
            }
        }
        // pass 2: decode window by window.  A symbol is stored as one
        // unaligned 8-byte LDS write (its padding bytes are overwritten by
        // the next symbol); a lane's last writes can spill up to 7 zero bytes
        // into the next lane's first bytes, so after the window every lane
        // writes its first 7 bytes again, exactly.
        const uint32_t dend = start + dsum;
        for (uint32_t w0 = 0; w0 < dtotal; w0 += kFsstStage) {
            const uint32_t wn = min((uint32_t)kFsstStage, dtotal - w0);
            const uint32_t wend = w0 + wn;
            const bool here = start < wend && dend > w0;
            if (here) {
                R.init(C.heap, h0, incl - lsum);
                uint32_t d = start;  // decoded position of the next byte
                uint32_t rem = lsum;
                while (rem && d < wend) {
                    uint32_t qa, qb;
                    R.peek8(qa, qb);
                    const uint32_t nq = min(rem, 8u);
                    uint64_t sv[8];
                    uint32_t l[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint32_t cd = ((j < 4 ? qa : qb) >> (8 * (j & 3))) & 0xFFu;
                        sv[j] = sym[cd];
                        l[j] = len[cd];
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if ((uint32_t)j < nq) {
                            const uint32_t cd = ((j < 4 ? qa : qb) >> (8 * (j & 3))) & 0xFFu;
                            const uint32_t L = esc ? 1u : l[j];
                            const uint64_t v = esc ? (uint64_t)cd : sv[j];
                            esc = !esc && cd == 255u;
                            if (d - w0 < wn) {
                                *reinterpret_cast<u64_ua*>(stage + (d - w0)) = v;
                            } else if (d < w0 && d + L > w0) {  // a symbol across the window's start
                                for (uint32_t b = w0 - d; b < L; ++b) stage[d + b - w0] = (uint8_t)(v >> (8 * b));
                            }
                            d += L;
                        }
                    }
                    rem -= nq;
                    R.advance(nq);
                }
                esc = false;
            }
            wave_lds_sync();
            // the lane's first bytes (at most 7), which the previous lanes'
            // spill may have zeroed, decoded again and stored byte by byte
            if (here && start >= w0) {
                const uint32_t hend = min(min(dend, start + 7u), wend);
                R.init(C.heap, h0, incl - lsum);
                uint32_t d = start, rem = lsum;
                while (rem && d < hend) {
                    const uint32_t cd = R.peek4() & 0xFFu;
                    uint32_t L = len[cd];
                    uint64_t v = sym[cd];
                    if (cd == 255u && rem > 1) {
                        R.advance(1);
                        --rem;
                        v = R.peek4() & 0xFFu;
                        L = 1;
                    }
                    for (uint32_t b = 0; b < L && d + b < hend; ++b) stage[d + b - w0] = (uint8_t)(v >> (8 * b));
                    d += L;
                    --rem;
                    R.advance(1);
                }
            }
            wave_lds_sync();
            // copy-out: bytes up to a 4-byte boundary of the destination,
            // then whole dwords (two aligned LDS dwords realigned), then the
            // tail
            uint8_t* dst = bytes + d0 + w0;
            const uint32_t head = min(wn, (uint32_t)((4u - ((uintptr_t)dst & 3u)) & 3u));
            if ((uint32_t)lane < head) dst[lane] = stage[lane];
            const uint32_t nd = (wn - head) >> 2;
            uint32_t* dw = reinterpret_cast<uint32_t*>(dst + head);
            const uint32_t* sw = reinterpret_cast<const uint32_t*>(stage);
            for (uint32_t i = lane; i < nd; i += kWave) {
                const uint32_t so = head + 4u * i;
                dw[i] = __builtin_amdgcn_alignbyte(sw[(so >> 2) + 1], sw[so >> 2], so & 3u);
            }
            for (uint32_t i = head + 4u * nd + lane; i < wn; i += kWave) dst[i] = stage[i];
            wave_lds_sync();
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[Q.nrows] = (int64_t)C.str_bytes;
    if (!ok) atomicOr(Q.status, ST_CORRUPT);
}

__global__ void frag_filter_int(const DevQuery* __restrict__ q, int pi, const int64_t* vals, uint8_t* flags,
                                int first) {
    CQ& Q = *ro(q);
    CP& P = Q.preds[pi];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q.nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t v4[4] = {vals[r], 0, 0, 0};
        bool t = eval_int_pred(P, Q.in_vals, v4) & 1u;
        flags[r] = (uint8_t)((first ? 1 : flags[r]) & t);
    }
}

// The string atom over the materialised column: the same heap scan as the
// fused kernel's string test (aligned-word table or byte windows), one wave
// per 256 rows, reading the decoded offsets and the copied bytes (mcol: the
// column's descriptor with its heap pointing at that copy); one flag per row.
template <int kMode>
__global__ __launch_bounds__(kBlock) void frag_filter_str(const DevQuery* __restrict__ q, const DevCol* __restrict__ mcol,
                                                          int pi, const int64_t* __restrict__ off, uint8_t* flags,
                                                          int first) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ __align__(16) uint32_t tab[32];
    CQ& Q = *ro(q);
    CP& P = Q.preds[pi];
    CC& C = *ro(mcol);
    if (threadIdx.x < 32) tab[threadIdx.x] = P.tab[threadIdx.x];
    __syncthreads();
    const int lane = lane_id();
    const int wave = uniform_i32(threadIdx.x >> 6);
    uint8_t* wa = smem + (size_t)wave * (260 * 4 + 2 * 256 * 4 + kRecCap * 16);
    uint32_t* offs = reinterpret_cast<uint32_t*>(wa);
    const StrLds L{tab, offs, offs + 260, offs + 516, reinterpret_cast<uint4*>(offs + 772)};
    bool ok = true;
    for (int m = blockIdx.x * kWaves + wave; m < Q.nmb; m += gridDim.x * kWaves) {
        const int64_t row0 = (int64_t)m * kMB;
        const int nvalid = (int)min((int64_t)kMB, Q.nrows - row0);
        StrTile S;
        S.h0 = (uint64_t)ro(off)[row0];
        S.h1 = (uint64_t)ro(off)[row0 + nvalid];
        S.ok = S.h0 <= S.h1 && S.h1 <= C.heap_bytes && (S.h1 - S.h0) < (uint64_t(1) << 30);
        const uint64_t a0 = S.h0 & ~uint64_t(15);
        S.g = (cptr<uint4>)(C.heap + a0);
        S.gp = C.heap + a0;
        const uint32_t nvec = S.ok ? (uint32_t)((S.h1 - a0 + 15u) >> 4) : 0u;
        if (S.ok) load_segment(S.cur, S, 0, nvec, lane);
        // row offsets within the mini block, from the materialised offsets
        uint4 ov;
        const int64_t rb = row0 + 4 * lane;
        const int64_t rend = row0 + nvalid;
        ov.x = (uint32_t)((uint64_t)ro(off)[min(rb, rend)] - S.h0);
        ov.y = (uint32_t)((uint64_t)ro(off)[min(rb + 1, rend)] - S.h0);
        ov.z = (uint32_t)((uint64_t)ro(off)[min(rb + 2, rend)] - S.h0);
        ov.w = (uint32_t)((uint64_t)ro(off)[min(rb + 3, rend)] - S.h0);
        reinterpret_cast<uint4*>(offs)[lane] = ov;
        if (lane == 0) offs[256] = (uint32_t)(S.h1 - S.h0);
        const uint32_t mask = str_finish<kMode, true>(C, P, lane, nvalid, S, L, ok);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = 64 * k + lane;
            if (i >= nvalid) continue;
            const int64_t r = row0 + i;
            const bool prev = first ? true : flags[r] != 0;
            flags[r] = (uint8_t)(prev && ((mask >> k) & 1u));
        }
        wave_lds_sync();
    }
    if (!ok) atomicOr(Q.status, ST_CORRUPT);
}

// flags -> row list (order not preserved; aggregation is order-free).  One
// global atomic per workgroup step of 1024 rows.
// Output space is reserved once per tile of kFragTile rows (16 per thread):
// one device-scope atomic on the list's counter per tile.  With one per
// 64- or 1,024-row step the atomics on that single counter serialised the
// kernels.
constexpr int kFragRows = 16;
constexpr int kFragTile = kBlock * kFragRows;

// Per wave: its survivors' count from the per-lane keep bits (bit k: row k
// of the lane), then the tile's reservation; returns the wave's first slot.
__device__ __forceinline__ unsigned long long frag_reserve(uint32_t keep, unsigned long long* count, int lane,
                                                           int wave) {
    __shared__ uint32_t wcnt[kWaves];
    __shared__ unsigned long long base_s;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kFragRows; ++k) c += (uint32_t)__popcll(__ballot((keep >> k) & 1u));
    if (lane == 0) wcnt[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) { const uint32_t x = wcnt[w]; wcnt[w] = t; t += x; }
        base_s = t ? atomicAdd(count, (unsigned long long)t) : 0;
    }
    __syncthreads();
    const unsigned long long o = base_s + wcnt[wave];
    __syncthreads();  // wcnt and base_s are rewritten by the next tile
    (void)lane;
    return o;
}

__global__ __launch_bounds__(kBlock) void frag_compact(const DevQuery* __restrict__ q, const uint8_t* flags,
                                                       FragRow* rows, unsigned long long* count) {
    CQ& Q = *ro(q);
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int64_t t0 = (int64_t)blockIdx.x * kFragTile; t0 < Q.nrows; t0 += (int64_t)gridDim.x * kFragTile) {
        uint32_t keep = 0;
#pragma unroll
        for (int k = 0; k < kFragRows; ++k) {
            const int64_t r = t0 + (int64_t)k * kBlock + threadIdx.x;
            keep |= (uint32_t)(r < Q.nrows && flags[r]) << k;
        }
        unsigned long long o = frag_reserve(keep, count, lane, wave);
#pragma unroll
        for (int k = 0; k < kFragRows; ++k) {
            const bool f = (keep >> k) & 1u;
            const uint64_t b = __ballot(f);
            if (f) rows[o + bits_below(b)] = (FragRow)(t0 + (int64_t)k * kBlock + threadIdx.x);
            o += (uint32_t)__popcll(b);
        }
    }
}

// all rows -> row list (plans without a fact predicate)
__global__ void frag_iota(const DevQuery* __restrict__ q, FragRow* rows, unsigned long long* count) {
    CQ& Q = *ro(q);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q.nrows;
         r += (int64_t)gridDim.x * blockDim.x)
        rows[r] = (FragRow)r;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = (unsigned long long)Q.nrows;
}

// Probe j: keep listed rows whose key is found; carry the earlier payload
// arrays along and append this probe's payloads.
__global__ __launch_bounds__(kBlock) void frag_probe(const DevQuery* __restrict__ q, int j, const int64_t* fkvals,
                                                     const FragRow* rin, const unsigned long long* nin,
                                                     FragRow* rout, unsigned long long* nout,
                                                     const FragBuffers fb, int src, int npay_before) {
    CQ& Q = *ro(q);
    CPR& P = Q.probes[j];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int64_t n = (int64_t)*nin;
    CC& fc = Q.cols[P.fk_col];
    for (int64_t t0 = (int64_t)blockIdx.x * kFragTile; t0 < n; t0 += (int64_t)gridDim.x * kFragTile) {
        uint32_t keep = 0;
        int slot[kFragRows];
#pragma unroll
        for (int k = 0; k < kFragRows; ++k) {
            const int64_t e = t0 + (int64_t)k * kBlock + threadIdx.x;
            slot[k] = -1;
            if (e < n) {
                int64_t fk = fkvals[(int64_t)rin[e]];
                bool okd = true;
                if (fc.enc == ENC_DICT) fk = dict_value(fc, fk, okd);
                // the same bitmap pre-test as the fused kernel's stage B
                if (!P.h.bits || bitmap_has_global(P.h, fk)) slot[k] = hash_find<false>(P.h, nullptr, fk);
            }
            keep |= (uint32_t)(slot[k] >= 0) << k;
        }
        unsigned long long o = frag_reserve(keep, nout, lane, wave);
#pragma unroll
        for (int k = 0; k < kFragRows; ++k) {
            const bool f = (keep >> k) & 1u;
            const uint64_t b = __ballot(f);
            if (f) {
                const int64_t e = t0 + (int64_t)k * kBlock + threadIdx.x;
                const unsigned long long w = o + bits_below(b);
                rout[w] = rin[e];
                for (int t = 0; t < npay_before; ++t) fb.pay[1 - src][t][w] = fb.pay[src][t][e];
                for (int p = 0; p < P.h.npay; ++p)
                    fb.pay[1 - src][npay_before + p][w] = hash_payload<false>(P.h, nullptr, p, slot[k]);
            }
            o += (uint32_t)__popcll(b);
        }
    }
}

// Aggregate the final row list: fact values gathered from the decoded
// columns, payloads from the aligned arrays; small group tables are
// accumulated per workgroup in LDS first.
__global__ __launch_bounds__(kBlock) void frag_aggregate(const DevQuery* __restrict__ q, const FragRow* rows,
                                                         const unsigned long long* nrows_list, const FragBuffers fb,
                                                         int src) {
    __shared__ unsigned long long tab[4096];
    CQ& Q = *ro(q);
    const int64_t n = (int64_t)*nrows_list;
    const bool local = !Q.agg_hash && Q.ngroups * Q.nacc <= 4096;
    if (local)
        for (int e = threadIdx.x; e < Q.ngroups * Q.nacc; e += blockDim.x) tab[e] = 0;
    __syncthreads();
    bool okall = true;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = (int64_t)rows[e];
        RegSlots sv;
        for (int s = 0; s < kMaxSlots; ++s) sv.v[s] = 0;
        int pidx = 0;
        for (int j = 0; j < Q.nprobes; ++j) {
            for (int k = 0; k < Q.probes[j].h.npay; ++k) {
                int sl = Q.probes[j].pay_slot[k];
                if (sl >= 0) sv.set(sl, fb.pay[src][pidx][e]);
                ++pidx;
            }
        }
        for (int l = 0; l < Q.nloads; ++l) {
            CL& Ld = Q.loads[l];
            int64_t x = fb.dec[Ld.col][r];
            if (Ld.dict_val) x = dict_value(Q.cols[Ld.col], x, okall);
            sv.set(l, x);
        }
        int64_t g;
        if (!group_index(Q, sv, g)) { okall = false; continue; }
        unsigned long long* T;
        if (local) {
            T = &tab[g * Q.nacc];
        } else {
            unsigned long long* A = reinterpret_cast<unsigned long long*>(Q.agg);
            const int64_t row = agg_row(Q, A, g);
            if (row < 0) { okall = false; continue; }
            T = A + row * Q.nacc;
        }
        atomicAdd(&T[0], 1ull);
        for (int a = 1; a < Q.nacc; ++a) atomicAdd(&T[a], (unsigned long long)acc_value(Q.accs[a], sv));
    }
    __syncthreads();
    if (local)
        for (int e = threadIdx.x; e < Q.ngroups * Q.nacc; e += blockDim.x)
            if (tab[e]) atomicAdd(reinterpret_cast<unsigned long long*>(Q.agg) + e, tab[e]);
    if (!okall) atomicOr(Q.status, ST_CORRUPT);
}

__global__ __launch_bounds__(kBlock) void frag_emit(const DevQuery* __restrict__ q) {
    __shared__ int32_t ctrl[4];
    CQ& Q = *ro(q);
    __threadfence();
    emit_records(Q, ctrl, reinterpret_cast<unsigned long long*>(Q.agg), Q.status);
    __threadfence_system();
}

__global__ void frag_reset_counts(unsigned long long* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Six instantiations per workgroup size: only batches with a string atom
// carry the string stage's code and registers (its segment buffers and
// record queue), and only those with an FSST atom the FSST walk; the plain
// instantiation is smaller and spills nothing.  Only batches with a hash
// group table carry its probing code in stage B (its mere presence there
// slowed the star join by 3%).
template <int NW, int kStr, bool kHash>
hipError_t launch_fused_nwh(const BatchArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_kernel<NW, kStr, kHash>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)kLdsStrTabBytes);
        attr_set = true;
    }
    hipLaunchKernelGGL((fused_kernel<NW, kStr, kHash>), dim3(grid), dim3(NW * kWave), lds_bytes, s, a);
    return hipGetLastError();
}

template <int NW, int kStr>
hipError_t launch_fused_nw(const BatchArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
    return a.agg_hash ? launch_fused_nwh<NW, kStr, true>(a, grid, lds_bytes, s)
                      : launch_fused_nwh<NW, kStr, false>(a, grid, lds_bytes, s);
}

}  // namespace

size_t fused_wave_area_bytes(bool str, bool pend) { return wave_area_bytes(str, pend); }

hipError_t launch_fused(const BatchArgs& a, int waves, int grid, size_t lds_bytes, hipStream_t s) {
    switch (waves) {
        case 4: return a.str_stage == 2 ? launch_fused_nw<4, 2>(a, grid, lds_bytes, s)
                       : a.str_stage ? launch_fused_nw<4, 1>(a, grid, lds_bytes, s)
                                     : launch_fused_nw<4, 0>(a, grid, lds_bytes, s);
        case 8: return a.str_stage == 2 ? launch_fused_nw<8, 2>(a, grid, lds_bytes, s)
                       : a.str_stage ? launch_fused_nw<8, 1>(a, grid, lds_bytes, s)
                                     : launch_fused_nw<8, 0>(a, grid, lds_bytes, s);
        case 16: return a.str_stage == 2 ? launch_fused_nw<16, 2>(a, grid, lds_bytes, s)
                        : a.str_stage ? launch_fused_nw<16, 1>(a, grid, lds_bytes, s)
                                      : launch_fused_nw<16, 0>(a, grid, lds_bytes, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hash_count(const HashBuildArgs* d_args, int grid, hipStream_t s) {
    hipLaunchKernelGGL(hash_count_kernel, dim3(grid), dim3(kBlock), 0, s, d_args);
    return hipGetLastError();
}

hipError_t launch_hash_insert(const HashBuildArgs* d_args, int grid, hipStream_t s) {
    hipLaunchKernelGGL(hash_insert_kernel, dim3(grid), dim3(kBlock), 0, s, d_args);
    return hipGetLastError();
}

hipError_t launch_stream_read(const void* p, uint64_t bytes, uint32_t key, uint32_t* sink, int grid,
                              hipStream_t s) {
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<const uint4*>(p),
                       (uint64_t)(bytes / 16), key, sink);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    int grid = (int)(blocks < 4096 ? blocks : 4096);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fill_kernel<int32_t>, dim3(grid), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    int grid = (int)(blocks < 4096 ? blocks : 4096);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fill_kernel<int64_t>, dim3(grid), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

int run_fragmented(const DevQuery* d_q, const DevQuery& Q, const FragBuffers& fb, hipStream_t s) {
    int launches = 0;
    const int grid = 2048;
    auto chk = [&]() { ++launches; return hipGetLastError() == hipSuccess; };
    hipLaunchKernelGGL(frag_reset_counts, dim3(1), dim3(64), 0, s, fb.counts, kMaxProbes + 2);
    if (!chk()) return -1;
    // 1) decompression kernels: every referenced column, fully materialised
    bool needed[kMaxCols] = {};
    for (int p = 0; p < Q.npreds; ++p) needed[Q.preds[p].col] = true;
    for (int j = 0; j < Q.nprobes; ++j) needed[Q.probes[j].fk_col] = true;
    for (int l = 0; l < Q.nloads; ++l) needed[Q.loads[l].col] = true;
    for (int c = 0; c < Q.ncols; ++c) {
        if (!needed[c]) continue;
        if (Q.cols[c].enc == ENC_VARLEN) {
            hipLaunchKernelGGL(frag_decode_str, dim3(grid), dim3(kBlock), 0, s, d_q, c, fb.str_off[c],
                               fb.str_bytes[c]);
        } else if (Q.cols[c].enc == ENC_FSST) {
            hipLaunchKernelGGL(frag_decode_fsst, dim3(grid), dim3(kBlock), kWaves * kFsstDecodeWaveBytes, s, d_q, c,
                               fb.str_off[c], fb.str_bytes[c]);
        } else {
            hipLaunchKernelGGL(frag_decode_int, dim3(grid), dim3(kBlock), 0, s, d_q, c, fb.dec[c]);
        }
        if (!chk()) return -1;
    }
    // 2) one filter kernel per predicate, then compaction to a row list
    for (int p = 0; p < Q.npreds; ++p) {
        const int c = Q.preds[p].col;
        if (Q.preds[p].kind == PK_STR) {
            const DevPred& P = Q.preds[p];
            const int mode = P.tab_rot ? kStrTable : (P.n1 < 4 || P.n2 < 4) ? kStrMasked : kStrShifted;
            const size_t lds = (size_t)kWaves * (260 * 4 + 2 * 256 * 4 + kRecCap * 16);
            const int64_t wgs = ((int64_t)Q.nmb + kWaves - 1) / kWaves;
            const int sgrid = (int)(wgs < 2048 ? (wgs > 0 ? wgs : 1) : 2048);
            if (mode == kStrTable)
                hipLaunchKernelGGL(frag_filter_str<kStrTable>, dim3(sgrid), dim3(kBlock), lds, s, d_q, fb.str_col[c], p,
                                   fb.str_off[c], fb.flags, p == 0 ? 1 : 0);
            else if (mode == kStrShifted)
                hipLaunchKernelGGL(frag_filter_str<kStrShifted>, dim3(sgrid), dim3(kBlock), lds, s, d_q, fb.str_col[c], p,
                                   fb.str_off[c], fb.flags, p == 0 ? 1 : 0);
            else
                hipLaunchKernelGGL(frag_filter_str<kStrMasked>, dim3(sgrid), dim3(kBlock), lds, s, d_q, fb.str_col[c], p,
                                   fb.str_off[c], fb.flags, p == 0 ? 1 : 0);
        } else
            hipLaunchKernelGGL(frag_filter_int, dim3(grid), dim3(256), 0, s, d_q, p, fb.dec[c], fb.flags,
                               p == 0 ? 1 : 0);
        if (!chk()) return -1;
    }
    if (Q.npreds > 0)
        hipLaunchKernelGGL(frag_compact, dim3(grid), dim3(kBlock), 0, s, d_q, fb.flags, fb.rows[0], &fb.counts[0]);
    else
        hipLaunchKernelGGL(frag_iota, dim3(grid), dim3(256), 0, s, d_q, fb.rows[0], &fb.counts[0]);
    if (!chk()) return -1;
    // 3) one probe kernel per dimension
    int src = 0, npay = 0;
    for (int j = 0; j < Q.nprobes; ++j) {
        hipLaunchKernelGGL(frag_probe, dim3(grid), dim3(kBlock), 0, s, d_q, j, fb.dec[Q.probes[j].fk_col],
                           fb.rows[src], &fb.counts[j], fb.rows[1 - src], &fb.counts[j + 1], fb, src, npay);
        if (!chk()) return -1;
        npay += Q.probes[j].h.npay;
        src = 1 - src;
    }
    // 4) aggregation and 5) result emission
    hipLaunchKernelGGL(frag_aggregate, dim3(grid), dim3(kBlock), 0, s, d_q, fb.rows[src], &fb.counts[Q.nprobes],
                       fb, src);
    if (!chk()) return -1;
    hipLaunchKernelGGL(frag_emit, dim3(1), dim3(kBlock), 0, s, d_q);
    if (!chk()) return -1;
    return launches;
}

}  // namespace dpf

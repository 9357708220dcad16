// kernels.hip -- gfx950 kernels of the data-path-fusion query library.
//
//  * fused_kernel: ONE persistent kernel per launch runs whole query
//    pipelines (paper Section 3.2 and Section 4.1 "Fused kernel
//    composition"): each workgroup claims (plan, mini-block range) work
//    items from a device queue, its four waves each take one 256-row mini
//    block at a time, decode the referenced columns straight from where the
//    chunks rest (HBM or pinned host memory mapped into the device), filter,
//    probe dimension hash tables (LDS copies for small ones), aggregate into
//    a per-workgroup LDS table, and the last workgroup to finish writes the
//    records to the host buffer -- nothing is materialised in between.
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

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t y = __shfl_up(x, (unsigned)d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, (unsigned)d, kWave);
        if (lane >= d) x += y;
    }
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

__device__ __forceinline__ uint64_t bits_at(const uint32_t* w, uint32_t bitpos, int b) {
    const uint32_t* p = w + (bitpos >> 5);
    uint32_t sh = bitpos & 31u;
    uint64_t x = *reinterpret_cast<const u64_a4*>(p) >> sh;
    if (b > 32) {
        uint64_t hi = p[2];
        if (sh) x |= hi << (64 - sh);
    }
    return b >= 64 ? x : (x & ((uint64_t(1) << b) - 1));
}

struct MbHdr {
    int64_t base;
    const uint32_t* w;
    int b;
    bool ok;
};

// Mini-block header with consistency checks (a corrupt header must not
// steer a load out of bounds).
__device__ __forceinline__ MbHdr mb_hdr(const DevCol& c, int m) {
    MbHdr h;
    uint32_t w0 = c.woff[m], w1 = c.woff[m + 1];
    uint32_t nw = w1 - w0;
    h.ok = (w0 <= w1) && (w1 <= c.nwords) && ((nw & 7u) == 0) && (nw <= 512u);
    h.b = (int)(nw >> 3);
    h.base = c.base[m];
    h.w = c.words + (h.ok ? w0 : 0);
    if (!h.ok) h.b = 0;
    return h;
}

// Dense decode of the wave's four rows (64k + lane) of mini block m.
// DICT columns yield codes; VARLEN yields lengths.  Returns false on a
// corrupt header.
__device__ __forceinline__ bool decode_dense(const DevCol& c, int m, int lane, int64_t v[4]) {
    MbHdr h = mb_hdr(c, m);
    uint64_t u[4];
    if (h.b == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = 0;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = bits_at(h.w, (uint32_t)(64 * k + lane) * (uint32_t)h.b, h.b);
    }
    if (c.enc == ENC_DELTA) {
        // value_i = anchor + i * dmin + sum_{j <= i} packed_j  (packed_0 = 0)
        uint64_t dmin = (uint64_t)c.dmin[m];
        uint64_t carry = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint64_t s = h.b ? wave_incl_scan_u64(u[k], lane) : 0;
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

// Value of row i of mini block m (random access).  DELTA sums the packed
// differences up to i.
__device__ __forceinline__ int64_t decode_at(const DevCol& c, int m, int i, bool& ok) {
    MbHdr h = mb_hdr(c, m);
    ok = ok && h.ok;
    if (c.enc == ENC_DELTA) {
        uint64_t s = 0;
        if (h.b)
            for (int j = 1; j <= i; ++j) s += bits_at(h.w, (uint32_t)j * (uint32_t)h.b, h.b);
        return (int64_t)((uint64_t)h.base + (uint64_t)i * (uint64_t)c.dmin[m] + s);
    }
    uint64_t u = h.b ? bits_at(h.w, (uint32_t)i * (uint32_t)h.b, h.b) : 0;
    return (int64_t)((uint64_t)h.base + u);
}

// DICT code -> value (bounds-checked).
__device__ __forceinline__ int64_t dict_value(const DevCol& c, int64_t code, bool& ok) {
    if (code < 0 || code >= c.ndict) { ok = false; return 0; }
    return c.dict[code];
}

// ---------------------------------------------------------------------------
// Integer predicates on four dense values -> 4-bit mask
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t eval_int_pred(const DevPred& p, const int64_t* in_vals,
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
// mini block, byte-parallel on an LDS copy of the mini block's heap.
//
// Each lane scans 4-byte words of the staged heap and flags every position
// where the first two bytes of a word match (a SWAR zero-byte test); flagged
// positions are verified, mapped to their row by binary search over the row
// offsets, and recorded as the row's leftmost s1 start and rightmost s2
// start.  A row matches iff rightmost_s2 >= leftmost_s1 + |s1|.
// ---------------------------------------------------------------------------
struct StrLds {
    uint32_t* offs;    // [257] row start offsets within the mini block's heap
    uint32_t* first1;  // [256] leftmost s1 start (0xffffffff: none)
    uint32_t* last2;   // [256] rightmost s2 start + 1 (0: none)
    uint32_t* heapw;   // staged heap words
};

__device__ __forceinline__ uint32_t zero_byte_flags(uint32_t z) {
    return ~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;
}

__device__ __forceinline__ uint32_t rep4(uint8_t c) { return 0x01010101u * c; }

__device__ __forceinline__ bool str_eq_lds(const uint8_t* hb, uint32_t q, const uint8_t* w, int n) {
    for (int i = 2; i < n; ++i)
        if (hb[q + i] != w[i]) return false;
    return true;
}

__device__ __forceinline__ int row_of(const uint32_t* offs, uint32_t p) {
    int lo = 0, hi = 255;  // largest r with offs[r] <= p
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ bool contains_seq_global(const uint8_t* s, uint32_t n, const DevPred& p) {
    uint32_t n1 = p.n1, n2 = p.n2;
    if (n < n1) return false;
    for (uint32_t a = 0; a + n1 <= n; ++a) {
        bool e = true;
        for (uint32_t i = 0; i < n1 && e; ++i) e = s[a + i] == p.s1[i];
        if (!e) continue;
        for (uint32_t b = a + n1; b + n2 <= n; ++b) {
            bool f = true;
            for (uint32_t i = 0; i < n2 && f; ++i) f = s[b + i] == p.s2[i];
            if (f) return true;
        }
        return false;  // the leftmost s1 leaves the most room for s2
    }
    return false;
}

// Returns the 4-bit match mask of the lane's rows; clears ok on corruption.
__device__ uint32_t eval_str_pred(const DevCol& c, const DevPred& p, int m, int lane, int nvalid,
                                  const StrLds& L, bool& ok) {
    MbHdr h = mb_hdr(c, m);
    uint64_t h0 = c.hoff[m], h1 = c.hoff[m + 1];
    bool hok = h.ok && h0 <= h1 && h1 <= c.heap_bytes && (h1 - h0) < (uint64_t(1) << 31);
    if (!hok) { ok = false; return 0; }
    uint32_t len[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int i = 64 * k + lane;
        uint32_t u = h.b ? (uint32_t)bits_at(h.w, (uint32_t)i * (uint32_t)h.b, h.b) : 0u;
        len[k] = i < nvalid ? (uint32_t)h.base + u : 0u;
    }
    uint32_t carry = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t s = wave_incl_scan_u32(len[k], lane);
        L.offs[64 * k + lane] = carry + s - len[k];
        carry += __builtin_amdgcn_readlane(s, 63);
    }
    const uint32_t total = carry;
    if (lane == 0) L.offs[256] = total;
    if ((uint64_t)total != h1 - h0) { ok = false; return 0; }

    uint32_t res = 0;
    if (total + 8u > (uint32_t)kStrHeapCap) {
        // Mini block too large for the staging area: lane-per-row scan of
        // the bytes where they rest.
        wave_lds_sync();
        for (int k = 0; k < 4; ++k) {
            int i = 64 * k + lane;
            if (i < nvalid) {
                uint32_t o = L.offs[i];
                res |= (uint32_t)contains_seq_global(c.heap + h0 + o, L.offs[i + 1] - o, p) << k;
            }
        }
        return res;
    }

    // Stage the heap bytes [h0, h1) into LDS as whole words (plus one spare
    // word so every position can read its successor).
    const uint32_t s0 = (uint32_t)(h0 & 3u);
    const uint32_t* g = reinterpret_cast<const uint32_t*>(c.heap) + (h0 >> 2);
    const uint32_t nw = (s0 + total + 3u) >> 2;
    for (uint32_t j = lane; j <= nw; j += kWave) L.heapw[j] = g[j];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        L.first1[64 * k + lane] = 0xFFFFFFFFu;
        L.last2[64 * k + lane] = 0u;
    }
    wave_lds_sync();

    const uint32_t a1 = rep4(p.s1[0]), a2 = rep4(p.s2[0]);
    const uint32_t b1 = rep4(p.n1 > 1 ? p.s1[1] : 0), b2 = rep4(p.n2 > 1 ? p.s2[1] : 0);
    const bool two1 = p.n1 > 1, two2 = p.n2 > 1;
    const uint8_t* hb = reinterpret_cast<const uint8_t*>(L.heapw);
    for (uint32_t j = lane; j < nw; j += kWave) {
        uint32_t w = L.heapw[j], nx = L.heapw[j + 1];
        uint32_t sh = __builtin_amdgcn_alignbit(nx, w, 8);  // bytes 1..4
        uint32_t z1 = (w ^ a1) | (two1 ? (sh ^ b1) : 0u);
        uint32_t z2 = (w ^ a2) | (two2 ? (sh ^ b2) : 0u);
        uint32_t f1 = zero_byte_flags(z1), f2 = zero_byte_flags(z2);
        if ((f1 | f2) == 0u) continue;
        for (int t = 0; t < 4; ++t) {
            uint32_t bit = 0x80u << (8 * t);
            if (!((f1 | f2) & bit)) continue;
            uint32_t q = 4 * j + t;
            if (q < s0 || q - s0 >= total) continue;
            uint32_t pos = q - s0;
            int r = row_of(L.offs, pos);
            uint32_t rend = L.offs[r + 1];
            if ((f1 & bit) && pos + p.n1 <= rend && str_eq_lds(hb, q, p.s1, p.n1))
                atomicMin(&L.first1[r], pos);
            if ((f2 & bit) && pos + p.n2 <= rend && str_eq_lds(hb, q, p.s2, p.n2))
                atomicMax(&L.last2[r], pos + 1);
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int i = 64 * k + lane;
        uint32_t f = L.first1[i], e = L.last2[i];
        bool hit = i < nvalid && f != 0xFFFFFFFFu && e != 0u && (uint64_t)(e - 1) >= (uint64_t)f + p.n1;
        res |= (uint32_t)hit << k;
    }
    return res;
}

// ---------------------------------------------------------------------------
// Value slots carried by a surviving row (uniform slot ids -> registers)
// ---------------------------------------------------------------------------
struct Slots {
    int64_t v[kMaxSlots];
};

__device__ __forceinline__ void set_slot(Slots& s, int id, int64_t x) {
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i)
        if (i == id) s.v[i] = x;
}

__device__ __forceinline__ int64_t get_slot(const Slots& s, int id) {
    int64_t x = 0;
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i)
        if (i == id) x = s.v[i];
    return x;
}

__device__ __forceinline__ uint32_t hash32(int32_t key, int log2cap) {
    return log2cap ? ((uint32_t)key * 0x9E3779B1u) >> (32 - log2cap) : 0u;
}

// Linear-probing lookup; returns the slot or -1.
template <bool kLds>
__device__ __forceinline__ int hash_find(const DevHash& h, const uint8_t* smem_shared, int64_t key) {
    if (key < INT32_MIN || key > INT32_MAX || key == kEmptyKey) return -1;
    const int32_t k = (int32_t)key;
    const int32_t* keys = kLds ? reinterpret_cast<const int32_t*>(smem_shared + h.lds_off) : h.keys;
    uint32_t s = hash32(k, h.log2cap);
    for (uint32_t n = 0; n <= h.cap_mask; ++n) {
        int32_t x = keys[s];
        if (x == k) return (int)s;
        if (x == kEmptyKey) return -1;
        s = (s + 1) & h.cap_mask;
    }
    return -1;
}

template <bool kLds>
__device__ __forceinline__ int64_t hash_payload(const DevHash& h, const uint8_t* smem_shared, int k,
                                                int slot) {
    const uint8_t* base;
    if (kLds) {
        // payload arrays follow the keys at the same relative offsets
        base = smem_shared + h.lds_off +
               ((const uint8_t*)h.pay[k] - (const uint8_t*)h.keys);
    } else {
        base = (const uint8_t*)h.pay[k];
    }
    return h.pay64[k] ? reinterpret_cast<const int64_t*>(base)[slot]
                      : (int64_t)reinterpret_cast<const int32_t*>(base)[slot];
}

// ---------------------------------------------------------------------------
// Aggregation of one surviving row into the (LDS or global) group table
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool group_index(const DevQuery& Q, const Slots& sv, int64_t& g) {
    g = 0;
    for (int k = 0; k < Q.nkeys; ++k) {
        const DevKey& K = Q.keys[k];
        int64_t d = get_slot(sv, K.slot) - K.min;
        if (d < 0 || d >= K.card) return false;
        g += d * K.stride;
    }
    return true;
}

__device__ __forceinline__ int64_t acc_value(const DevAcc& A, const Slots& sv) {
    int64_t prod = 1;
    for (int t = 0; t < A.nterms; ++t) {
        const DevTerm& T = A.t[t];
        int64_t x = T.slot >= 0 ? T.mul * get_slot(sv, T.slot) + T.add : T.add;
        prod *= x;
    }
    return prod;
}

__device__ __forceinline__ void aggregate_row(const DevQuery& Q, uint8_t* smem_shared, const Slots& sv,
                                              int64_t g) {
    const int nacc = Q.nacc;
    if (Q.agg_lds) {
        unsigned long long* T = reinterpret_cast<unsigned long long*>(smem_shared + Q.agg_lds_off) + g * nacc;
        atomicAdd(&T[0], 1ull);
        for (int a = 1; a < nacc; ++a) atomicAdd(&T[a], (unsigned long long)acc_value(Q.accs[a], sv));
    } else {
        unsigned long long* T = reinterpret_cast<unsigned long long*>(Q.agg) + g * nacc;
        atomicAdd(&T[0], 1ull);
        for (int a = 1; a < nacc; ++a) atomicAdd(&T[a], (unsigned long long)acc_value(Q.accs[a], sv));
    }
}

// ---------------------------------------------------------------------------
// Stage B: probes, value loads and aggregation for one row (lane-local)
// ---------------------------------------------------------------------------
template <bool kLdsAny>
__device__ __forceinline__ void process_row(const DevQuery& Q, uint8_t* smem_shared, int m, int i,
                                            bool active, bool& ok_hdr) {
    bool ok = active;
    Slots sv;
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) sv.v[s] = 0;
    const int nprobes = Q.nprobes;
    for (int j = 0; j < nprobes; ++j) {
        if (__ballot(ok) == 0) return;
        const DevProbe& P = Q.probes[j];
        if (ok) {
            int64_t fk = decode_at(Q.cols[P.fk_col], m, i, ok_hdr);
            const DevCol& fc = Q.cols[P.fk_col];
            if (fc.enc == ENC_DICT) fk = dict_value(fc, fk, ok_hdr);
            int slot = (kLdsAny && P.h.lds_off >= 0) ? hash_find<true>(P.h, smem_shared, fk)
                                                     : hash_find<false>(P.h, smem_shared, fk);
            ok = slot >= 0;
            if (ok) {
                for (int k = 0; k < P.h.npay; ++k) {
                    if (P.pay_slot[k] < 0) continue;
                    int64_t pv = (kLdsAny && P.h.lds_off >= 0) ? hash_payload<true>(P.h, smem_shared, k, slot)
                                                               : hash_payload<false>(P.h, smem_shared, k, slot);
                    set_slot(sv, P.pay_slot[k], pv);
                }
            }
        }
    }
    if (!ok) return;
    for (int l = 0; l < Q.nloads; ++l) {
        const DevLoad& Ld = Q.loads[l];
        const DevCol& lc = Q.cols[Ld.col];
        int64_t x = decode_at(lc, m, i, ok_hdr);
        if (Ld.dict_val) x = dict_value(lc, x, ok_hdr);
        set_slot(sv, Ld.slot, x);
    }
    int64_t g;
    if (!group_index(Q, sv, g)) { ok_hdr = false; return; }
    aggregate_row(Q, smem_shared, sv, g);
}

// ---------------------------------------------------------------------------
// One mini block of one plan, by one wave
// ---------------------------------------------------------------------------
template <bool kLdsAny>
__device__ void process_tile(const DevQuery& Q, uint8_t* smem_shared, uint8_t* wave_area, bool str_stage,
                             int m, int lane, bool& ok_hdr) {
    const int64_t row0 = (int64_t)m * kMB;
    const int nvalid = (int)min((int64_t)kMB, Q.nrows - row0);
    uint16_t* rows = reinterpret_cast<uint16_t*>(wave_area);
    const int npreds = Q.npreds;

    if (npreds == 0) {
        // No fact predicate: every valid row goes to the probe/aggregate stage.
        for (int k = 0; k < 4; ++k) {
            int i = 64 * k + lane;
            if (64 * k >= nvalid) break;
            process_row<kLdsAny>(Q, smem_shared, m, i, i < nvalid, ok_hdr);
        }
        return;
    }

    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(64 * k + lane < nvalid) << k;

    int64_t v[4];
    int last_col = -1;
    for (int a = 0; a < npreds; ++a) {
        const DevPred& P = Q.preds[a];
        if (P.kind == PK_STR) {
            if (!str_stage) { ok_hdr = false; return; }
            StrLds L;
            L.offs = reinterpret_cast<uint32_t*>(wave_area + 512);
            L.first1 = L.offs + 260;
            L.last2 = L.first1 + 256;
            L.heapw = L.last2 + 256;
            mask &= eval_str_pred(Q.cols[P.col], P, m, lane, nvalid, L, ok_hdr);
        } else {
            if (P.col != last_col) {
                ok_hdr &= decode_dense(Q.cols[P.col], m, lane, v);
                last_col = P.col;
            }
            mask &= eval_int_pred(P, Q.in_vals, v);
        }
        if (__ballot(mask != 0) == 0) return;  // no survivor in this mini block
    }

    // Compact survivors (wave ballot + mbcnt) into the wave's row list.
    uint32_t nsurv = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool bit = (mask >> k) & 1u;
        uint64_t b = __ballot(bit);
        if (bit) rows[nsurv + bits_below(b)] = (uint16_t)(64 * k + lane);
        nsurv += (uint32_t)__popcll(b);
    }
    wave_lds_sync();
    for (uint32_t base = 0; base < nsurv; base += kWave) {
        uint32_t idx = base + lane;
        bool act = idx < nsurv;
        int i = act ? rows[idx] : 0;
        process_row<kLdsAny>(Q, smem_shared, m, i, act, ok_hdr);
    }
    wave_lds_sync();
}

__device__ __forceinline__ size_t wave_area_bytes(bool str_stage) {
    return 512 + (str_stage ? (1040 + 1024 + 1024 + kStrHeapCap + 64) : 0);
}

// Merge the workgroup's LDS group table into the plan's global table.
__device__ void flush_lds_agg(const DevQuery& Q, uint8_t* smem_shared) {
    if (!Q.agg_lds) return;
    const int64_t n = Q.ngroups * Q.nacc;
    unsigned long long* T = reinterpret_cast<unsigned long long*>(smem_shared + Q.agg_lds_off);
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        unsigned long long x = T[e];
        if (x) atomicAdd(reinterpret_cast<unsigned long long*>(Q.agg) + e, x);
        T[e] = 0;
    }
}

// Load a plan's LDS-resident dimension tables and clear its LDS group table.
__device__ void load_lds_state(const DevQuery& Q, uint8_t* smem_shared) {
    for (int j = 0; j < Q.nprobes; ++j) {
        const DevHash& h = Q.probes[j].h;
        if (h.lds_off < 0) continue;
        const uint4* src = reinterpret_cast<const uint4*>(h.keys);
        uint4* dst = reinterpret_cast<uint4*>(smem_shared + h.lds_off);
        for (uint32_t e = threadIdx.x; e < h.bytes / 16u; e += blockDim.x) dst[e] = src[e];
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
// format and returned to the host), then clear the device table for the next
// execution.  Run by one workgroup after every other one has finished.
__device__ void emit_records(const DevQuery& Q, int32_t* ctrl) {
    const int nacc = Q.nacc;
    const int64_t G = Q.ngroups;
    unsigned long long* T = reinterpret_cast<unsigned long long*>(Q.agg);
    if (threadIdx.x == 0) ctrl[2] = 0;
    __syncthreads();
    for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
        unsigned long long cnt = ld_acq(&T[g * nacc]);
        if (cnt == 0) continue;
        int pos = atomicAdd(&ctrl[2], 1);
        int64_t* rec = Q.host_out + 2 + (int64_t)pos * (1 + nacc);
        rec[0] = g;
        rec[1] = (int64_t)cnt;
        T[g * nacc] = 0;
        for (int a = 1; a < nacc; ++a) {
            rec[1 + a] = (int64_t)ld_acq(&T[g * nacc + a]);
            T[g * nacc + a] = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t st = __hip_atomic_exchange(Q.status, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.host_out[0] = (int64_t)st;
        Q.host_out[1] = (int64_t)ctrl[2];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The persistent fused kernel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void fused_kernel(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    int32_t* ctrl = reinterpret_cast<int32_t*>(smem);
    uint8_t* shared_area = smem + 64;
    const bool str_stage = a.str_stage != 0;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint8_t* wave_area = smem + 64 + a.lds_shared + (size_t)wave * wave_area_bytes(str_stage);
    const int total_items = a.item_start[a.nq];

    int cur = -1;
    bool ok_hdr = true;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) ctrl[0] = (int32_t)atomicAdd(&a.counters[0], 1u);
        __syncthreads();
        const int item = uniform_i32(ctrl[0]);
        if (item >= total_items) break;
        int qi = 0;
        while (qi + 1 < a.nq && a.item_start[qi + 1] <= item) ++qi;
        qi = uniform_i32(qi);
        const DevQuery& Q = *a.q[qi];
        if (qi != cur) {
            if (cur >= 0) {
                __syncthreads();
                flush_lds_agg(*a.q[cur], shared_area);
                if (!ok_hdr) atomicOr(a.q[cur]->status, ST_CORRUPT);
                ok_hdr = true;
            }
            __syncthreads();
            load_lds_state(Q, shared_area);
            __syncthreads();
            cur = qi;
        }
        const int mb0 = (item - a.item_start[qi]) * a.mb_per_item;
        const int mb1 = min(mb0 + a.mb_per_item, Q.nmb);
        const bool lds_any = Q.lds_shared > 0;
        for (int m = mb0 + wave; m < mb1; m += kWaves) {
            if (lds_any) process_tile<true>(Q, shared_area, wave_area, str_stage, m, lane, ok_hdr);
            else process_tile<false>(Q, shared_area, wave_area, str_stage, m, lane, ok_hdr);
        }
    }
    if (cur >= 0) {
        __syncthreads();
        flush_lds_agg(*a.q[cur], shared_area);
        if (!ok_hdr) atomicOr(a.q[cur]->status, ST_CORRUPT);
    }
    // Last workgroup out emits every plan's records and resets the queue.
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) ctrl[1] = (int32_t)atomicAdd(&a.counters[1], 1u);
    __syncthreads();
    if ((uint32_t)ctrl[1] != gridDim.x - 1) return;
    __threadfence();
    for (int qi = 0; qi < a.nq; ++qi) emit_records(*a.q[qi], ctrl);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&a.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence_system();
}

// ---------------------------------------------------------------------------
// Hash build (dimension scan -> filter -> insert)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hash_tile_mask(const HashBuildArgs& A, int m, int lane, int nvalid,
                                                   int64_t key[4], int64_t pay[2][4], bool& ok) {
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mask |= (uint32_t)(64 * k + lane < nvalid) << k;
    int64_t v[4];
    for (int p = 0; p < A.npreds; ++p) {
        const DevPred& P = A.preds[p];
        ok &= decode_dense(A.cols[P.col], m, lane, v);
        mask &= eval_int_pred(P, A.in_vals, v);
    }
    const DevCol& kc = A.cols[A.key_col];
    ok &= decode_dense(kc, m, lane, key);
    if (kc.enc == ENC_DICT)
        for (int k = 0; k < 4; ++k) key[k] = dict_value(kc, key[k], ok);
    for (int j = 0; j < A.npay; ++j) {
        const DevCol& pc = A.cols[A.pay_col[j]];
        ok &= decode_dense(pc, m, lane, pay[j]);
        if (pc.enc == ENC_DICT)
            for (int k = 0; k < 4; ++k) pay[j][k] = dict_value(pc, pay[j][k], ok);
    }
    return mask;
}

__global__ __launch_bounds__(kBlock) void hash_count_kernel(const HashBuildArgs* __restrict__ args) {
    const HashBuildArgs& A = *args;
    const int lane = lane_id();
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    unsigned long long cnt = 0;
    long long mn[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, mx[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int m = gw; m < A.nmb; m += nw) {
        const int nvalid = (int)min((int64_t)kMB, A.nrows - (int64_t)m * kMB);
        int64_t key[4], pay[2][4];
        uint32_t mask = hash_tile_mask(A, m, lane, nvalid, key, pay, ok);
        for (int k = 0; k < 4; ++k) {
            if (!((mask >> k) & 1u)) continue;
            cnt += 1;
            mn[0] = min(mn[0], (long long)key[k]);
            mx[0] = max(mx[0], (long long)key[k]);
            for (int j = 0; j < A.npay; ++j) {
                mn[1 + j] = min(mn[1 + j], (long long)pay[j][k]);
                mx[1 + j] = max(mx[1 + j], (long long)pay[j][k]);
            }
        }
    }
    if (cnt) {
        atomicAdd(A.count, cnt);
        for (int j = 0; j < 1 + A.npay; ++j) {
            atomicMin(&A.mm[2 * j], mn[j]);
            atomicMax(&A.mm[2 * j + 1], mx[j]);
        }
    }
    if (!ok) atomicOr(A.status, ST_CORRUPT);
}

__global__ __launch_bounds__(kBlock) void hash_insert_kernel(const HashBuildArgs* __restrict__ args) {
    const HashBuildArgs& A = *args;
    const int lane = lane_id();
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
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

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Fragmented execution: one kernel per step, intermediates in HBM
// ---------------------------------------------------------------------------
// Decode one integer column to int64 (codes for DICT).
__global__ __launch_bounds__(kBlock) void frag_decode_int(const DevQuery* __restrict__ q, int c, int64_t* out) {
    const DevQuery& Q = *q;
    const DevCol& C = Q.cols[c];
    const int lane = lane_id();
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
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
    const DevQuery& Q = *q;
    const DevCol& C = Q.cols[c];
    const int lane = lane_id();
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    bool ok = true;
    for (int m = gw; m < Q.nmb; m += nw) {
        const int nvalid = (int)min((int64_t)kMB, Q.nrows - (int64_t)m * kMB);
        MbHdr h = mb_hdr(C, m);
        ok &= h.ok;
        uint64_t h0 = C.hoff[m], h1 = C.hoff[m + 1];
        if (!(h0 <= h1 && h1 <= C.heap_bytes)) { ok = false; continue; }
        uint64_t carry = h0;
        for (int k = 0; k < 4; ++k) {
            int i = 64 * k + lane;
            uint64_t len = (i < nvalid) ? (uint64_t)h.base + (h.b ? bits_at(h.w, (uint32_t)i * h.b, h.b) : 0) : 0;
            uint64_t s = wave_incl_scan_u64(len, lane);
            if (i < nvalid) off[(int64_t)m * kMB + i] = (int64_t)(carry + s - len);
            carry += readlane_u64(s, 63);
        }
        if (carry != h1) ok = false;
        for (uint64_t b = h0 + lane; b < h1; b += kWave) bytes[b] = C.heap[b];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[Q.nrows] = (int64_t)Q.cols[c].heap_bytes;
    if (!ok) atomicOr(Q.status, ST_CORRUPT);
}

__global__ void frag_filter_int(const DevQuery* __restrict__ q, int pi, const int64_t* vals, uint8_t* flags,
                                int first) {
    const DevQuery& Q = *q;
    const DevPred& P = Q.preds[pi];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q.nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t v4[4] = {vals[r], 0, 0, 0};
        bool t = eval_int_pred(P, Q.in_vals, v4) & 1u;
        flags[r] = (uint8_t)((first ? 1 : flags[r]) & t);
    }
}

__global__ void frag_filter_str(const DevQuery* __restrict__ q, int pi, const int64_t* off, const uint8_t* bytes,
                                uint8_t* flags, int first) {
    const DevQuery& Q = *q;
    const DevPred& P = Q.preds[pi];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q.nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        bool prev = first ? true : flags[r] != 0;
        bool t = prev && contains_seq_global(bytes + off[r], (uint32_t)(off[r + 1] - off[r]), P);
        flags[r] = (uint8_t)t;
    }
}

// flags -> row list (order not preserved; aggregation is order-free)
__global__ __launch_bounds__(kBlock) void frag_compact(const DevQuery* __restrict__ q, const uint8_t* flags,
                                                       int32_t* rows, unsigned long long* count) {
    const DevQuery& Q = *q;
    const int lane = lane_id();
    for (int64_t b0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) & ~63ll; b0 < Q.nrows;
         b0 += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = b0 + lane;
        bool f = r < Q.nrows && flags[r];
        uint64_t bal = __ballot(f);
        unsigned long long base = 0;
        if (lane == 0 && bal) base = atomicAdd(count, (unsigned long long)__popcll(bal));
        base = __shfl(base, 0, kWave);
        if (f) rows[base + bits_below(bal)] = (int32_t)r;
    }
}

// all rows -> row list (plans without a fact predicate)
__global__ void frag_iota(const DevQuery* __restrict__ q, int32_t* rows, unsigned long long* count) {
    const DevQuery& Q = *q;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q.nrows;
         r += (int64_t)gridDim.x * blockDim.x)
        rows[r] = (int32_t)r;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = (unsigned long long)Q.nrows;
}

// Probe j: keep listed rows whose key is found; carry the earlier payload
// arrays along and append this probe's payloads.
__global__ __launch_bounds__(kBlock) void frag_probe(const DevQuery* __restrict__ q, int j, const int64_t* fkvals,
                                                     const int32_t* rin, const unsigned long long* nin,
                                                     int32_t* rout, unsigned long long* nout,
                                                     const FragBuffers fb, int src, int npay_before) {
    const DevQuery& Q = *q;
    const DevProbe& P = Q.probes[j];
    const int lane = lane_id();
    const int64_t n = (int64_t)*nin;
    for (int64_t b0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) & ~63ll; b0 < n;
         b0 += (int64_t)gridDim.x * blockDim.x) {
        int64_t e = b0 + lane;
        bool act = e < n;
        int slot = -1;
        int32_t r = act ? rin[e] : 0;
        if (act) {
            int64_t fk = fkvals[r];
            const DevCol& fc = Q.cols[P.fk_col];
            bool okd = true;
            if (fc.enc == ENC_DICT) fk = dict_value(fc, fk, okd);
            slot = hash_find<false>(P.h, nullptr, fk);
        }
        bool keep = slot >= 0;
        uint64_t bal = __ballot(keep);
        unsigned long long base = 0;
        if (lane == 0 && bal) base = atomicAdd(nout, (unsigned long long)__popcll(bal));
        base = __shfl(base, 0, kWave);
        if (keep) {
            unsigned long long o = base + bits_below(bal);
            rout[o] = r;
            for (int t = 0; t < npay_before; ++t) fb.pay[1 - src][t][o] = fb.pay[src][t][e];
            for (int k = 0; k < P.h.npay; ++k)
                fb.pay[1 - src][npay_before + k][o] = hash_payload<false>(P.h, nullptr, k, slot);
        }
    }
}

// Aggregate the final row list: fact values gathered from the decoded
// columns, payloads from the aligned arrays.
__global__ __launch_bounds__(kBlock) void frag_aggregate(const DevQuery* __restrict__ q, const int32_t* rows,
                                                         const unsigned long long* nrows_list, const FragBuffers fb,
                                                         int src) {
    const DevQuery& Q = *q;
    const int64_t n = (int64_t)*nrows_list;
    bool okall = true;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = rows[e];
        Slots sv;
        for (int s = 0; s < kMaxSlots; ++s) sv.v[s] = 0;
        int pidx = 0;
        for (int j = 0; j < Q.nprobes; ++j) {
            for (int k = 0; k < Q.probes[j].h.npay; ++k) {
                int sl = Q.probes[j].pay_slot[k];
                if (sl >= 0) set_slot(sv, sl, fb.pay[src][pidx][e]);
                ++pidx;
            }
        }
        for (int l = 0; l < Q.nloads; ++l) {
            const DevLoad& Ld = Q.loads[l];
            int64_t x = fb.dec[Ld.col][r];
            if (Ld.dict_val) x = dict_value(Q.cols[Ld.col], x, okall);
            set_slot(sv, Ld.slot, x);
        }
        int64_t g;
        if (!group_index(Q, sv, g)) { okall = false; continue; }
        unsigned long long* T = reinterpret_cast<unsigned long long*>(Q.agg) + g * Q.nacc;
        atomicAdd(&T[0], 1ull);
        for (int a = 1; a < Q.nacc; ++a) atomicAdd(&T[a], (unsigned long long)acc_value(Q.accs[a], sv));
    }
    if (!okall) atomicOr(Q.status, ST_CORRUPT);
}

__global__ __launch_bounds__(kBlock) void frag_emit(const DevQuery* __restrict__ q) {
    __shared__ int32_t ctrl[4];
    __threadfence();
    emit_records(*q, ctrl);
    __threadfence_system();
}

__global__ void frag_reset_counts(unsigned long long* c, int n) {
    if (threadIdx.x < n) c[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_fused(const BatchArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    hipLaunchKernelGGL(fused_kernel, dim3(grid), dim3(kBlock), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_hash_count(const HashBuildArgs* d_args, int grid, hipStream_t s) {
    hipLaunchKernelGGL(hash_count_kernel, dim3(grid), dim3(kBlock), 0, s, d_args);
    return hipGetLastError();
}

hipError_t launch_hash_insert(const HashBuildArgs* d_args, int grid, hipStream_t s) {
    hipLaunchKernelGGL(hash_insert_kernel, dim3(grid), dim3(kBlock), 0, s, d_args);
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
        } else {
            hipLaunchKernelGGL(frag_decode_int, dim3(grid), dim3(kBlock), 0, s, d_q, c, fb.dec[c]);
        }
        if (!chk()) return -1;
    }
    // 2) one filter kernel per predicate, then compaction to a row list
    for (int p = 0; p < Q.npreds; ++p) {
        const int c = Q.preds[p].col;
        if (Q.preds[p].kind == PK_STR)
            hipLaunchKernelGGL(frag_filter_str, dim3(grid), dim3(256), 0, s, d_q, p, fb.str_off[c],
                               fb.str_bytes[c], fb.flags, p == 0 ? 1 : 0);
        else
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

// encode.cpp -- host-side type-specific compression (paper Section 3.4 and
// the loader of Section 4.2), written for the gfx950 kernels' access pattern:
//
//  * every column is cut into mini blocks of 256 values; row r of the table
//    is value r % 256 of global mini block r / 256 (chunk sizes are
//    multiples of 256, so all columns of a table share mini-block
//    boundaries and any mini block decodes on its own);
//  * a mini block stores its values LSB-first at bit i * width in 32-bit
//    words, so 256 values always fill whole words (8 * width of them) and a
//    wave reads a contiguous run of bits per load instruction;
//  * headers live in separate arrays (base, word offset, ...) rather than
//    inline, so the kernel fetches them with scalar loads.
#include "encode.h"

#include <algorithm>
#include <cstring>
#include <thread>

#include "fsst.h"

namespace dpf {
namespace {

constexpr int kMB = 256;
constexpr int64_t kMaxDict = 1 << 16;

inline int bit_width(uint64_t r) { return r ? 64 - __builtin_clzll(r) : 0; }

template <class F>
void parallel_for(int64_t n, int threads, F f) {
    if (n <= 0) return;
    if (threads <= 1 || n < 64) {
        f((int64_t)0, n);
        return;
    }
    int t = (int)std::min<int64_t>(threads, n);
    std::vector<std::thread> pool;
    int64_t step = (n + t - 1) / t;
    for (int k = 0; k < t; ++k) {
        int64_t a = k * step, b = std::min(n, a + step);
        if (a >= b) break;
        pool.emplace_back([=, &f] { f(a, b); });
    }
    for (auto& th : pool) th.join();
}

void pack(const uint64_t* u, int n, int b, uint32_t* w) {
    if (b == 0) return;
    for (int i = 0; i < n; ++i) {
        uint64_t pos = (uint64_t)i * (uint64_t)b;
        uint32_t* p = w + (pos >> 5);
        int sh = (int)(pos & 31);
        unsigned __int128 x = (unsigned __int128)u[i] << sh;
        p[0] |= (uint32_t)x;
        if (sh + b > 32) p[1] |= (uint32_t)(x >> 32);
        if (sh + b > 64) p[2] |= (uint32_t)(x >> 64);
    }
}

inline uint64_t unpack(const uint32_t* w, int i, int b) {
    if (b == 0) return 0;
    uint64_t pos = (uint64_t)i * (uint64_t)b;
    const uint32_t* p = w + (pos >> 5);
    int sh = (int)(pos & 31);
    unsigned __int128 x = (unsigned __int128)p[0] | ((unsigned __int128)p[1] << 32) |
                          ((unsigned __int128)p[2] << 64);
    uint64_t v = (uint64_t)(x >> sh);
    return b >= 64 ? v : (v & ((uint64_t(1) << b) - 1));
}

// Frame of reference (or delta + frame of reference) of one mini block's
// integer stream x[0..n): fills u (n entries, pads stay 0), returns width.
int prepare_block(const int64_t* x, int n, bool delta, int64_t* base, int64_t* dmin, uint64_t* u) {
    if (n == 0) { *base = 0; if (dmin) *dmin = 0; return 0; }
    if (!delta) {
        int64_t mn = x[0];
        for (int i = 1; i < n; ++i) mn = std::min(mn, x[i]);
        uint64_t mx = 0;
        for (int i = 0; i < n; ++i) {
            u[i] = (uint64_t)x[i] - (uint64_t)mn;
            mx = std::max(mx, u[i]);
        }
        *base = mn;
        return bit_width(mx);
    }
    *base = x[0];
    int64_t dm = 0;
    for (int i = 1; i < n; ++i) {
        int64_t d = (int64_t)((uint64_t)x[i] - (uint64_t)x[i - 1]);
        dm = (i == 1) ? d : std::min(dm, d);
    }
    *dmin = dm;
    uint64_t mx = 0;
    u[0] = 0;
    for (int i = 1; i < n; ++i) {
        u[i] = (uint64_t)x[i] - (uint64_t)x[i - 1] - (uint64_t)dm;
        mx = std::max(mx, u[i]);
    }
    return bit_width(mx);
}

}  // namespace

int64_t compressed_bytes(const HostColumn& c) {
    int64_t b = c.nmb * 8 + (c.nmb + 1) * 4 + (int64_t)c.nwords * 4;
    if (c.enc == DPF_ENC_DELTA) b += c.nmb * 8;
    if (c.enc == DPF_ENC_VARLEN) b += (c.nmb + 1) * 8 + (int64_t)c.heap_bytes;
    if (c.enc == DPF_ENC_FSST) b += (c.nmb + 1) * 8 + (int64_t)c.heap_bytes + c.nchunks * (int64_t)kFsstTableBytes;
    if (c.enc == DPF_ENC_DICT) b += (int64_t)c.dict.size() * 8;
    return b;
}

ColView view_of(const HostColumn& c) {
    ColView v;
    v.base = c.base.data();
    v.woff = c.woff.data();
    v.words = c.words.data();
    v.dmin = c.dmin.empty() ? nullptr : c.dmin.data();
    v.hoff = c.hoff.empty() ? nullptr : c.hoff.data();
    v.heap = c.heap.empty() ? nullptr : c.heap.data();
    v.dict = c.dict.empty() ? nullptr : c.dict.data();
    v.doff = c.doff.empty() ? nullptr : c.doff.data();
    v.symtab = c.symtab.empty() ? nullptr : c.symtab.data();
    return v;
}

dpf_status encode_column(const dpf_column_src& src, int32_t enc, int32_t chunk_rows, int32_t threads,
                         HostColumn* out, std::string* err) {
    const int64_t n = src.nrows;
    if (n < 0) { *err = "negative row count"; return DPF_ERR_INVALID_ARG; }
    if (chunk_rows == 0) chunk_rows = 65536;
    if (chunk_rows < kMB || chunk_rows % kMB != 0) {
        *err = "chunk_rows must be a positive multiple of 256";
        return DPF_ERR_INVALID_ARG;
    }
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = std::min(threads, 64);
    const bool is_str = src.type == DPF_TYPE_STR;
    if (!is_str && src.type != DPF_TYPE_I32 && src.type != DPF_TYPE_I64) {
        *err = "unknown column type";
        return DPF_ERR_INVALID_ARG;
    }
    if (n > 0 && ((is_str && (!src.str_offsets || !src.str_bytes)) || (!is_str && !src.values))) {
        *err = "missing source array";
        return DPF_ERR_INVALID_ARG;
    }
    if (is_str && !src.str_offsets) { *err = "missing offsets"; return DPF_ERR_INVALID_ARG; }
    const bool fsst = is_str && enc == DPF_ENC_FSST;
    if (is_str) {
        if (enc == DPF_ENC_AUTO) enc = DPF_ENC_VARLEN;
        if (enc != DPF_ENC_VARLEN && enc != DPF_ENC_FSST) {
            *err = "strings use VARLEN or FSST";
            return DPF_ERR_INVALID_ARG;
        }
        if (src.str_offsets[0] != 0) { *err = "string offsets must start at 0"; return DPF_ERR_INVALID_ARG; }
        for (int64_t i = 0; i < n; ++i)
            if (src.str_offsets[i + 1] < src.str_offsets[i]) {
                *err = "string offsets must be non-decreasing";
                return DPF_ERR_INVALID_ARG;
            }
    } else if (enc == DPF_ENC_VARLEN || enc == DPF_ENC_FSST) {
        *err = "VARLEN and FSST are for strings";
        return DPF_ERR_INVALID_ARG;
    }
    if (is_str && enc == DPF_ENC_PLAIN) { *err = "PLAIN is for integers"; return DPF_ERR_INVALID_ARG; }
    auto val = [&](int64_t i) -> int64_t {
        return src.type == DPF_TYPE_I32 ? (int64_t)((const int32_t*)src.values)[i] : ((const int64_t*)src.values)[i];
    };
    if (enc == DPF_ENC_AUTO) {
        bool sorted = true;
        for (int64_t i = 1; i < n && sorted; ++i) sorted = val(i) >= val(i - 1);
        enc = (sorted && n > 0) ? DPF_ENC_DELTA : DPF_ENC_FOR;
    }
    if (enc < DPF_ENC_FOR || enc > DPF_ENC_FSST) { *err = "unknown encoding"; return DPF_ERR_INVALID_ARG; }

    HostColumn& c = *out;
    c = HostColumn();
    c.type = src.type;
    c.enc = enc;
    c.chunk_rows = chunk_rows;
    c.nrows = n;
    c.nmb = (n + kMB - 1) / kMB;
    c.nchunks = (n + chunk_rows - 1) / chunk_rows;
    const int64_t nmb = c.nmb;

    // Integer stream of the column: values, dictionary codes or lengths.
    std::vector<int32_t> codes;
    if (enc == DPF_ENC_DICT) {
        std::vector<std::vector<int64_t>> parts(threads);
        bool too_many = false;
        std::vector<int64_t> bounds(threads + 1, n);
        int64_t step = (n + threads - 1) / std::max(1, threads);
        for (int t = 0; t <= threads; ++t) bounds[t] = std::min(n, (int64_t)t * step);
        std::vector<std::thread> pool;
        for (int t = 0; t < threads; ++t) {
            pool.emplace_back([&, t] {
                std::vector<int64_t>& d = parts[t];
                for (int64_t i = bounds[t]; i < bounds[t + 1] && !too_many; ++i) {
                    int64_t x = val(i);
                    auto it = std::lower_bound(d.begin(), d.end(), x);
                    if (it == d.end() || *it != x) {
                        d.insert(it, x);
                        if ((int64_t)d.size() > kMaxDict) too_many = true;
                    }
                }
            });
        }
        for (auto& th : pool) th.join();
        if (too_many) { *err = "more than 65536 distinct values for DICT"; return DPF_ERR_UNSUPPORTED; }
        for (auto& d : parts) c.dict.insert(c.dict.end(), d.begin(), d.end());
        std::sort(c.dict.begin(), c.dict.end());
        c.dict.erase(std::unique(c.dict.begin(), c.dict.end()), c.dict.end());
        if ((int64_t)c.dict.size() > kMaxDict) { *err = "more than 65536 distinct values for DICT"; return DPF_ERR_UNSUPPORTED; }
        codes.resize(n);
        parallel_for(n, threads, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i)
                codes[i] = (int32_t)(std::lower_bound(c.dict.begin(), c.dict.end(), val(i)) - c.dict.begin());
        });
    }
    // FSST: per chunk, a symbol table from a sample of the chunk's strings
    // (every k-th string, up to kSampleBytes, each cut to 4 KB), then every
    // string compressed with it; clen holds the code bytes per row.
    std::vector<uint32_t> clen;
    if (fsst) {
        constexpr size_t kSampleBytes = 32768;
        constexpr size_t kSampleCut = 4096;
        clen.resize(n);
        c.symtab.assign(c.nchunks * kFsstTableBytes, 0);
        std::vector<std::vector<uint8_t>> parts(c.nchunks);
        std::vector<int> bad(c.nchunks, 0);
        parallel_for(c.nchunks, threads, [&](int64_t a, int64_t b) {
            for (int64_t k = a; k < b; ++k) {
                const int64_t r0 = k * chunk_rows, r1 = std::min<int64_t>(n, r0 + chunk_rows);
                const uint64_t bytes = (uint64_t)(src.str_offsets[r1] - src.str_offsets[r0]);
                const int64_t stride = std::max<int64_t>(1, (int64_t)(bytes / kSampleBytes));
                std::vector<const uint8_t*> sp;
                std::vector<size_t> sl;
                size_t got = 0;
                for (int64_t r = r0; r < r1 && got < kSampleBytes; r += stride) {
                    const size_t l = std::min<size_t>(kSampleCut, (size_t)(src.str_offsets[r + 1] - src.str_offsets[r]));
                    sp.push_back(src.str_bytes + src.str_offsets[r]);
                    sl.push_back(l);
                    got += l;
                }
                const FsstTable t = fsst_build(sp, sl);
                fsst_serialize(t, c.symtab.data() + k * kFsstTableBytes);
                const FsstMatcher mt(t);
                std::vector<uint8_t>& out = parts[k];
                out.reserve(bytes / 2 + 64);
                for (int64_t r = r0; r < r1; ++r) {
                    const size_t cl = fsst_compress(mt, src.str_bytes + src.str_offsets[r],
                                                    (size_t)(src.str_offsets[r + 1] - src.str_offsets[r]), out);
                    if (cl > 0xFFFFFFFFu) bad[k] = 1;
                    clen[r] = (uint32_t)cl;
                }
            }
        });
        if (std::count(bad.begin(), bad.end(), 1)) { *err = "FSST record over 4 GB"; return DPF_ERR_UNSUPPORTED; }
        uint64_t tot = 0;
        for (auto& pt : parts) tot += pt.size();
        c.heap_bytes = tot;
        c.heap.assign(tot + kHeapPad, 0);
        uint64_t at = 0;
        for (auto& pt : parts) {
            if (!pt.empty()) std::memcpy(c.heap.data() + at, pt.data(), pt.size());
            at += pt.size();
            std::vector<uint8_t>().swap(pt);
        }
    }
    auto stream_at = [&](int64_t i) -> int64_t {
        if (enc == DPF_ENC_DICT) return codes[i];
        if (enc == DPF_ENC_VARLEN) return src.str_offsets[i + 1] - src.str_offsets[i];
        if (enc == DPF_ENC_FSST) return clen[i];
        return val(i);
    };

    c.base.assign(nmb, 0);
    c.woff.assign(nmb + 1, 0);
    if (enc == DPF_ENC_DELTA) c.dmin.assign(nmb, 0);
    std::vector<uint8_t> width(nmb, 0);
    const bool delta = enc == DPF_ENC_DELTA;
    // PLAIN: FOR at full width from a fixed base, whatever the block holds
    const bool plain = enc == DPF_ENC_PLAIN;
    const int plain_w = src.type == DPF_TYPE_I32 ? 32 : 64;
    const int64_t plain_base = src.type == DPF_TYPE_I32 ? (int64_t)INT32_MIN : INT64_MIN;
    auto prepare = [&](const int64_t* x, int cnt, int64_t* bs, int64_t* dm, uint64_t* u) -> int {
        if (!plain) return prepare_block(x, cnt, delta, bs, dm, u);
        *bs = plain_base;
        for (int i = 0; i < cnt; ++i) u[i] = (uint64_t)x[i] - (uint64_t)plain_base;
        return cnt ? plain_w : 0;
    };
    parallel_for(nmb, threads, [&](int64_t a, int64_t b) {
        int64_t x[kMB];
        uint64_t u[kMB];
        for (int64_t m = a; m < b; ++m) {
            int cnt = (int)std::min<int64_t>(kMB, n - m * kMB);
            for (int i = 0; i < cnt; ++i) x[i] = stream_at(m * kMB + i);
            int64_t dm = 0;
            width[m] = (uint8_t)prepare(x, cnt, &c.base[m], delta ? &dm : nullptr, u);
            if (delta) c.dmin[m] = dm;
        }
    });
    uint64_t total = 0;
    for (int64_t m = 0; m < nmb; ++m) {
        c.woff[m] = (uint32_t)total;
        total += 8u * width[m];
        if (total > 0xFFFFFFF0ull - kWordPad) {
            *err = "column exceeds 2^32 packed words";
            return DPF_ERR_UNSUPPORTED;
        }
    }
    c.woff[nmb] = (uint32_t)total;
    c.nwords = total;
    c.words.assign(total + kWordPad, 0u);
    parallel_for(nmb, threads, [&](int64_t a, int64_t b) {
        int64_t x[kMB];
        uint64_t u[kMB];
        for (int64_t m = a; m < b; ++m) {
            int cnt = (int)std::min<int64_t>(kMB, n - m * kMB);
            for (int i = 0; i < cnt; ++i) x[i] = stream_at(m * kMB + i);
            for (int i = cnt; i < kMB; ++i) u[i] = 0;
            int64_t bs, dm;
            int w = prepare(x, cnt, &bs, delta ? &dm : nullptr, u);
            pack(u, cnt, w, c.words.data() + c.woff[m]);
        }
    });

    if (enc == DPF_ENC_VARLEN) {
        c.heap_bytes = n ? (uint64_t)src.str_offsets[n] : 0;
        c.heap.assign(c.heap_bytes + kHeapPad, 0);
        if (c.heap_bytes) std::memcpy(c.heap.data(), src.str_bytes, c.heap_bytes);
        c.hoff.resize(nmb + 1);
        for (int64_t m = 0; m < nmb; ++m) c.hoff[m] = (uint64_t)src.str_offsets[m * kMB];
        c.hoff[nmb] = c.heap_bytes;
    }
    if (is_str) c.str_bytes = n ? (uint64_t)src.str_offsets[n] : 0;
    if (fsst) {
        c.hoff.resize(nmb + 1);
        c.doff.resize(nmb + 1);
        uint64_t h = 0;
        for (int64_t m = 0; m < nmb; ++m) {
            c.hoff[m] = h;
            c.doff[m] = (uint64_t)src.str_offsets[m * kMB];
            const int64_t e = std::min<int64_t>(n, (m + 1) * kMB);
            for (int64_t r = m * kMB; r < e; ++r) h += clen[r];
        }
        c.hoff[nmb] = h;
        c.doff[nmb] = c.str_bytes;
    }

    // Chunk directory: row-id index (prefix of row counts), byte ranges and
    // zone maps (value min/max; lengths for strings).
    c.chunks.resize(c.nchunks);
    const int64_t mbpc = chunk_rows / kMB;
    parallel_for(c.nchunks, threads, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            ChunkInfo& ci = c.chunks[k];
            ci.row_start = k * chunk_rows;
            ci.nrows = std::min<int64_t>(chunk_rows, n - ci.row_start);
            int64_t m0 = k * mbpc, m1 = std::min(nmb, m0 + mbpc);
            if (is_str) {
                ci.byte_offset = (int64_t)c.hoff[m0];
                ci.byte_length = (int64_t)(c.hoff[m1] - c.hoff[m0]);
            } else {
                ci.byte_offset = (int64_t)c.woff[m0] * 4;
                ci.byte_length = (int64_t)(c.woff[m1] - c.woff[m0]) * 4;
            }
            int64_t mn = INT64_MAX, mx = INT64_MIN;
            for (int64_t i = ci.row_start; i < ci.row_start + ci.nrows; ++i) {
                int64_t x = is_str ? src.str_offsets[i + 1] - src.str_offsets[i] : val(i);
                mn = std::min(mn, x);
                mx = std::max(mx, x);
            }
            ci.min = ci.nrows ? mn : 0;
            ci.max = ci.nrows ? mx : 0;
        }
    });
    if (c.nchunks) {
        c.minv = INT64_MAX;
        c.maxv = INT64_MIN;
        for (auto& ci : c.chunks) {
            c.minv = std::min(c.minv, ci.min);
            c.maxv = std::max(c.maxv, ci.max);
        }
    }
    return DPF_OK;
}

dpf_status decode_column(const HostColumn& c, const ColView& v, void* values, int64_t* str_offsets,
                         uint8_t* str_bytes, size_t cap, std::string* err) {
    const int64_t n = c.nrows;
    const bool is_str = c.enc == DPF_ENC_VARLEN || c.enc == DPF_ENC_FSST;
    if (is_str) {
        if (!str_offsets || (c.str_bytes && !str_bytes)) { *err = "missing output arrays"; return DPF_ERR_INVALID_ARG; }
        if (cap < c.str_bytes) { *err = "string byte capacity too small"; return DPF_ERR_INVALID_ARG; }
    } else if (!values && n) {
        *err = "missing output array";
        return DPF_ERR_INVALID_ARG;
    }
    int64_t off = 0;
    if (str_offsets) str_offsets[0] = 0;
    // FSST: the lengths are code bytes; each record decodes with its chunk's
    // table into the output at the running decoded offset.
    const int64_t mbpc = c.chunk_rows / kMB;
    FsstTable tab;
    int64_t tab_chunk = -1;
    uint64_t coff = 0;  // code offset of the current row
    for (int64_t m = 0; m < c.nmb; ++m) {
        uint32_t nw = v.woff[m + 1] - v.woff[m];
        if (nw % 8 != 0 || nw > 512) { *err = "corrupt mini-block header"; return DPF_ERR_CORRUPT; }
        int b = (int)(nw / 8);
        const uint32_t* w = v.words + v.woff[m];
        int cnt = (int)std::min<int64_t>(kMB, n - m * kMB);
        uint64_t run = 0;
        for (int i = 0; i < cnt; ++i) {
            uint64_t u = unpack(w, i, b);
            int64_t x;
            if (c.enc == DPF_ENC_DELTA) {
                run += (i ? (uint64_t)v.dmin[m] : 0) + u;
                x = (int64_t)((uint64_t)v.base[m] + run);
            } else {
                x = (int64_t)((uint64_t)v.base[m] + u);
            }
            int64_t r = m * kMB + i;
            if (c.enc == DPF_ENC_DICT) {
                if (x < 0 || x >= (int64_t)c.dict.size()) { *err = "corrupt dictionary code"; return DPF_ERR_CORRUPT; }
                x = v.dict[x];
            }
            if (c.enc == DPF_ENC_VARLEN) {
                off += x;
                str_offsets[r + 1] = off;
            } else if (c.enc == DPF_ENC_FSST) {
                if (m / mbpc != tab_chunk) {
                    tab_chunk = m / mbpc;
                    if (!fsst_deserialize(v.symtab + tab_chunk * kFsstTableBytes, &tab)) {
                        *err = "corrupt FSST symbol table";
                        return DPF_ERR_CORRUPT;
                    }
                }
                if (i == 0) coff = v.hoff[m];
                if (x < 0 || coff + (uint64_t)x > c.heap_bytes) { *err = "corrupt FSST lengths"; return DPF_ERR_CORRUPT; }
                const int64_t d = fsst_decode(tab, v.heap + coff, (size_t)x, str_bytes + off, cap - (size_t)off);
                if (d < 0) { *err = "corrupt FSST codes"; return DPF_ERR_CORRUPT; }
                coff += (uint64_t)x;
                off += d;
                str_offsets[r + 1] = off;
            } else if (c.type == DPF_TYPE_I32) {
                ((int32_t*)values)[r] = (int32_t)x;
            } else {
                ((int64_t*)values)[r] = x;
            }
        }
    }
    if (c.enc == DPF_ENC_VARLEN) {
        if ((uint64_t)off != c.heap_bytes) { *err = "string lengths disagree with the heap"; return DPF_ERR_CORRUPT; }
        if (c.heap_bytes) std::memcpy(str_bytes, v.heap, c.heap_bytes);
    }
    if (c.enc == DPF_ENC_FSST && (uint64_t)off != c.str_bytes) {
        *err = "decoded strings disagree with the column's size";
        return DPF_ERR_CORRUPT;
    }
    return DPF_OK;
}

}  // namespace dpf

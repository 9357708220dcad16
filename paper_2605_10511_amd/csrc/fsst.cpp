// fsst.cpp -- FSST symbol tables, compression and decoding on the host.
#include "fsst.h"

#include <algorithm>
#include <cstring>

namespace dpf {
namespace {

constexpr int kGenerations = 5;

inline uint64_t low_mask(int nbytes) { return nbytes >= 8 ? ~uint64_t(0) : (uint64_t(1) << (8 * nbytes)) - 1; }

// Up to 8 bytes of s as a little-endian word (bytes past n are zero).
inline uint64_t load8(const uint8_t* s, size_t n) {
    uint64_t x = 0;
    std::memcpy(&x, s, n < 8 ? n : 8);
    return x;
}

struct Cand {
    uint64_t v;
    int len;
    uint64_t gain;
};

}  // namespace

FsstMatcher::FsstMatcher(const FsstTable& t) : t_(t), start_(65537, 0) {
    for (int b = 0; b < 256; ++b) single_[b] = -1;
    std::vector<int> multi;
    for (int c = 0; c < t.n; ++c) {
        if (t.len[c] == 1)
            single_[t.sym[c] & 0xFF] = (int16_t)c;
        else
            multi.push_back(c);
    }
    std::sort(multi.begin(), multi.end(), [&](int a, int b) {
        uint32_t ka = (uint32_t)(t.sym[a] & 0xFFFF), kb = (uint32_t)(t.sym[b] & 0xFFFF);
        if (ka != kb) return ka < kb;
        if (t.len[a] != t.len[b]) return t.len[a] > t.len[b];
        return a < b;
    });
    for (int c : multi) start_[(t.sym[c] & 0xFFFF) + 1]++;
    for (int k = 0; k < 65536; ++k) start_[k + 1] += start_[k];
    order_.assign(multi.begin(), multi.end());
}

int FsstMatcher::match(const uint8_t* s, size_t n, int* len) const {
    if (n >= 2) {
        const uint64_t x = load8(s, n);
        const uint32_t key = (uint32_t)(x & 0xFFFF);
        for (uint32_t i = start_[key]; i < start_[key + 1]; ++i) {
            const int c = order_[i];
            const int l = t_.len[c];
            if ((size_t)l <= n && ((x ^ t_.sym[c]) & low_mask(l)) == 0) {
                *len = l;
                return c;
            }
        }
    }
    const int c = single_[s[0]];
    *len = 1;
    return c;
}

FsstTable fsst_build(const std::vector<const uint8_t*>& ptr, const std::vector<size_t>& len) {
    // Usage ids: 0..254 table symbols, 255 + b the literal byte b.
    constexpr int kIds = 255 + 256;
    FsstTable t;
    std::vector<uint32_t> cnt1(kIds), cnt2((size_t)kIds * kIds);
    for (int gen = 0; gen < kGenerations; ++gen) {
        FsstMatcher m(t);
        std::fill(cnt1.begin(), cnt1.end(), 0u);
        std::fill(cnt2.begin(), cnt2.end(), 0u);
        for (size_t r = 0; r < ptr.size(); ++r) {
            const uint8_t* s = ptr[r];
            const size_t n = len[r];
            int prev = -1;
            for (size_t p = 0; p < n;) {
                int l;
                const int c = m.match(s + p, n - p, &l);
                const int id = c >= 0 ? c : 255 + s[p];
                cnt1[id]++;
                if (prev >= 0) cnt2[(size_t)prev * kIds + id]++;
                prev = id;
                p += (size_t)l;
            }
        }
        auto sym_of = [&](int id, uint64_t* v) -> int {
            if (id < 255) {
                *v = t.sym[id];
                return t.len[id];
            }
            *v = (uint64_t)(id - 255);
            return 1;
        };
        std::vector<Cand> cands;
        for (int a = 0; a < kIds; ++a) {
            if (!cnt1[a]) continue;
            uint64_t va;
            const int la = sym_of(a, &va);
            cands.push_back({va, la, (uint64_t)cnt1[a] * (uint64_t)la});
            if (la == 8) continue;  // a concatenation would be cut back to a itself
            for (int b = 0; b < kIds; ++b) {
                const uint32_t k = cnt2[(size_t)a * kIds + b];
                if (!k) continue;
                uint64_t vb;
                const int lb = sym_of(b, &vb);
                const int l = std::min(la + lb, 8);
                const uint64_t v = (va | (vb << (8 * la))) & low_mask(l);
                cands.push_back({v, l, (uint64_t)k * (uint64_t)l});
            }
        }
        // merge equal candidates, then keep the 255 of highest gain
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) {
            return x.len != y.len ? x.len < y.len : x.v < y.v;
        });
        std::vector<Cand> merged;
        for (const Cand& c : cands) {
            if (!merged.empty() && merged.back().len == c.len && merged.back().v == c.v)
                merged.back().gain += c.gain;
            else
                merged.push_back(c);
        }
        std::sort(merged.begin(), merged.end(), [](const Cand& x, const Cand& y) {
            if (x.gain != y.gain) return x.gain > y.gain;
            return x.len != y.len ? x.len > y.len : x.v < y.v;
        });
        FsstTable next;
        next.n = (int)std::min<size_t>(merged.size(), kFsstSymbols);
        for (int c = 0; c < next.n; ++c) {
            next.sym[c] = merged[c].v;
            next.len[c] = (uint8_t)merged[c].len;
        }
        t = next;
    }
    return t;
}

size_t fsst_compress(const FsstMatcher& m, const uint8_t* s, size_t n, std::vector<uint8_t>& out) {
    const size_t before = out.size();
    for (size_t p = 0; p < n;) {
        int l;
        const int c = m.match(s + p, n - p, &l);
        if (c >= 0) {
            out.push_back((uint8_t)c);
        } else {
            out.push_back((uint8_t)kFsstEscape);
            out.push_back(s[p]);
        }
        p += (size_t)l;
    }
    return out.size() - before;
}

int64_t fsst_decode(const FsstTable& t, const uint8_t* codes, size_t n, uint8_t* out, size_t cap) {
    size_t o = 0;
    for (size_t i = 0; i < n; ++i) {
        const int c = codes[i];
        if (c == kFsstEscape) {
            if (i + 1 >= n || o + 1 > cap) return -1;
            out[o++] = codes[++i];
            continue;
        }
        if (c >= t.n) return -1;
        const int l = t.len[c];
        if (o + (size_t)l > cap) return -1;
        const uint64_t v = t.sym[c];
        std::memcpy(out + o, &v, (size_t)l);
        o += (size_t)l;
    }
    return (int64_t)o;
}

void fsst_serialize(const FsstTable& t, uint8_t* dst) {
    std::memset(dst, 0, kFsstTableBytes);
    std::memcpy(dst, t.sym, (size_t)t.n * 8);
    std::memcpy(dst + 256 * 8, t.len, (size_t)t.n);
}

bool fsst_deserialize(const uint8_t* src, FsstTable* t) {
    *t = FsstTable();
    std::memcpy(t->sym, src, 256 * 8);
    std::memcpy(t->len, src + 256 * 8, 256);
    int n = 0;
    while (n < kFsstSymbols && t->len[n] != 0) ++n;
    t->n = n;
    for (int c = 0; c < 256; ++c) {
        if (c < n ? (t->len[c] > 8 || (t->sym[c] & ~low_mask(t->len[c])) != 0) : (t->len[c] != 0 || t->sym[c] != 0))
            return false;
    }
    return true;
}

}  // namespace dpf

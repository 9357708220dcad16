// fsst.h -- host-side FSST string compression (paper Section 3.4.2: strings
// compressed with FSST, one static symbol table per page/chunk; Section 4.1:
// a 255-entry table lets every record decode on its own).
//
// A symbol is 1..8 bytes.  A compressed record is a byte string of codes:
// code c < 255 stands for symbol c, code 255 (the escape) for the byte that
// follows it.  Tables are built by the iterative method of the FSST paper
// (Boncz, Neumann, Leis, VLDB 2020): a few generations of compressing a
// sample with the current table, counting how often each symbol, each
// literal byte and each pair of consecutive ones is used, and keeping the
// 255 candidates -- those symbols and bytes, and the concatenations of the
// pairs cut to 8 bytes -- of highest gain (count times length).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace dpf {

constexpr int kFsstSymbols = 255;  // codes 0..254; 255 is the escape
constexpr int kFsstEscape = 255;
// Serialized table: sym[256] (uint64, little endian, bytes past the length
// zero) then len[256] (uint8; entry 255 unused and 0).
constexpr size_t kFsstTableBytes = 256 * 8 + 256;

struct FsstTable {
    uint64_t sym[256] = {};
    uint8_t len[256] = {};
    int n = 0;  // symbols in use: codes 0..n-1
};

// Longest-symbol lookup used by the compressor.
class FsstMatcher {
public:
    explicit FsstMatcher(const FsstTable& t);
    // Code of the longest symbol that is a prefix of s[0..n) (n >= 1), or
    // -1 when no symbol starts with s[0]; *len receives its length.
    int match(const uint8_t* s, size_t n, int* len) const;

private:
    const FsstTable& t_;
    std::vector<uint32_t> start_;  // [65537] first entry of each two-byte prefix in order_
    std::vector<uint8_t> order_;   // codes of length >= 2 by prefix, longest first
    int16_t single_[256];          // code of the one-byte symbol b, or -1
};

// Builds a table from sample strings (pointers and lengths).
FsstTable fsst_build(const std::vector<const uint8_t*>& ptr, const std::vector<size_t>& len);

// Appends the codes of s[0..n) to out; returns the number of code bytes.
size_t fsst_compress(const FsstMatcher& m, const uint8_t* s, size_t n, std::vector<uint8_t>& out);

// Decodes codes[0..n) with t into out (at most cap bytes).  Returns the
// decoded length, or -1 on a dangling escape, an unused code or overflow.
int64_t fsst_decode(const FsstTable& t, const uint8_t* codes, size_t n, uint8_t* out, size_t cap);

void fsst_serialize(const FsstTable& t, uint8_t* dst);    // kFsstTableBytes
bool fsst_deserialize(const uint8_t* src, FsstTable* t);  // false: malformed

}  // namespace dpf

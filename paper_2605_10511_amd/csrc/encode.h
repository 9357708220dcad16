// encode.h -- host-side type-specific column encoder and decoder.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "dpf.h"

namespace dpf {

struct ChunkInfo {
    int64_t row_start, nrows;
    int64_t byte_offset, byte_length;
    int64_t min, max;
};

// Pointers to the encoded arrays wherever they live on the host (the
// encoder's vectors, or a pinned host blob).
struct ColView {
    const int64_t* base = nullptr;   // [nmb]
    const uint32_t* woff = nullptr;  // [nmb + 1]
    const uint32_t* words = nullptr; // [nwords + pad]
    const int64_t* dmin = nullptr;   // DELTA [nmb]
    const uint64_t* hoff = nullptr;  // VARLEN, FSST [nmb + 1]
    const uint8_t* heap = nullptr;   // VARLEN, FSST [heap_bytes + pad]
    const int64_t* dict = nullptr;   // DICT [ndict]
    const uint64_t* doff = nullptr;  // FSST [nmb + 1]
    const uint8_t* symtab = nullptr; // FSST [nchunks * kFsstTableBytes]
};

struct HostColumn {
    int32_t type = 0, enc = 0, chunk_rows = 0;
    int64_t nrows = 0, nmb = 0, nchunks = 0;
    int64_t minv = 0, maxv = 0;
    std::vector<int64_t> base;
    std::vector<uint32_t> woff;
    std::vector<uint32_t> words;  // includes kWordPad trailing zero words
    std::vector<int64_t> dmin;
    std::vector<uint64_t> hoff;
    std::vector<uint8_t> heap;    // includes kHeapPad trailing zero bytes
    std::vector<int64_t> dict;
    // FSST: the heap holds codes and the packed lengths count code bytes;
    // doff[m] is the decoded byte offset of mini block m, symtab one
    // serialized symbol table per chunk.
    std::vector<uint64_t> doff;
    std::vector<uint8_t> symtab;
    std::vector<ChunkInfo> chunks;
    uint64_t nwords = 0;          // packed words, excluding padding
    uint64_t heap_bytes = 0;      // string (FSST: code) bytes, excluding padding
    uint64_t str_bytes = 0;       // decoded string bytes
};

constexpr int kWordPad = 16;
constexpr int kHeapPad = 64;

// Bytes a full scan of the column reads: packed words and mini-block headers
// (base, word offset; DELTA minimum difference; VARLEN heap offset and heap;
// FSST heap offset, code heap and one symbol table per chunk; DICT
// dictionary).
int64_t compressed_bytes(const HostColumn& c);

// Encodes src.  enc is a DPF_ENC_* value (AUTO resolved here).  Returns a
// dpf_status and fills err on failure.
dpf_status encode_column(const dpf_column_src& src, int32_t enc, int32_t chunk_rows, int32_t threads,
                         HostColumn* out, std::string* err);

ColView view_of(const HostColumn& c);

// Host decode of an encoded column through a view.
dpf_status decode_column(const HostColumn& meta, const ColView& v, void* values, int64_t* str_offsets,
                         uint8_t* str_bytes, size_t cap, std::string* err);

}  // namespace dpf

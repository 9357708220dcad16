// runtime.cpp -- the C ABI (include/dpf.h): contexts, encoded columns in HBM
// or pinned host memory, dimension hash builds, plan compilation into device
// descriptors, fused / fragmented execution and record decoding.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "dpf.h"
#include "dpf_internal.h"
#include "encode.h"

using namespace dpf;

namespace {
thread_local std::string g_err;

dpf_status fail(dpf_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

dpf_status hip_fail(hipError_t e, const char* what) {
    return fail(DPF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                              \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) return hip_fail(_e, #expr);          \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
}  // namespace

// ---------------------------------------------------------------------------
// Objects
// ---------------------------------------------------------------------------
struct dpf_ctx_s {
    int32_t device = -1;
    dpf_allocator alloc{};
    bool custom = false;
    int32_t ncu = 0;
    int64_t lds_per_block = 0;
    int64_t hbm = 0;
    std::atomic<int64_t> launches{0};
    uint8_t* scratch = nullptr;  // this device's address of the static scratch array
    hipStream_t upload = nullptr;  // plan uploads (non-blocking, default priority)

    // Allocations up to kPoolMax (plan workspaces, result buffers, hash
    // tables, build scratch) are recycled through power-of-two size classes:
    // in ROCm hipFree and hipHostFree synchronise the whole device, which
    // would stall a serving loop behind every kernel in flight on every
    // plan release.  Memory is returned when the context is destroyed.
    static constexpr size_t kPoolMin = 4096, kPoolMax = size_t(64) << 20;
    static constexpr int kClasses = 15;  // 4 KB .. 64 MB
    std::mutex pool_mu;
    std::unordered_map<void*, std::pair<int, int>> pooled;  // block -> (kind, class)
    std::vector<void*> pool_free[2][kClasses];

    void* raw_alloc(size_t bytes, int kind) {
        if (custom) return alloc.alloc(alloc.user, bytes, kind);
        void* p = nullptr;
        if (kind == DPF_MEM_HBM) {
            if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        } else {
            if (hipHostMalloc(&p, bytes, hipHostMallocMapped) != hipSuccess) return nullptr;
        }
        return p;
    }
    void raw_free(void* p, int kind) {
        if (custom) {
            // the caller's allocator may hand the block out again at once:
            // no kernel may still be reading it
            if (device >= 0) (void)hipDeviceSynchronize();
            alloc.free(alloc.user, p, kind);
            return;
        }
        if (kind == DPF_MEM_HBM) (void)hipFree(p);
        else (void)hipHostFree(p);
    }
    void* alloc_mem(size_t bytes, int kind) {
        if (bytes == 0) bytes = 16;
        if (bytes > kPoolMax) return raw_alloc(bytes, kind);
        int c = 0;
        while ((kPoolMin << c) < bytes) ++c;
        {
            std::lock_guard<std::mutex> g(pool_mu);
            std::vector<void*>& fl = pool_free[kind][c];
            if (!fl.empty()) {
                void* p = fl.back();
                fl.pop_back();
                return p;
            }
        }
        void* p = raw_alloc(kPoolMin << c, kind);
        if (p) {
            std::lock_guard<std::mutex> g(pool_mu);
            pooled[p] = {kind, c};
        }
        return p;
    }
    void free_mem(void* p, int kind) {
        if (!p) return;
        {
            std::lock_guard<std::mutex> g(pool_mu);
            auto it = pooled.find(p);
            if (it != pooled.end()) {
                pool_free[it->second.first][it->second.second].push_back(p);
                return;
            }
        }
        raw_free(p, kind);
    }
    ~dpf_ctx_s() {
        if (device >= 0) (void)hipDeviceSynchronize();
        if (upload) (void)hipStreamDestroy(upload);
        for (auto& kv : pooled) raw_free(kv.first, kv.second.first);
    }
    void* device_ptr(void* host) {  // device address of pinned host memory
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) return nullptr;
        return d;
    }
};

struct dpf_column_s {
    dpf_ctx ctx = nullptr;
    std::atomic<int> refs{1};
    HostColumn host;
    ColView view;
    int32_t placement = DPF_PLACE_HOST;
    void* blob = nullptr;  // HBM or pinned host allocation
    size_t blob_bytes = 0;
    DevCol dev{};
};

struct dpf_hash_s {
    dpf_ctx ctx = nullptr;
    std::atomic<int> refs{1};
    void* mem = nullptr;
    size_t bytes = 0;
    DevHash dev{};
    dpf_hash_stats stats{};
};

struct KeyOut {
    int64_t min = 0, card = 1, stride = 1;
    const int64_t* dict = nullptr;  // codes -> values
};

struct dpf_plan_s {
    dpf_ctx ctx = nullptr;
    std::atomic<int> refs{1};
    std::vector<dpf_column> cols;
    std::vector<dpf_hash> hashes;
    std::vector<int> hash_place;  // requested placement per probe
    DevQuery hq{};
    void* dmem = nullptr;  // [DevQuery][agg][status][counters]
    size_t dmem_bytes = 0;
    DevQuery* dq = nullptr;
    uint32_t* counters = nullptr;
    int64_t* host_out = nullptr;
    size_t host_out_bytes = 0;
    std::vector<KeyOut> keys;
    std::vector<std::pair<int, int>> outcols;  // (acc, kind): kind 0 = acc value
    int64_t nblocks = 0, nlive = 0;            // chunk pruning: blocks in all, blocks scanned
    int32_t lds_budget = -2;
    int32_t naggs_out = 0;
    bool issued = false;
    // The descriptor, block list and zeroed workspace go to the device on the
    // context's upload stream from this pinned staging copy; executions wait
    // for `uploaded` while `upload_pending`.
    void* staging = nullptr;
    hipEvent_t uploaded = nullptr;
    bool upload_pending = false;
    // fragmented execution buffers
    bool frag_ready = false;
    FragBuffers fb{};
    std::vector<void*> frag_allocs;
    size_t frag_bytes = 0;
};

struct dpf_result_s {
    hipEvent_t done = nullptr;  // recorded after the launch (absent under stream capture)
    std::vector<dpf_plan> plans;
    std::vector<std::vector<int64_t>> rows;
    std::vector<int32_t> ncols;
    std::vector<char> read;
};

// ---------------------------------------------------------------------------
// Static scratch for dpf_execute_noalloc: the work-queue counters, group
// tables and status words of one fused launch.  Every GPU holds its own copy
// of the array at its own address until the process ends; host code uses that
// address (from hipGetSymbolAddress), never the array's name, which on the
// host is only a stand-in for the symbol.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
uint8_t* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
// Looked up once per device and kept.
dpf_status static_scratch(int32_t device, uint8_t** out) {
    if (device < 0 || device >= kMaxDevices) return fail(DPF_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_addr[device] = (uint8_t*)p;
    }
    *out = g_scratch_addr[device];
    return DPF_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
extern "C" const char* dpf_last_error(void) { return g_err.c_str(); }

extern "C" dpf_status dpf_ctx_create(int32_t device, const dpf_allocator* allocator, dpf_ctx* out) {
    if (!out) return fail(DPF_ERR_INVALID_ARG, "out is NULL");
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(DPF_ERR_INVALID_ARG, "allocator needs alloc and free");
    dpf_ctx c = new (std::nothrow) dpf_ctx_s();
    if (!c) return fail(DPF_ERR_OOM, "ctx");
    c->device = device;
    if (allocator) { c->alloc = *allocator; c->custom = true; }
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            delete c;
            return fail(DPF_ERR_HIP, "no such HIP device");
        }
        e = hipSetDevice(device);
        hipDeviceProp_t prop;
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipGetDeviceProperties");
        }
        c->ncu = prop.multiProcessorCount;
        c->lds_per_block = (int64_t)prop.sharedMemPerBlock;
        if (c->lds_per_block < 160 * 1024) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
                c->lds_per_block = std::max<int64_t>(c->lds_per_block, v);
        }
        c->hbm = (int64_t)prop.totalGlobalMem;
        dpf_status st = static_scratch(device, &c->scratch);  // hipSetDevice(device) above made it current
        if (st != DPF_OK) {
            delete c;
            return st;
        }
        e = hipStreamCreateWithFlags(&c->upload, hipStreamNonBlocking);
        if (e != hipSuccess) {
            c->upload = nullptr;
            delete c;
            return hip_fail(e, "hipStreamCreateWithFlags(upload)");
        }
    }
    *out = c;
    return DPF_OK;
}

extern "C" void dpf_ctx_destroy(dpf_ctx ctx) { delete ctx; }

extern "C" dpf_status dpf_ctx_get_info(dpf_ctx ctx, dpf_ctx_info* out) {
    if (!ctx || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    out->device = ctx->device;
    out->num_cus = ctx->ncu;
    out->lds_per_block = ctx->lds_per_block;
    out->hbm_bytes = ctx->hbm;
    out->launches = ctx->launches.load();
    return DPF_OK;
}

// ---------------------------------------------------------------------------
// Columns
// ---------------------------------------------------------------------------
namespace {
// Lays the encoded arrays out in one blob (256-byte aligned sections);
// returns offsets.
struct BlobLayout {
    size_t base, woff, words, dmin, hoff, heap, dict, doff, symtab, total;
};

BlobLayout layout_of(const HostColumn& h) {
    BlobLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.base = take(h.base.size() * 8);
    L.woff = take(h.woff.size() * 4);
    L.words = take(h.words.size() * 4);
    L.dmin = take(h.dmin.size() * 8);
    L.hoff = take(h.hoff.size() * 8);
    L.heap = take(h.heap.size());
    L.dict = take(h.dict.size() * 8);
    L.doff = take(h.doff.size() * 8);
    L.symtab = take(h.symtab.size());
    L.total = std::max<size_t>(o, 256);
    return L;
}

void fill_blob(const HostColumn& h, const BlobLayout& L, uint8_t* dst) {
    auto put = [&](size_t at, const void* src, size_t bytes) { if (bytes) std::memcpy(dst + at, src, bytes); };
    put(L.base, h.base.data(), h.base.size() * 8);
    put(L.woff, h.woff.data(), h.woff.size() * 4);
    put(L.words, h.words.data(), h.words.size() * 4);
    put(L.dmin, h.dmin.data(), h.dmin.size() * 8);
    put(L.hoff, h.hoff.data(), h.hoff.size() * 8);
    put(L.heap, h.heap.data(), h.heap.size());
    put(L.dict, h.dict.data(), h.dict.size() * 8);
    put(L.doff, h.doff.data(), h.doff.size() * 8);
    put(L.symtab, h.symtab.data(), h.symtab.size());
}

DevCol dev_view(const HostColumn& h, const BlobLayout& L, const uint8_t* base) {
    DevCol d{};
    d.base = reinterpret_cast<const int64_t*>(base + L.base);
    d.woff = reinterpret_cast<const uint32_t*>(base + L.woff);
    d.words = reinterpret_cast<const uint32_t*>(base + L.words);
    d.dmin = h.dmin.empty() ? nullptr : reinterpret_cast<const int64_t*>(base + L.dmin);
    d.hoff = h.hoff.empty() ? nullptr : reinterpret_cast<const uint64_t*>(base + L.hoff);
    d.heap = h.heap.empty() ? nullptr : base + L.heap;
    d.dict = h.dict.empty() ? nullptr : reinterpret_cast<const int64_t*>(base + L.dict);
    d.doff = h.doff.empty() ? nullptr : reinterpret_cast<const uint64_t*>(base + L.doff);
    d.symtab = h.symtab.empty() ? nullptr : base + L.symtab;
    d.mbpc = h.chunk_rows / 256;
    d.nrows = h.nrows;
    d.heap_bytes = h.heap_bytes;
    d.str_bytes = h.str_bytes;
    d.nwords = (uint32_t)h.nwords;
    d.nmb = (int32_t)h.nmb;
    d.enc = h.enc == DPF_ENC_PLAIN ? ENC_FOR : h.enc;  // PLAIN is FOR at full width
    d.ndict = (int32_t)h.dict.size();
    return d;
}

ColView host_view(const HostColumn& h, const BlobLayout& L, const uint8_t* base) {
    ColView v;
    v.base = reinterpret_cast<const int64_t*>(base + L.base);
    v.woff = reinterpret_cast<const uint32_t*>(base + L.woff);
    v.words = reinterpret_cast<const uint32_t*>(base + L.words);
    v.dmin = h.dmin.empty() ? nullptr : reinterpret_cast<const int64_t*>(base + L.dmin);
    v.hoff = h.hoff.empty() ? nullptr : reinterpret_cast<const uint64_t*>(base + L.hoff);
    v.heap = h.heap.empty() ? nullptr : base + L.heap;
    v.dict = h.dict.empty() ? nullptr : reinterpret_cast<const int64_t*>(base + L.dict);
    v.doff = h.doff.empty() ? nullptr : reinterpret_cast<const uint64_t*>(base + L.doff);
    v.symtab = h.symtab.empty() ? nullptr : base + L.symtab;
    return v;
}
}  // namespace

extern "C" dpf_status dpf_column_encode(dpf_ctx ctx, const dpf_column_src* src, const dpf_encode_opts* opts,
                                        dpf_column* out) {
    if (!ctx || !src || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    dpf_encode_opts o{};
    if (opts) o = *opts;
    if (o.placement < DPF_PLACE_HBM || o.placement > DPF_PLACE_HOST)
        return fail(DPF_ERR_INVALID_ARG, "unknown placement");
    if (ctx->device < 0 && o.placement != DPF_PLACE_HOST)
        return fail(DPF_ERR_INVALID_ARG, "a host-only context supports DPF_PLACE_HOST only");
    try {
        dpf_column c = new dpf_column_s();
        c->ctx = ctx;
        std::string err;
        dpf_status st = encode_column(*src, o.encoding, o.chunk_rows, o.threads, &c->host, &err);
        if (st != DPF_OK) {
            delete c;
            return fail(st, err);
        }
        c->placement = o.placement;
        c->view = view_of(c->host);
        if (o.placement != DPF_PLACE_HOST) {
            BlobLayout L = layout_of(c->host);
            int kind = o.placement == DPF_PLACE_HBM ? DPF_MEM_HBM : DPF_MEM_HOST_MAPPED;
            c->blob = ctx->alloc_mem(L.total, kind);
            if (!c->blob) {
                delete c;
                return fail(DPF_ERR_OOM, "column allocation failed");
            }
            c->blob_bytes = L.total;
            if (kind == DPF_MEM_HBM) {
                std::vector<uint8_t> staging(L.total, 0);
                fill_blob(c->host, L, staging.data());
                hipError_t e = hipMemcpy(c->blob, staging.data(), L.total, hipMemcpyHostToDevice);
                if (e != hipSuccess) {
                    ctx->free_mem(c->blob, kind);
                    delete c;
                    return hip_fail(e, "hipMemcpy(column)");
                }
                c->dev = dev_view(c->host, L, (const uint8_t*)c->blob);
            } else {
                std::memset(c->blob, 0, L.total);
                fill_blob(c->host, L, (uint8_t*)c->blob);
                void* d = ctx->device_ptr(c->blob);
                if (!d) {
                    ctx->free_mem(c->blob, kind);
                    delete c;
                    return fail(DPF_ERR_HIP, "hipHostGetDevicePointer failed");
                }
                c->dev = dev_view(c->host, L, (const uint8_t*)d);
                // the pinned blob is now the only copy the kernels and the
                // host decoder use
                c->view = host_view(c->host, L, (const uint8_t*)c->blob);
                HostColumn& h = c->host;
                std::vector<int64_t>().swap(h.base);
                std::vector<uint32_t>().swap(h.woff);
                std::vector<uint32_t>().swap(h.words);
                std::vector<int64_t>().swap(h.dmin);
                std::vector<uint64_t>().swap(h.hoff);
                std::vector<uint8_t>().swap(h.heap);
                std::vector<uint64_t>().swap(h.doff);
                std::vector<uint8_t>().swap(h.symtab);
                // the dictionary stays on the host for result decoding
                c->view.dict = h.dict.empty() ? nullptr : h.dict.data();
            }
        }
        *out = c;
        return DPF_OK;
    } catch (const std::bad_alloc&) {
        return fail(DPF_ERR_OOM, "host allocation failed");
    }
}

extern "C" dpf_status dpf_column_info(dpf_column col, dpf_column_stats* out) {
    if (!col || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    const HostColumn& h = col->host;
    dpf_column_stats s{};
    s.type = h.type;
    s.encoding = h.enc;
    s.placement = col->placement;
    s.chunk_rows = h.chunk_rows;
    s.nrows = h.nrows;
    s.nchunks = h.nchunks;
    s.nminiblocks = h.nmb;
    s.compressed_bytes = compressed_bytes(h);
    s.min = h.minv;
    s.max = h.maxv;
    s.ndict = (int64_t)h.dict.size();
    s.str_bytes = (int64_t)h.str_bytes;
    *out = s;
    return DPF_OK;
}

extern "C" dpf_status dpf_column_chunk(dpf_column col, int64_t chunk, dpf_chunk_info* out) {
    if (!col || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (chunk < 0 || chunk >= col->host.nchunks) return fail(DPF_ERR_INVALID_ARG, "chunk out of range");
    const ChunkInfo& c = col->host.chunks[chunk];
    out->row_start = c.row_start;
    out->nrows = c.nrows;
    out->byte_offset = c.byte_offset;
    out->byte_length = c.byte_length;
    out->min = c.min;
    out->max = c.max;
    return DPF_OK;
}

extern "C" dpf_status dpf_column_decode(dpf_column col, void* values, int64_t* str_offsets, uint8_t* str_bytes,
                                        size_t cap) {
    if (!col) return fail(DPF_ERR_INVALID_ARG, "NULL column");
    std::string err;
    dpf_status st = decode_column(col->host, col->view, values, str_offsets, str_bytes, cap, &err);
    if (st != DPF_OK) return fail(st, err);
    return DPF_OK;
}

extern "C" dpf_status dpf_column_debug_offsets(dpf_column col, uint32_t** offsets) {
    if (!col || !offsets) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (col->placement == DPF_PLACE_HBM) return fail(DPF_ERR_INVALID_ARG, "offsets live in device memory");
    *offsets = const_cast<uint32_t*>(col->view.woff);
    return DPF_OK;
}

extern "C" void dpf_column_release(dpf_column col) {
    if (!col) return;
    if (--col->refs > 0) return;
    if (col->blob)
        col->ctx->free_mem(col->blob, col->placement == DPF_PLACE_HBM ? DPF_MEM_HBM : DPF_MEM_HOST_MAPPED);
    delete col;
}

// ---------------------------------------------------------------------------
// Predicates: value space -> the column's code space
// ---------------------------------------------------------------------------
namespace {
// Inclusive value range of LT..BETWEEN; false if empty.
bool pred_range(const dpf_pred& p, int64_t* lo, int64_t* hi) {
    *lo = INT64_MIN;
    *hi = INT64_MAX;
    switch (p.op) {
        case DPF_OP_LT: if (p.a == INT64_MIN) return false; *hi = p.a - 1; return true;
        case DPF_OP_LE: *hi = p.a; return true;
        case DPF_OP_GT: if (p.a == INT64_MAX) return false; *lo = p.a + 1; return true;
        case DPF_OP_GE: *lo = p.a; return true;
        case DPF_OP_EQ: *lo = *hi = p.a; return true;
        case DPF_OP_BETWEEN: *lo = p.a; *hi = p.b; return p.a <= p.b;
        default: return false;
    }
}

// The aligned-word lookup table of a string atom whose words both have at
// least 7 bytes (every occurrence then covers a whole 4-byte-aligned heap
// word, equal to one of the word's four 4-byte shifts): the first rotation
// that gives the distinct shifts distinct slots.  Leaves tab_rot = 0 when
// none does (the kernels then compare byte windows).
void build_str_table(DevPred& d) {
    d.tab_rot = 0;
    if (d.n1 < 7 || d.n2 < 7) return;
    uint32_t keys[8];
    for (int j = 0; j < 4; ++j) {
        uint32_t a = 0, b = 0;
        for (int t = 3; t >= 0; --t) {
            a = (a << 8) | d.s1[j + t];
            b = (b << 8) | d.s2[j + t];
        }
        keys[j] = a;
        keys[4 + j] = b;
    }
    for (uint32_t r = 1; r < 32; ++r) {
        bool used[32] = {};
        uint32_t owner[32] = {};
        bool ok = true;
        for (uint32_t k : keys) {
            const uint32_t sl = str_slot(k, r);
            if (used[sl] && owner[sl] != k) { ok = false; break; }
            used[sl] = true;
            owner[sl] = k;
        }
        if (!ok) continue;
        for (uint32_t i = 0; i < 32; ++i) {
            if (used[i]) { d.tab[i] = owner[i]; continue; }
            uint32_t e = 0;
            while (str_slot(e, r) == i) ++e;
            d.tab[i] = e;
        }
        d.tab_rot = r;
        return;
    }
}

inline bool is_string_enc(int32_t enc) { return enc == DPF_ENC_VARLEN || enc == DPF_ENC_FSST; }

// Byte automaton of LIKE '%s1%s2%' for FSST columns: the Knuth-Morris-Pratt
// automata of the two words in sequence.  States 0 .. n1-1 hold the length
// of the longest prefix of s1 that ends at the current byte; completing s1
// (its leftmost end) leads to state n1, where the search for s2 starts, and
// states n1 .. n1+n2-1 hold n1 plus the matched prefix of s2; n1 + n2 is the
// accept state, absorbing.  Row q holds the next state for each byte value.
std::vector<uint8_t> seq_automaton(const uint8_t* s1, int n1, const uint8_t* s2, int n2) {
    const int S = n1 + n2 + 1;
    std::vector<uint8_t> D((size_t)S * 256);
    auto word = [&](const uint8_t* w, int n, int base, int done) {
        // t[j][x]: matched prefix length after byte x from length j (KMP)
        std::vector<int> t((size_t)n * 256, 0);
        t[w[0]] = 1;
        for (int j = 1, back = 0; j < n; ++j) {
            for (int x = 0; x < 256; ++x) t[(size_t)j * 256 + x] = t[(size_t)back * 256 + x];
            t[(size_t)j * 256 + w[j]] = j + 1;
            back = t[(size_t)back * 256 + w[j]];
        }
        for (int j = 0; j < n; ++j)
            for (int x = 0; x < 256; ++x) {
                const int v = t[(size_t)j * 256 + x];
                D[(size_t)(base + j) * 256 + x] = (uint8_t)(v == n ? done : base + v);
            }
    };
    word(s1, n1, 0, n1);
    word(s2, n2, n1, n1 + n2);
    for (int x = 0; x < 256; ++x) D[(size_t)(S - 1) * 256 + x] = (uint8_t)(S - 1);
    return D;
}

// Translates p on column c into d.  *drop = the atom is always true.
dpf_status translate_pred(const dpf_pred& p, const HostColumn& c, std::vector<int64_t>& in_vals, DevPred& d,
                          bool* drop) {
    *drop = false;
    std::memset(&d, 0, sizeof d);
    d.col = p.col;
    const bool dict = c.enc == DPF_ENC_DICT;
    if (p.op == DPF_OP_STR_CONTAINS_SEQ) {
        if (!is_string_enc(c.enc)) return fail(DPF_ERR_INVALID_ARG, "string predicate on a non-string column");
        if (p.n1 < 1 || p.n2 < 1 || p.n1 > kMaxWord || p.n2 > kMaxWord || !p.s1 || !p.s2)
            return fail(DPF_ERR_UNSUPPORTED, "string predicate words must have 1..32 bytes");
        d.kind = PK_STR;
        d.n1 = p.n1;
        d.n2 = p.n2;
        std::memcpy(d.s1, p.s1, p.n1);
        std::memcpy(d.s2, p.s2, p.n2);
        if (c.enc == DPF_ENC_VARLEN) build_str_table(d);
        return DPF_OK;
    }
    if (is_string_enc(c.enc)) return fail(DPF_ERR_UNSUPPORTED, "integer predicate on a string column");
    if (p.op == DPF_OP_NE) {
        if (dict) {
            auto it = std::lower_bound(c.dict.begin(), c.dict.end(), p.a);
            if (it == c.dict.end() || *it != p.a) { *drop = true; return DPF_OK; }
            d.kind = PK_NE;
            d.lo = it - c.dict.begin();
        } else {
            if (c.nrows && (p.a < c.minv || p.a > c.maxv)) { *drop = true; return DPF_OK; }
            d.kind = PK_NE;
            d.lo = p.a;
        }
        return DPF_OK;
    }
    if (p.op == DPF_OP_IN) {
        if (p.n_in < 0 || p.n_in > kMaxIn || (p.n_in > 0 && !p.in_values))
            return fail(DPF_ERR_UNSUPPORTED, "IN lists hold at most 64 values");
        std::vector<int64_t> vals;
        for (int i = 0; i < p.n_in; ++i) {
            int64_t x = p.in_values[i];
            if (dict) {
                auto it = std::lower_bound(c.dict.begin(), c.dict.end(), x);
                if (it == c.dict.end() || *it != x) continue;
                x = it - c.dict.begin();
            }
            vals.push_back(x);
        }
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        if (vals.empty()) { d.kind = PK_FALSE; return DPF_OK; }
        if (dict && c.dict.size() <= 64) {
            d.kind = PK_INMASK;
            for (int64_t x : vals) d.mask |= uint64_t(1) << x;
            return DPF_OK;
        }
        if (in_vals.size() + vals.size() > (size_t)kMaxIn)
            return fail(DPF_ERR_UNSUPPORTED, "more than 64 IN values in one plan");
        d.kind = PK_INLIST;
        d.in_off = (int32_t)in_vals.size();
        d.n_in = (int32_t)vals.size();
        in_vals.insert(in_vals.end(), vals.begin(), vals.end());
        return DPF_OK;
    }
    int64_t lo, hi;
    if (p.op < DPF_OP_LT || p.op > DPF_OP_BETWEEN) return fail(DPF_ERR_INVALID_ARG, "unknown predicate op");
    if (!pred_range(p, &lo, &hi)) { d.kind = PK_FALSE; return DPF_OK; }
    if (dict) {
        int64_t clo = std::lower_bound(c.dict.begin(), c.dict.end(), lo) - c.dict.begin();
        int64_t chi = (std::upper_bound(c.dict.begin(), c.dict.end(), hi) - c.dict.begin()) - 1;
        if (clo > chi) { d.kind = PK_FALSE; return DPF_OK; }
        if (clo == 0 && chi == (int64_t)c.dict.size() - 1) { *drop = true; return DPF_OK; }
        lo = clo;
        hi = chi;
    } else if (c.nrows && lo <= c.minv && hi >= c.maxv) {
        *drop = true;  // the zone covers the whole column
        return DPF_OK;
    }
    d.kind = PK_RANGE;
    d.lo = lo;
    d.hi = hi;
    return DPF_OK;
}

// Integer-only value range of a column (value space).
void col_range(const HostColumn& c, int64_t* lo, int64_t* hi) {
    if (c.enc == DPF_ENC_DICT && !c.dict.empty()) {
        *lo = c.dict.front();
        *hi = c.dict.back();
    } else {
        *lo = c.minv;
        *hi = c.maxv;
    }
}
}  // namespace

// ---------------------------------------------------------------------------
// Hash build
// ---------------------------------------------------------------------------
extern "C" dpf_status dpf_hash_build(dpf_ctx ctx, const dpf_hash_desc* desc, dpf_stream stream, dpf_hash* out) {
    if (!ctx || !desc || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (ctx->device < 0) return fail(DPF_ERR_INVALID_ARG, "hash builds need a device context");
    if (desc->ncols < 1 || desc->ncols > kMaxHashCols || !desc->cols)
        return fail(DPF_ERR_INVALID_ARG, "1..8 dimension columns");
    if (desc->key_col < 0 || desc->key_col >= desc->ncols) return fail(DPF_ERR_INVALID_ARG, "bad key column");
    if (desc->npayloads < 0 || desc->npayloads > 2) return fail(DPF_ERR_INVALID_ARG, "0..2 payloads");
    if (desc->npreds < 0 || desc->npreds > kMaxHashPreds || (desc->npreds && !desc->preds))
        return fail(DPF_ERR_INVALID_ARG, "0..8 dimension predicates");
    if (desc->placement < DPF_HASH_AUTO || desc->placement > DPF_HASH_HBM)
        return fail(DPF_ERR_INVALID_ARG, "unknown hash placement");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nrows = desc->cols[0] ? desc->cols[0]->host.nrows : -1;
    for (int i = 0; i < desc->ncols; ++i) {
        dpf_column c = desc->cols[i];
        if (!c || c->host.nrows != nrows) return fail(DPF_ERR_INVALID_ARG, "dimension columns differ in length");
        if (c->placement == DPF_PLACE_HOST) return fail(DPF_ERR_INVALID_ARG, "dimension column not on the device");
    }
    auto int_col = [&](int i) { return i >= 0 && i < desc->ncols && !is_string_enc(desc->cols[i]->host.enc); };
    if (!int_col(desc->key_col)) return fail(DPF_ERR_INVALID_ARG, "key column must be an integer column");
    if (desc->nprobes < 0 || desc->nprobes > 2 || (desc->nprobes && !desc->probes))
        return fail(DPF_ERR_INVALID_ARG, "0..2 probes of the build side");
    for (int j = 0; j < desc->nprobes; ++j) {
        const dpf_probe& pr = desc->probes[j];
        if (!pr.hash || pr.hash->ctx != ctx) return fail(DPF_ERR_INVALID_ARG, "bad hash handle in a build-side probe");
        if (!int_col(pr.fk_col)) return fail(DPF_ERR_INVALID_ARG, "build-side probe key must be an integer column");
    }
    for (int j = 0; j < desc->npayloads; ++j) {
        const int src = desc->nprobes ? desc->payload_probe[j] : -1;
        if (src < 0) {
            if (!int_col(desc->payload_cols[j])) return fail(DPF_ERR_INVALID_ARG, "payload columns must be integer");
        } else if (src >= desc->nprobes || desc->payload_cols[j] < 0 ||
                   desc->payload_cols[j] >= desc->probes[src].hash->stats.npayloads) {
            return fail(DPF_ERR_INVALID_ARG, "payload taken from a build-side probe: bad probe or payload index");
        }
    }

    HashBuildArgs A;
    std::memset(&A, 0, sizeof A);
    A.ncols = desc->ncols;
    for (int i = 0; i < desc->ncols; ++i) A.cols[i] = desc->cols[i]->dev;
    std::vector<int64_t> in_vals;
    int np = 0;
    for (int i = 0; i < desc->npreds; ++i) {
        const dpf_pred& p = desc->preds[i];
        if (p.col < 0 || p.col >= desc->ncols) return fail(DPF_ERR_INVALID_ARG, "predicate column out of range");
        if (p.op == DPF_OP_STR_CONTAINS_SEQ) return fail(DPF_ERR_UNSUPPORTED, "string predicates on dimensions");
        bool drop;
        dpf_status st = translate_pred(p, desc->cols[p.col]->host, in_vals, A.preds[np], &drop);
        if (st != DPF_OK) return st;
        if (!drop) ++np;
    }
    A.npreds = np;
    std::copy(in_vals.begin(), in_vals.end(), A.in_vals);
    A.key_col = desc->key_col;
    A.npay = desc->npayloads;
    A.pay_col[0] = desc->npayloads > 0 ? desc->payload_cols[0] : 0;
    A.pay_col[1] = desc->npayloads > 1 ? desc->payload_cols[1] : 0;
    A.pay_src[0] = A.pay_src[1] = -1;
    for (int j = 0; j < desc->npayloads && desc->nprobes; ++j) A.pay_src[j] = desc->payload_probe[j];
    A.nsub = desc->nprobes;
    for (int j = 0; j < desc->nprobes; ++j) {
        DevProbe& P = A.sub[j];
        P.fk_col = desc->probes[j].fk_col;
        P.pay_slot[0] = P.pay_slot[1] = -1;
        P.h = desc->probes[j].hash->dev;  // read from device memory during the build
        P.h.lds_off = P.h.filt_lds_off = P.h.bits_lds_off = -1;
    }
    A.nrows = nrows;
    A.nmb = (int32_t)desc->cols[0]->host.nmb;

    // scratch: [args][count u64][mm 6 x i64][status]
    const size_t args_off = 0, cnt_off = align_up(sizeof(HashBuildArgs), 256), mm_off = cnt_off + 64,
                 st_off = mm_off + 64, scratch_bytes = st_off + 64;
    uint8_t* scratch = (uint8_t*)ctx->alloc_mem(scratch_bytes, DPF_MEM_HBM);
    if (!scratch) return fail(DPF_ERR_OOM, "hash scratch");
    struct Guard {
        dpf_ctx c; void* p;
        ~Guard() { c->free_mem(p, DPF_MEM_HBM); }
    } guard{ctx, scratch};
    A.count = (unsigned long long*)(scratch + cnt_off);
    A.mm = (long long*)(scratch + mm_off);
    A.status = (uint32_t*)(scratch + st_off);
    long long mm_init[6] = {INT64_MAX, INT64_MIN, INT64_MAX, INT64_MIN, INT64_MAX, INT64_MIN};
    uint8_t init[192] = {};
    std::memcpy(init + 64, mm_init, sizeof mm_init);
    HIP_TRY(hipMemcpyAsync(scratch + cnt_off, init, 192, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(scratch + args_off, &A, sizeof A, hipMemcpyHostToDevice, s));
    const int grid = std::max(1, std::min<int>((int)((A.nmb + 3) / 4), ctx->ncu * 8));
    HIP_TRY(launch_hash_count((const HashBuildArgs*)(scratch + args_off), grid, s));
    ctx->launches++;
    uint8_t back[192];
    HIP_TRY(hipMemcpyAsync(back, scratch + cnt_off, 192, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint64_t count;
    long long mm[6];
    uint32_t status;
    std::memcpy(&count, back, 8);
    std::memcpy(mm, back + 64, sizeof mm);
    std::memcpy(&status, back + 128, 4);
    if (status & ST_CORRUPT) return fail(DPF_ERR_CORRUPT, "corrupt dimension column");

    int log2cap = 4;
    while ((uint64_t(1) << log2cap) < 2 * count) ++log2cap;
    if (log2cap > 30) return fail(DPF_ERR_UNSUPPORTED, "hash table too large");
    const uint64_t cap = uint64_t(1) << log2cap;
    int pay64[2] = {0, 0};
    for (int j = 0; j < A.npay; ++j)
        pay64[j] = count && (mm[2 + 2 * j] < INT32_MIN || mm[3 + 2 * j] > INT32_MAX);
    size_t bytes = cap * 4;
    size_t pay_off[2] = {0, 0};
    for (int j = 0; j < A.npay; ++j) {
        pay_off[j] = bytes;
        bytes += cap * (pay64[j] ? 8 : 4);
    }
    // membership bitmap over the qualifying keys' range (not copied to LDS)
    const uint64_t kspan = count ? (uint64_t)(mm[1] - mm[0]) + 1 : 0;
    const bool use_bits = count && (uint64_t)(mm[1] - mm[0]) < kMaxBitmapBits;
    const size_t bits_off = align_up(bytes, 256);
    const size_t bits_words = use_bits ? (size_t)((kspan + 127) / 128) * 4 : 0;  // whole 16-byte units
    // LDS bit filter for small tables: two hashes, ~128 bits per key (a
    // false-positive rate near 1e-4), at most 2^kMaxFilterLog2 bits
    int flog2 = 0;
    if (count && count <= (uint64_t(1) << kMaxFilterLog2) / 16) {
        flog2 = 12;
        while (flog2 < kMaxFilterLog2 && (uint64_t(1) << flog2) < count * 128) ++flog2;
    }
    const size_t filt_off = align_up(use_bits ? bits_off + bits_words * 4 : bytes, 256);
    const size_t filt_words = flog2 ? (size_t(1) << flog2) / 32 : 0;
    const size_t alloc_bytes = flog2 ? filt_off + filt_words * 4 : (use_bits ? bits_off + bits_words * 4 : bytes);
    dpf_hash h = new (std::nothrow) dpf_hash_s();
    if (!h) return fail(DPF_ERR_OOM, "hash");
    h->ctx = ctx;
    h->mem = ctx->alloc_mem(alloc_bytes, DPF_MEM_HBM);
    if (!h->mem) {
        delete h;
        return fail(DPF_ERR_OOM, "hash table allocation failed");
    }
    h->bytes = alloc_bytes;  // device footprint (the LDS copy is dev.bytes: keys and payloads)
    auto bail = [&](dpf_status st, const std::string& m) {
        ctx->free_mem(h->mem, DPF_MEM_HBM);
        delete h;
        return fail(st, m);
    };
    A.keys = (int32_t*)h->mem;
    for (int j = 0; j < A.npay; ++j) {
        A.pay[j] = (uint8_t*)h->mem + pay_off[j];
        A.pay64[j] = pay64[j];
    }
    A.cap_mask = (uint32_t)(cap - 1);
    A.log2cap = log2cap;
    A.bits = use_bits ? (uint32_t*)((uint8_t*)h->mem + bits_off) : nullptr;
    A.bmin = use_bits ? mm[0] : 0;
    hipError_t e = launch_fill_i32((int32_t*)h->mem, kEmptyKey, (int64_t)cap, s);
    if (e == hipSuccess && use_bits) e = launch_fill_i32((int32_t*)A.bits, 0, (int64_t)bits_words, s);
    A.filt = flog2 ? (uint32_t*)((uint8_t*)h->mem + filt_off) : nullptr;
    A.flog2 = flog2;
    if (e == hipSuccess && flog2) e = launch_fill_i32((int32_t*)A.filt, 0, (int64_t)filt_words, s);
    if (e == hipSuccess) e = hipMemcpyAsync(scratch + args_off, &A, sizeof A, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_hash_insert((const HashBuildArgs*)(scratch + args_off), grid, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&status, A.status, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->launches += 2;
    if (e != hipSuccess) return bail(DPF_ERR_HIP, std::string("hash insert: ") + hipGetErrorString(e));
    if (status & ST_DUPLICATE) return bail(DPF_ERR_DUPLICATE_KEY, "duplicate key among qualifying rows");
    if (status & ST_UNSUPPORTED) return bail(DPF_ERR_UNSUPPORTED, "hash keys must fit int32 and differ from INT32_MIN");
    if (status & (ST_CORRUPT | ST_CAPACITY)) return bail(DPF_ERR_CORRUPT, "hash insert failed");

    DevHash& d = h->dev;
    d.keys = (const int32_t*)h->mem;
    for (int j = 0; j < 2; ++j) d.pay[j] = j < A.npay ? A.pay[j] : nullptr;
    d.cap_mask = (uint32_t)(cap - 1);
    d.log2cap = log2cap;
    d.npay = A.npay;
    d.pay64[0] = pay64[0];
    d.pay64[1] = pay64[1];
    d.lds_off = -1;
    d.bytes = (uint32_t)bytes;
    d.bits = A.bits;
    d.bmin = A.bmin;
    d.bspan = use_bits ? kspan : 0;
    d.filt = A.filt;
    d.flog2 = flog2;
    d.filt_lds_off = -1;
    d.bits_lds_off = -1;
    dpf_hash_stats& st = h->stats;
    st.entries = (int64_t)count;
    st.capacity = (int64_t)cap;
    st.bytes = (int64_t)bytes;
    st.lds_eligible = bytes <= 96 * 1024;
    st.device_bytes = (int64_t)alloc_bytes;
    st.placement = desc->placement;
    st.npayloads = A.npay;
    st.key_min = count ? mm[0] : 0;
    st.key_max = count ? mm[1] : 0;
    for (int j = 0; j < 2; ++j) {
        st.payload_min[j] = (count && j < A.npay) ? mm[2 + 2 * j] : 0;
        st.payload_max[j] = (count && j < A.npay) ? mm[3 + 2 * j] : 0;
    }
    *out = h;
    return DPF_OK;
}

extern "C" dpf_status dpf_hash_info(dpf_hash h, dpf_hash_stats* out) {
    if (!h || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    *out = h->stats;
    return DPF_OK;
}

extern "C" void dpf_hash_release(dpf_hash h) {
    if (!h) return;
    if (--h->refs > 0) return;
    h->ctx->free_mem(h->mem, DPF_MEM_HBM);
    delete h;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
namespace {
constexpr int32_t kDefaultLdsHash = 72 * 1024;
constexpr int64_t kAggLdsMax = 16 * 1024;

constexpr int64_t kDefaultMbPerItem = 64;  // 16,384 rows
constexpr int kTargetWavesPerCU = 24;       // string stage: 6 waves per SIMD (its register occupancy)
constexpr int kTargetWavesPerCUNoStr = 24;  // without it: also 6 waves per SIMD

// Places the plan's dimension tables and group table in the workgroup's LDS
// shared area within budget; fills lds offsets and lds_shared.
void assign_lds(dpf_plan p, int32_t budget) {
    DevQuery& q = p->hq;
    if (budget < 0) budget = kDefaultLdsHash;
    std::vector<int> order;
    int32_t off = 0;
    // an FSST atom's code table comes first (the kernel takes its address as
    // the start of the shared area): it is not optional
    q.fs_lds_off = -1;
    if (q.fs_pred >= 0) {
        q.fs_lds_off = off;
        off += (int32_t)align_up((size_t)(2 * q.fs_states + 1) * 256, 16);
    }
    // A probe that needs no payload only asks membership: its key-range
    // bitmap (when it has one) is the structure placed in LDS.
    for (int j = 0; j < q.nprobes; ++j) {
        DevProbe& P = q.probes[j];
        P.h.lds_off = -1;
        P.h.bits_lds_off = -1;
        if (p->hash_place[j] == DPF_HASH_HBM) continue;
        if (P.h.bits && P.pay_slot[0] < 0 && P.pay_slot[1] < 0) {
            const int32_t b = (int32_t)align_up((size_t)((P.h.bspan + 127) / 128) * 16, 16);
            if (off + (int64_t)b <= budget) {
                P.h.bits_lds_off = off;
                off += b;
                continue;
            }
        }
        order.push_back(j);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        // explicit LDS requests first, then smallest first
        int ra = p->hash_place[a] == DPF_HASH_LDS ? 0 : 1, rb = p->hash_place[b] == DPF_HASH_LDS ? 0 : 1;
        if (ra != rb) return ra < rb;
        return q.probes[a].h.bytes < q.probes[b].h.bytes;
    });
    for (int j : order) {
        uint32_t b = q.probes[j].h.bytes;
        if (off + (int64_t)b > budget) continue;
        q.probes[j].h.lds_off = off;
        off += (int32_t)align_up(b, 16);
    }
    // bit filters of the tables that stay in HBM, in probe order
    for (int j = 0; j < q.nprobes; ++j) {
        DevHash& h = q.probes[j].h;
        h.filt_lds_off = -1;
        if (!h.filt || h.lds_off >= 0 || h.bits_lds_off >= 0) continue;
        const int32_t b = (int32_t)((size_t(1) << h.flog2) / 8);
        if (off + (int64_t)b > budget) continue;
        h.filt_lds_off = off;
        off += (int32_t)align_up((size_t)b, 16);
    }
    const int64_t aggb = q.ngroups * q.nacc * 8;
    q.agg_lds = !q.agg_hash && aggb <= kAggLdsMax;
    q.agg_lds_off = off;
    if (q.agg_lds) off += (int32_t)align_up((size_t)aggb, 16);
    q.lds_shared = off;
    p->lds_budget = budget;
}

// Largest |mul * x + add| over x in [lo, hi].
__int128 term_bound(int64_t mul, int64_t add, int64_t lo, int64_t hi) {
    __int128 a = (__int128)mul * lo + add, b = (__int128)mul * hi + add;
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    return a > b ? a : b;
}

void free_frag(dpf_plan p) {
    for (void* a : p->frag_allocs) p->ctx->free_mem(a, DPF_MEM_HBM);
    p->frag_allocs.clear();
    p->frag_bytes = 0;
    p->frag_ready = false;
}
}  // namespace

// Chunk pruning (paper Section 3.1.1: Kernel #0 checks the predicates
// against the zone maps and passes on the pages that may qualify).  A mini
// block is excluded when, by the min/max its column recorded for the chunk
// holding it at encode time, one fact atom is false for every row, or one
// probe's foreign keys all miss the qualifying keys' range (the join is
// inner).  String chunks record lengths: rows shorter than |s1| + |s2|
// cannot match.  Blocks of prune_mb mini blocks (the smallest chunk of the
// plan's columns) that hold no surviving mini block are dropped.  Returns
// prune_mb, with the surviving blocks in live, or 0 when nothing is dropped.
int32_t prune_blocks(const dpf_plan_desc* desc, int32_t nmb, std::vector<int32_t>& live, int64_t* nblocks) {
    int64_t unit = INT64_MAX;
    for (int i = 0; i < desc->ncols; ++i) unit = std::min<int64_t>(unit, desc->cols[i]->host.chunk_rows / kMB);
    unit = std::max<int64_t>(1, std::min<int64_t>(unit, nmb > 0 ? nmb : 1));
    *nblocks = nmb > 0 ? (nmb + unit - 1) / unit : 0;
    if (nmb <= 0) return 0;
    std::vector<uint8_t> dead((size_t)nmb, 0);
    bool all_dead = false;
    auto kill = [&](const HostColumn& c, auto&& excluded) {
        for (const ChunkInfo& ci : c.chunks) {
            if (ci.nrows <= 0 || !excluded(ci.min, ci.max)) continue;
            const int64_t m0 = ci.row_start / kMB;
            const int64_t m1 = std::min<int64_t>(nmb, (ci.row_start + ci.nrows + kMB - 1) / kMB);
            if (m0 < m1) std::fill(dead.begin() + m0, dead.begin() + m1, 1);
        }
    };
    for (int i = 0; i < desc->npreds; ++i) {
        const dpf_pred& pr = desc->preds[i];
        const HostColumn& c = desc->cols[pr.col]->host;
        if (pr.op == DPF_OP_STR_CONTAINS_SEQ) {
            const int64_t need = (int64_t)pr.n1 + pr.n2;
            kill(c, [&](int64_t, int64_t hi) { return hi < need; });
        } else if (pr.op == DPF_OP_NE) {
            kill(c, [&](int64_t lo, int64_t hi) { return lo == hi && lo == pr.a; });
        } else if (pr.op == DPF_OP_IN) {
            kill(c, [&](int64_t lo, int64_t hi) {
                for (int k = 0; k < pr.n_in; ++k)
                    if (pr.in_values[k] >= lo && pr.in_values[k] <= hi) return false;
                return true;
            });
        } else {
            int64_t a, b;
            if (!pred_range(pr, &a, &b)) { all_dead = true; break; }
            kill(c, [&](int64_t lo, int64_t hi) { return hi < a || lo > b; });
        }
    }
    for (int j = 0; j < desc->nprobes && !all_dead; ++j) {
        const dpf_hash_stats& hs = desc->probes[j].hash->stats;
        if (hs.entries == 0) { all_dead = true; break; }
        kill(desc->cols[desc->probes[j].fk_col]->host,
             [&](int64_t lo, int64_t hi) { return hi < hs.key_min || lo > hs.key_max; });
    }
    live.clear();
    if (!all_dead)
        for (int64_t b = 0; b < *nblocks; ++b) {
            const int64_t m0 = b * unit, m1 = std::min<int64_t>(nmb, m0 + unit);
            for (int64_t m = m0; m < m1; ++m)
                if (!dead[(size_t)m]) { live.push_back((int32_t)b); break; }
        }
    if ((int64_t)live.size() == *nblocks) { live.clear(); return 0; }
    return (int32_t)unit;
}

extern "C" dpf_status dpf_plan_build(dpf_ctx ctx, const dpf_plan_desc* desc, dpf_plan* out) {
    if (!ctx || !desc || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (ctx->device < 0) return fail(DPF_ERR_INVALID_ARG, "plans need a device context");
    if (desc->ncols < 1 || desc->ncols > kMaxCols || !desc->cols) return fail(DPF_ERR_INVALID_ARG, "1..16 fact columns");
    if (desc->npreds < 0 || desc->npreds > kMaxPreds || (desc->npreds && !desc->preds))
        return fail(DPF_ERR_UNSUPPORTED, "0..12 predicates");
    if (desc->nprobes < 0 || desc->nprobes > kMaxProbes || (desc->nprobes && !desc->probes))
        return fail(DPF_ERR_UNSUPPORTED, "0..4 probes");
    if (desc->nkeys < 0 || desc->nkeys > kMaxKeys || (desc->nkeys && !desc->keys))
        return fail(DPF_ERR_UNSUPPORTED, "0..4 group keys");
    if (desc->naggs < 1 || !desc->aggs) return fail(DPF_ERR_INVALID_ARG, "at least one aggregate");
    const int64_t nrows = desc->cols[0] ? desc->cols[0]->host.nrows : -1;
    for (int i = 0; i < desc->ncols; ++i) {
        dpf_column c = desc->cols[i];
        if (!c || c->host.nrows != nrows) return fail(DPF_ERR_INVALID_ARG, "fact columns differ in length");
        if (c->placement == DPF_PLACE_HOST) return fail(DPF_ERR_INVALID_ARG, "fact column not on the device");
        if (c->ctx != ctx) return fail(DPF_ERR_INVALID_ARG, "column from another context");
    }
    if (nrows > (int64_t)UINT32_MAX) return fail(DPF_ERR_UNSUPPORTED, "tables are limited to 2^32 - 1 rows");

    dpf_plan p = new (std::nothrow) dpf_plan_s();
    if (!p) return fail(DPF_ERR_OOM, "plan");
    auto bail = [&](dpf_status st) {
        if (p->dmem) ctx->free_mem(p->dmem, DPF_MEM_HBM);
        if (p->host_out) ctx->free_mem(p->host_out, DPF_MEM_HOST_MAPPED);
        delete p;
        return st;
    };
    p->ctx = ctx;
    DevQuery& q = p->hq;
    std::memset(&q, 0, sizeof q);
    q.nrows = nrows;
    q.nmb = (int32_t)((nrows + kMB - 1) / kMB);
    q.ncols = desc->ncols;
    for (int i = 0; i < desc->ncols; ++i) q.cols[i] = desc->cols[i]->dev;

    // predicates: integer atoms (grouped by column) first, then strings
    std::vector<int64_t> in_vals;
    std::vector<DevPred> ints, strs;
    for (int i = 0; i < desc->npreds; ++i) {
        const dpf_pred& pr = desc->preds[i];
        if (pr.col < 0 || pr.col >= desc->ncols) return bail(fail(DPF_ERR_INVALID_ARG, "predicate column out of range"));
        DevPred d;
        bool drop;
        dpf_status st = translate_pred(pr, desc->cols[pr.col]->host, in_vals, d, &drop);
        if (st != DPF_OK) return bail(st);
        if (drop) continue;
        (d.kind == PK_STR ? strs : ints).push_back(d);
    }
    std::stable_sort(ints.begin(), ints.end(), [](const DevPred& a, const DevPred& b) { return a.col < b.col; });
    for (auto& d : ints) q.preds[q.npreds++] = d;
    q.nint_preds = q.npreds;
    for (auto& d : strs) q.preds[q.npreds++] = d;
    q.has_str = !strs.empty();
    // the fused kernel keeps the code table of one FSST atom per plan
    q.fs_pred = -1;
    std::vector<uint8_t> fs_dfa;
    for (int i = q.nint_preds; i < q.npreds; ++i) {
        if (desc->cols[q.preds[i].col]->host.enc != DPF_ENC_FSST) continue;
        if (q.fs_pred >= 0) return bail(fail(DPF_ERR_UNSUPPORTED, "a plan takes at most one FSST string predicate"));
        q.fs_pred = i;
        const DevPred& d = q.preds[i];
        fs_dfa = seq_automaton(d.s1, d.n1, d.s2, d.n2);
        q.fs_states = d.n1 + d.n2 + 1;
    }
    std::copy(in_vals.begin(), in_vals.end(), q.in_vals);

    // probes
    q.nprobes = desc->nprobes;
    for (int j = 0; j < desc->nprobes; ++j) {
        const dpf_probe& pr = desc->probes[j];
        if (!pr.hash || pr.hash->ctx != ctx) return bail(fail(DPF_ERR_INVALID_ARG, "bad hash handle"));
        if (pr.fk_col < 0 || pr.fk_col >= desc->ncols || is_string_enc(desc->cols[pr.fk_col]->host.enc))
            return bail(fail(DPF_ERR_INVALID_ARG, "probe key must be an integer fact column"));
        q.probes[j].fk_col = pr.fk_col;
        q.probes[j].pay_slot[0] = q.probes[j].pay_slot[1] = -1;
        q.probes[j].h = pr.hash->dev;
        p->hash_place.push_back(pr.hash->stats.placement);
    }

    // value slots: (fact column, as value) or (probe, payload)
    struct SlotKey { int kind, a, b; };
    std::vector<SlotKey> slots;
    auto slot_of = [&](const dpf_ref& r, bool as_value, int* slot, int64_t* lo, int64_t* hi, const int64_t** dict) -> dpf_status {
        SlotKey k{};
        if (r.kind == DPF_REF_COL) {
            if (r.idx < 0 || r.idx >= desc->ncols) return fail(DPF_ERR_INVALID_ARG, "reference column out of range");
            const HostColumn& c = desc->cols[r.idx]->host;
            if (is_string_enc(c.enc)) return fail(DPF_ERR_UNSUPPORTED, "string columns cannot be keys or terms");
            bool dict_code = c.enc == DPF_ENC_DICT && !as_value;
            k = {0, r.idx, dict_code ? 0 : 1};
            if (dict_code) { *lo = 0; *hi = (int64_t)c.dict.size() - 1; *dict = desc->cols[r.idx]->view.dict; }
            else { col_range(c, lo, hi); *dict = nullptr; }
            if (c.enc == DPF_ENC_DICT && c.dict.empty()) { *lo = 0; *hi = 0; }
        } else if (r.kind == DPF_REF_PAYLOAD) {
            if (r.probe < 0 || r.probe >= desc->nprobes) return fail(DPF_ERR_INVALID_ARG, "reference probe out of range");
            const dpf_hash_stats& hs = desc->probes[r.probe].hash->stats;
            if (r.idx < 0 || r.idx >= hs.npayloads) return fail(DPF_ERR_INVALID_ARG, "payload index out of range");
            k = {1, r.probe, r.idx};
            *lo = hs.payload_min[r.idx];
            *hi = hs.payload_max[r.idx];
            *dict = nullptr;
        } else {
            return fail(DPF_ERR_INVALID_ARG, "unknown reference kind");
        }
        for (size_t s = 0; s < slots.size(); ++s)
            if (slots[s].kind == k.kind && slots[s].a == k.a && slots[s].b == k.b) { *slot = (int)s; return DPF_OK; }
        if ((int)slots.size() >= kMaxSlots) return fail(DPF_ERR_UNSUPPORTED, "more than 8 distinct key/term values");
        slots.push_back(k);
        *slot = (int)slots.size() - 1;
        return DPF_OK;
    };

    // group keys
    __int128 G = 1;
    q.nkeys = desc->nkeys;
    p->keys.resize(desc->nkeys);
    for (int k = 0; k < desc->nkeys; ++k) {
        int slot;
        int64_t lo, hi;
        const int64_t* dict;
        dpf_status st = slot_of(desc->keys[k], false, &slot, &lo, &hi, &dict);
        if (st != DPF_OK) return bail(st);
        __int128 card = (__int128)hi - lo + 1;
        if (card < 1) card = 1;
        q.keys[k].slot = slot;
        q.keys[k].min = lo;
        q.keys[k].card = (int64_t)std::min<__int128>(card, INT64_MAX);
        p->keys[k].min = lo;
        p->keys[k].card = q.keys[k].card;
        p->keys[k].dict = dict;
        G *= card;
        if (G > kMaxGroupDomain) return bail(fail(DPF_ERR_UNSUPPORTED, "group-key domain exceeds 2^62"));
    }
    int64_t stride = 1;
    for (int k = desc->nkeys - 1; k >= 0; --k) {
        q.keys[k].stride = stride;
        p->keys[k].stride = stride;
        stride *= q.keys[k].card;
    }
    // A domain above kMaxGroups aggregates through a hash table (paper
    // Section 3.1, Kernel #3): at least twice as many slots as the groups
    // that can occur (no more than the domain, nor than the table's rows).
    q.agg_hash = G > kMaxGroups;
    if (q.agg_hash) {
        const int64_t can = std::min<int64_t>((int64_t)G, std::max<int64_t>(nrows, 1));
        int64_t slots = 64;
        while (slots < 2 * can) slots *= 2;
        if (slots > kMaxHashSlots)
            return bail(fail(DPF_ERR_UNSUPPORTED, "a hash group table above 2^22 slots (a group-key domain above "
                                                  "2^22 over more than 2^21 rows)"));
        q.ngroups = slots;
    } else {
        q.ngroups = (int64_t)G;
    }

    // accumulators: 0 = count, then one per SUM/AVG; int64 bound proof
    q.nacc = 1;
    p->outcols.clear();
    const __int128 lim = (__int128)INT64_MAX;
    for (int a = 0; a < desc->naggs; ++a) {
        const dpf_agg& ag = desc->aggs[a];
        if (ag.op == DPF_AGG_COUNT) { p->outcols.push_back({0, 0}); continue; }
        if (ag.op != DPF_AGG_SUM && ag.op != DPF_AGG_AVG) return bail(fail(DPF_ERR_INVALID_ARG, "unknown aggregate"));
        if (ag.nterms < 1 || ag.nterms > kMaxTerms) return bail(fail(DPF_ERR_INVALID_ARG, "1..3 terms"));
        if (q.nacc >= kMaxAccs) return bail(fail(DPF_ERR_UNSUPPORTED, "more than 11 sums"));
        DevAcc& A = q.accs[q.nacc];
        A.nterms = ag.nterms;
        __int128 bound = 1;
        for (int t = 0; t < ag.nterms; ++t) {
            const dpf_term& tm = ag.terms[t];
            __int128 tb;
            if (tm.has_ref) {
                int slot;
                int64_t lo, hi;
                const int64_t* dict;
                dpf_status st = slot_of(tm.ref, true, &slot, &lo, &hi, &dict);
                if (st != DPF_OK) return bail(st);
                A.t[t].slot = slot;
                A.t[t].mul = tm.mul;
                A.t[t].add = tm.add;
                tb = nrows ? term_bound(tm.mul, tm.add, lo, hi) : 0;
            } else {
                A.t[t].slot = -1;
                A.t[t].mul = 0;
                A.t[t].add = tm.add;
                tb = tm.add < 0 ? -(__int128)tm.add : (__int128)tm.add;
            }
            if (tb > lim) return bail(fail(DPF_ERR_OVERFLOW, "an aggregate term can exceed int64"));
            bound *= tb;
            if (bound > lim) return bail(fail(DPF_ERR_OVERFLOW, "an aggregate product can exceed int64"));
        }
        if (bound * (__int128)std::max<int64_t>(nrows, 1) > lim)
            return bail(fail(DPF_ERR_OVERFLOW, "an aggregate sum can exceed int64 over this table"));
        p->outcols.push_back({q.nacc, 1});
        if (ag.op == DPF_AGG_AVG) p->outcols.push_back({0, 0});
        q.nacc++;
    }
    // Renumber slots so fact-column loads take slots 0..nloads-1 (the kernel
    // writes those with compile-time indices) and payloads the ones after.
    std::vector<int> remap(slots.size());
    q.nloads = 0;
    for (size_t s = 0; s < slots.size(); ++s) {
        if (slots[s].kind != 0) continue;
        remap[s] = q.nloads;
        q.loads[q.nloads].col = slots[s].a;
        q.loads[q.nloads].slot = q.nloads;
        q.loads[q.nloads].dict_val = desc->cols[slots[s].a]->host.enc == DPF_ENC_DICT && slots[s].b == 1;
        q.nloads++;
    }
    int next = q.nloads;
    for (size_t s = 0; s < slots.size(); ++s) {
        if (slots[s].kind == 0) continue;
        remap[s] = next;
        q.probes[slots[s].a].pay_slot[slots[s].b] = next++;
    }
    for (int k = 0; k < q.nkeys; ++k) q.keys[k].slot = remap[q.keys[k].slot];
    for (int a = 1; a < q.nacc; ++a)
        for (int t = 0; t < q.accs[a].nterms; ++t)
            if (q.accs[a].t[t].slot >= 0) q.accs[a].t[t].slot = remap[q.accs[a].t[t].slot];
    assign_lds(p, -1);

    // chunk pruning
    std::vector<int32_t> live;
    const int32_t prune_mb = prune_blocks(desc, q.nmb, live, &p->nblocks);
    p->nlive = prune_mb ? (int64_t)live.size() : p->nblocks;

    // device memory: [DevQuery][agg table][status][counters][live blocks]
    // [FSST byte automaton]
    const size_t q_off = 0, agg_off = align_up(sizeof(DevQuery), 256);
    const size_t agg_bytes = agg_table_bytes(q);
    const size_t st_off = align_up(agg_off + agg_bytes, 256), cnt_off = st_off + 256;
    const size_t live_off = align_up(cnt_off + (size_t)kCounterWords * 4, 256);
    const size_t dfa_off = align_up(live_off + live.size() * 4, 256);
    p->dmem_bytes = dfa_off + fs_dfa.size();
    p->dmem = ctx->alloc_mem(p->dmem_bytes, DPF_MEM_HBM);
    if (!p->dmem) return bail(fail(DPF_ERR_OOM, "plan workspace"));
    p->host_out_bytes = (2 + (size_t)q.ngroups * (1 + q.nacc)) * 8;
    p->host_out = (int64_t*)ctx->alloc_mem(p->host_out_bytes, DPF_MEM_HOST_MAPPED);
    if (!p->host_out) return bail(fail(DPF_ERR_OOM, "pinned result buffer"));
    std::memset(p->host_out, 0, 16);
    int64_t* host_out_dev = (int64_t*)ctx->device_ptr(p->host_out);
    if (!host_out_dev) return bail(fail(DPF_ERR_HIP, "hipHostGetDevicePointer(result)"));
    uint8_t* d = (uint8_t*)p->dmem;
    p->dq = (DevQuery*)(d + q_off);
    q.agg = (int64_t*)(d + agg_off);
    q.status = (uint32_t*)(d + st_off);
    p->counters = (uint32_t*)(d + cnt_off);
    q.host_out = host_out_dev;
    q.live = prune_mb ? (const int32_t*)(d + live_off) : nullptr;
    q.nlive = (int32_t)live.size();
    q.prune_mb = prune_mb;
    q.fs_dfa = fs_dfa.empty() ? nullptr : d + dfa_off;
    // Asynchronous upload on the context's upload stream: a fill kernel
    // zeroes the group table, status and queue counters, and the descriptor
    // and block list are copied from pinned staging.  The first executions
    // wait for the event (see wait_uploads); nothing here blocks the host.
    const size_t stage_q = align_up(sizeof(DevQuery), 256);
    const size_t stage_dfa = align_up(stage_q + live.size() * 4, 256);
    p->staging = ctx->alloc_mem(stage_dfa + fs_dfa.size(), DPF_MEM_HOST_MAPPED);
    if (!p->staging) return bail(fail(DPF_ERR_OOM, "plan staging"));
    std::memcpy(p->staging, &q, sizeof q);
    if (!live.empty()) std::memcpy((uint8_t*)p->staging + stage_q, live.data(), live.size() * 4);
    if (!fs_dfa.empty()) std::memcpy((uint8_t*)p->staging + stage_dfa, fs_dfa.data(), fs_dfa.size());
    hipError_t e = launch_fill_i32((int32_t*)(d + agg_off), 0, (int64_t)((live_off - agg_off) / 4), ctx->upload);
    if (e == hipSuccess && !live.empty())
        e = hipMemcpyAsync(d + live_off, (uint8_t*)p->staging + stage_q, live.size() * 4, hipMemcpyHostToDevice,
                           ctx->upload);
    if (e == hipSuccess && !fs_dfa.empty())
        e = hipMemcpyAsync(d + dfa_off, (uint8_t*)p->staging + stage_dfa, fs_dfa.size(), hipMemcpyHostToDevice,
                           ctx->upload);
    if (e == hipSuccess) e = hipMemcpyAsync(p->dq, p->staging, sizeof q, hipMemcpyHostToDevice, ctx->upload);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p->uploaded, ctx->upload);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(ctx->upload);
        if (p->uploaded) (void)hipEventDestroy(p->uploaded);
        ctx->free_mem(p->staging, DPF_MEM_HOST_MAPPED);
        return bail(hip_fail(e, "plan upload"));
    }
    p->upload_pending = true;
    ctx->launches++;

    for (int i = 0; i < desc->ncols; ++i) { desc->cols[i]->refs++; p->cols.push_back(desc->cols[i]); }
    for (int j = 0; j < desc->nprobes; ++j) { desc->probes[j].hash->refs++; p->hashes.push_back(desc->probes[j].hash); }
    *out = p;
    return DPF_OK;
}

extern "C" dpf_status dpf_plan_footprint(dpf_plan plan, size_t* hbm_bytes) {
    if (!plan || !hbm_bytes) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    size_t b = plan->dmem_bytes + plan->frag_bytes;
    *hbm_bytes = b;
    return DPF_OK;
}

extern "C" dpf_status dpf_plan_blocks(dpf_plan plan, int64_t* scanned_blocks, int64_t* total_blocks) {
    if (!plan || !scanned_blocks || !total_blocks) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    *scanned_blocks = plan->nlive;
    *total_blocks = plan->nblocks;
    return DPF_OK;
}

extern "C" void dpf_plan_release(dpf_plan plan) {
    if (!plan) return;
    if (--plan->refs > 0) return;
    if (plan->uploaded) {
        (void)hipEventSynchronize(plan->uploaded);  // the staging copy may still be read
        (void)hipEventDestroy(plan->uploaded);
    }
    if (plan->staging) plan->ctx->free_mem(plan->staging, DPF_MEM_HOST_MAPPED);
    free_frag(plan);
    plan->ctx->free_mem(plan->dmem, DPF_MEM_HBM);
    plan->ctx->free_mem(plan->host_out, DPF_MEM_HOST_MAPPED);
    for (dpf_column c : plan->cols) dpf_column_release(c);
    for (dpf_hash h : plan->hashes) dpf_hash_release(h);
    delete plan;
}

// ---------------------------------------------------------------------------
// Execution
// ---------------------------------------------------------------------------
namespace {
dpf_status ensure_frag(dpf_plan p) {
    if (p->frag_ready) return DPF_OK;
    const DevQuery& q = p->hq;
    dpf_ctx ctx = p->ctx;
    auto get = [&](size_t bytes) -> void* {
        void* a = ctx->alloc_mem(bytes, DPF_MEM_HBM);
        if (a) {
            p->frag_allocs.push_back(a);
            p->frag_bytes += bytes;
        }
        return a;
    };
    FragBuffers& fb = p->fb;
    std::memset(&fb, 0, sizeof fb);
    const size_t n = (size_t)std::max<int64_t>(q.nrows, 1);
    bool needed[kMaxCols] = {};
    for (int i = 0; i < q.npreds; ++i) needed[q.preds[i].col] = true;
    for (int j = 0; j < q.nprobes; ++j) needed[q.probes[j].fk_col] = true;
    for (int l = 0; l < q.nloads; ++l) needed[q.loads[l].col] = true;
    for (int c = 0; c < q.ncols; ++c) {
        if (!needed[c]) continue;
        if (q.cols[c].enc == ENC_VARLEN || q.cols[c].enc == ENC_FSST) {
            fb.str_off[c] = (int64_t*)get((n + 1) * 8);
            fb.str_bytes[c] = (uint8_t*)get(q.cols[c].str_bytes + 64);
            DevCol* dc = (DevCol*)get(sizeof(DevCol));
            if (!fb.str_off[c] || !fb.str_bytes[c] || !dc) goto oom;
            DevCol mc = q.cols[c];
            mc.heap = fb.str_bytes[c];  // the string scan reads the materialised copy
            mc.heap_bytes = mc.str_bytes;
            mc.enc = ENC_VARLEN;
            if (hipMemcpy(dc, &mc, sizeof mc, hipMemcpyHostToDevice) != hipSuccess) goto oom;
            fb.str_col[c] = dc;
        } else {
            fb.dec[c] = (int64_t*)get(n * 8);
            if (!fb.dec[c]) goto oom;
        }
    }
    fb.flags = (uint8_t*)get(n);
    fb.rows[0] = (FragRow*)get(n * sizeof(FragRow));
    fb.rows[1] = (FragRow*)get(n * sizeof(FragRow));
    fb.counts = (unsigned long long*)get(64 * 8);
    if (!fb.flags || !fb.rows[0] || !fb.rows[1] || !fb.counts) goto oom;
    {
        int npay = 0;
        for (int j = 0; j < q.nprobes; ++j) npay += q.probes[j].h.npay;
        for (int s = 0; s < 2; ++s)
            for (int t = 0; t < npay; ++t) {
                fb.pay[s][t] = (int64_t*)get(n * 8);
                if (!fb.pay[s][t]) goto oom;
            }
    }
    p->frag_ready = true;
    return DPF_OK;
oom:
    free_frag(p);
    return fail(DPF_ERR_OOM, "fragmented-execution buffers");
}
}  // namespace

namespace {
// Where a fused launch keeps its scratch state: the work-queue counters and,
// per plan, the group table and the status word.  clear/clear_bytes: a
// region to zero (a fill kernel on the stream) before the launch.
struct FusedWorkspace {
    uint32_t* counters;
    int64_t* agg[kMaxBatch];
    uint32_t* status[kMaxBatch];
    void* clear;
    size_t clear_bytes;
};

// Orders each plan's execution after its upload: an upload still in flight
// is waited for on the stream (or, under stream capture, on the host, since
// a captured graph cannot depend on work outside it).  Once the event has
// completed the plan needs no wait again.
dpf_status wait_uploads(int32_t n, const dpf_plan* plans, hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    bool capturing = false;
    for (int i = 0; i < n; ++i) {
        dpf_plan p = plans[i];
        if (!p->upload_pending) continue;
        if (hipEventQuery(p->uploaded) == hipSuccess) {
            p->upload_pending = false;
            continue;
        }
        if (!capturing && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            capturing = true;
        if (capturing) {
            HIP_TRY(hipEventSynchronize(p->uploaded));
            p->upload_pending = false;
        } else {
            HIP_TRY(hipStreamWaitEvent(s, p->uploaded, 0));
        }
    }
    return DPF_OK;
}

dpf_status check_batch(dpf_ctx ctx, int32_t n, const dpf_plan* plans) {
    if (ctx->device < 0) return fail(DPF_ERR_INVALID_ARG, "execution needs a device context");
    if (n < 1) return fail(DPF_ERR_INVALID_ARG, "n must be >= 1");
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || plans[i]->ctx != ctx) return fail(DPF_ERR_INVALID_ARG, "bad plan handle");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(DPF_ERR_INVALID_ARG, "a plan appears twice in one execution");
    }
    return DPF_OK;
}

dpf_status check_fused_opts(int32_t n, const dpf_exec_opts& o) {
    if (n > kMaxBatch) return fail(DPF_ERR_UNSUPPORTED, "at most 64 plans per fused launch");
    if (o.rows_per_item && (o.rows_per_item < kMB || o.rows_per_item % kMB))
        return fail(DPF_ERR_INVALID_ARG, "rows_per_item: multiple of 256");
    return DPF_OK;
}

// One launch of the persistent fused kernel over n plans.
dpf_status launch_fused_batch(dpf_ctx ctx, int32_t n, const dpf_plan* plans, const dpf_exec_opts& o,
                              const FusedWorkspace& ws, hipStream_t s) {
    // LDS placement follows the requested budget (re-uploads the
    // descriptor only when the budget changes).  Auto: none for batches
    // of more than 8 plans, whose workgroups switch plans often and would
    // re-copy the tables at every switch (64-query mix: 2.83 -> 2.20 ms).
    const int32_t auto_lds = n > 8 ? 0 : kDefaultLdsHash;
    for (int i = 0; i < n; ++i) {
        dpf_plan p = plans[i];
        int32_t want = o.lds_hash_bytes < 0 ? auto_lds : o.lds_hash_bytes;
        if (p->lds_budget != want) {
            assign_lds(p, want);
            HIP_TRY(hipMemcpyAsync(p->dq, &p->hq, sizeof(DevQuery), hipMemcpyHostToDevice, s));
        }
    }
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.nq = n;
    a.counters = ws.counters;
    bool str = false, pend = false, fsst = false;
    int32_t shared = 0;
    int64_t total_mb = 0;
    for (int i = 0; i < n; ++i) {
        const DevQuery& q = plans[i]->hq;
        a.q[i] = plans[i]->dq;
        a.agg[i] = ws.agg[i];
        a.status[i] = ws.status[i];
        str |= q.has_str != 0;
        fsst |= q.fs_pred >= 0;
        pend |= q.npreds > 0 || q.nprobes > 0;
        a.agg_hash |= q.agg_hash;
        shared = std::max(shared, q.lds_shared);
        total_mb += q.live ? std::min<int64_t>(q.nmb, (int64_t)q.nlive * q.prune_mb) : q.nmb;
    }
    a.lds_shared = (int32_t)align_up((size_t)shared, 16);
    a.str_stage = fsst ? 2 : str ? 1 : 0;
    a.pend_stage = pend;
    auto lds_for = [&](int w) { return kLdsHeadBytes + (size_t)a.lds_shared + (size_t)w * fused_wave_area_bytes(str, pend); };
    // Waves per workgroup: large LDS-resident dimension tables are shared
    // by more waves (one copy per workgroup); otherwise small workgroups.
    int waves = o.waves_per_wg;
    if (waves == 0) {
        waves = 4;
        if (a.lds_shared >= 32 * 1024)
            for (int w : {16, 8})
                if ((int64_t)lds_for(w) <= ctx->lds_per_block) { waves = w; break; }
    }
    if (waves != 4 && waves != 8 && waves != 16) return fail(DPF_ERR_INVALID_ARG, "waves_per_wg: 4, 8 or 16");
    const size_t lds = lds_for(waves);
    if ((int64_t)lds > ctx->lds_per_block)
        return fail(DPF_ERR_UNSUPPORTED, "plan LDS needs exceed the workgroup limit; lower lds_hash_bytes");
    const int lds_cu = 160 * 1024;
    int wg = o.wg_per_cu;
    if (wg <= 0) wg = std::max(1, (str ? kTargetWavesPerCU : kTargetWavesPerCUNoStr) / waves);
    wg = std::max(1, std::min<int>(wg, (int)(lds_cu / lds)));
    int grid = std::max(1, ctx->ncu * wg);
    if (o.max_workgroups > 0) grid = std::min(grid, o.max_workgroups);
    // Work-item size: the caller's, else 64 mini blocks (16,384 rows),
    // shrunk for small batches so that every workgroup gets about three
    // items, but never below one mini block per wave.
    int64_t mb_per_item = o.rows_per_item / kMB;
    if (mb_per_item == 0) {
        mb_per_item = std::min<int64_t>(kDefaultMbPerItem, (total_mb + 3LL * grid - 1) / (3LL * grid));
        mb_per_item = std::max<int64_t>(mb_per_item, waves);  // total_mb is 0 when every block is pruned
        // a pruned plan's items are slices of its blocks: even slices
        for (int i = 0; i < n; ++i)
            if (plans[i]->hq.live) {
                const int64_t u = plans[i]->hq.prune_mb, k = (u + mb_per_item - 1) / mb_per_item;
                mb_per_item = (u + k - 1) / k;
                break;
            }
        mb_per_item = std::max<int64_t>(mb_per_item, waves);
    }
    a.mb_per_item = (int32_t)mb_per_item;
    int64_t items = 0;
    for (int i = 0; i < n; ++i) {
        a.item_start[i] = (int32_t)items;
        const DevQuery& q = plans[i]->hq;
        items += q.live ? (int64_t)q.nlive * ((q.prune_mb + mb_per_item - 1) / mb_per_item)
                        : (q.nmb + mb_per_item - 1) / mb_per_item;
    }
    if (items > INT32_MAX) return fail(DPF_ERR_UNSUPPORTED, "too many work items; raise rows_per_item");
    a.item_start[n] = (int32_t)items;
    // no more workgroups than items: an idle workgroup still claims and signs off
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, items));
    if (ws.clear_bytes) HIP_TRY(launch_fill_i32((int32_t*)ws.clear, 0, (int64_t)(ws.clear_bytes / 4), s));
    HIP_TRY(launch_fused(a, waves, grid, lds - kLdsStrTabBytes, s));  // the table is static LDS
    ctx->launches += ws.clear_bytes ? 2 : 1;
    return DPF_OK;
}

// The result handle of an execution; with_event records a completion event
// (not under stream capture) that dpf_result_release waits for.
dpf_status make_result(int32_t n, const dpf_plan* plans, hipStream_t s, bool with_event, dpf_result* out) {
    dpf_result r = new (std::nothrow) dpf_result_s();
    if (!r) return fail(DPF_ERR_OOM, "result");
    // Completion event for the release (not under graph capture, where the
    // caller owns the ordering of replays).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (with_event && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
        if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) r->done = nullptr;
        else if (hipEventRecord(r->done, s) != hipSuccess) {
            (void)hipEventDestroy(r->done);
            r->done = nullptr;
        }
    }
    for (int i = 0; i < n; ++i) {
        plans[i]->refs++;
        plans[i]->issued = true;
        r->plans.push_back(plans[i]);
    }
    r->rows.resize(n);
    r->ncols.assign(n, 0);
    r->read.assign(n, 0);
    *out = r;
    return DPF_OK;
}
}  // namespace

extern "C" dpf_status dpf_execute(dpf_ctx ctx, int32_t n, const dpf_plan* plans, const dpf_exec_opts* opts,
                                  dpf_stream stream, dpf_result* out) {
    if (!ctx || !plans || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    dpf_status st = check_batch(ctx, n, plans);
    if (st != DPF_OK) return st;
    dpf_exec_opts o{};
    o.lds_hash_bytes = -1;
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    st = wait_uploads(n, plans, s);
    if (st != DPF_OK) return st;
    if (o.mode == DPF_MODE_FRAGMENTED) {
        for (int i = 0; i < n; ++i) {
            dpf_plan p = plans[i];
            st = ensure_frag(p);
            if (st != DPF_OK) return st;
            int launched = run_fragmented(p->dq, p->hq, p->fb, s);
            if (launched < 0) return fail(DPF_ERR_HIP, "fragmented launch failed");
            ctx->launches += launched;
        }
    } else if (o.mode == DPF_MODE_FUSED) {
        st = check_fused_opts(n, o);
        if (st != DPF_OK) return st;
        // The plans' own workspaces: the first plan's queue counters, each
        // plan's group table and status word (zero between executions).
        FusedWorkspace ws{};
        ws.counters = plans[0]->counters;
        for (int i = 0; i < n; ++i) {
            ws.agg[i] = plans[i]->hq.agg;
            ws.status[i] = plans[i]->hq.status;
        }
        st = launch_fused_batch(ctx, n, plans, o, ws, s);
        if (st != DPF_OK) return st;
    } else {
        return fail(DPF_ERR_INVALID_ARG, "unknown execution mode");
    }
    return make_result(n, plans, s, true, out);
}

extern "C" dpf_status dpf_execute_noalloc(dpf_ctx ctx, int32_t n, const dpf_plan* plans, const dpf_exec_opts* opts,
                                          dpf_stream stream, dpf_result* out) {
    if (!ctx || !plans || !out) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    dpf_status st = check_batch(ctx, n, plans);
    if (st != DPF_OK) return st;
    dpf_exec_opts o{};
    o.lds_hash_bytes = -1;
    if (opts) o = *opts;
    if (o.mode != DPF_MODE_FUSED) return fail(DPF_ERR_UNSUPPORTED, "dpf_execute_noalloc runs the fused mode only");
    st = check_fused_opts(n, o);
    if (st != DPF_OK) return st;
    if (!ctx->scratch) return fail(DPF_ERR_HIP, "no static scratch address for this device");
    // Layout in the static array: the queue counters, then per plan a status
    // word and the group table, each on its own 256-byte boundary.
    FusedWorkspace ws{};
    size_t off = align_up((size_t)kCounterWords * 4, 256);
    ws.counters = (uint32_t*)ctx->scratch;
    for (int i = 0; i < n; ++i) {
        const DevQuery& q = plans[i]->hq;
        const size_t agg_bytes = agg_table_bytes(q);
        if (agg_bytes > kStaticScratchBytes) off = kStaticScratchBytes + 1;
        if (off > kStaticScratchBytes) break;
        ws.status[i] = (uint32_t*)(ctx->scratch + off);
        off += 256;
        ws.agg[i] = (int64_t*)(ctx->scratch + off);
        off = align_up(off + agg_bytes, 256);
    }
    if (off > kStaticScratchBytes)
        return fail(DPF_ERR_UNSUPPORTED, "the plans' group tables, status words and queue counters exceed the "
                                         "8 MiB static scratch of dpf_execute_noalloc; use dpf_execute");
    st = wait_uploads(n, plans, (hipStream_t)stream);
    if (st != DPF_OK) return st;
    // The array keeps the last call's contents: zero what this launch uses.
    ws.clear = ctx->scratch;
    ws.clear_bytes = off;
    st = launch_fused_batch(ctx, n, plans, o, ws, (hipStream_t)stream);
    if (st != DPF_OK) return st;
    return make_result(n, plans, (hipStream_t)stream, false, out);
}

extern "C" dpf_status dpf_result_get(dpf_result res, int32_t i, int64_t* ngroups, int32_t* ncols, const int64_t** rows) {
    if (!res || !ngroups || !ncols || !rows) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (i < 0 || i >= (int32_t)res->plans.size()) return fail(DPF_ERR_INVALID_ARG, "result index out of range");
    dpf_plan p = res->plans[i];
    const DevQuery& q = p->hq;
    const int64_t* h = p->host_out;
    const int64_t status = h[0];
    if (status & ST_CORRUPT) return fail(DPF_ERR_CORRUPT, "the kernel found a corrupt mini block");
    if (status & ST_CAPACITY) return fail(DPF_ERR_CAPACITY, "a device table ran out of capacity");
    if (status) return fail(DPF_ERR_CORRUPT, "device status " + std::to_string(status));
    const int64_t nrec = h[1];
    if (nrec < 0 || nrec > q.ngroups) return fail(DPF_ERR_CORRUPT, "bad record count");
    const int nk = q.nkeys;
    const int nout = nk + (int)p->outcols.size();
    {
        std::vector<int64_t>& out = res->rows[i];
        out.assign((size_t)nrec * nout, 0);
        for (int64_t r = 0; r < nrec; ++r) {
            const int64_t* rec = h + 2 + r * (1 + q.nacc);
            int64_t g = rec[0];
            int64_t* o = out.data() + r * nout;
            for (int k = 0; k < nk; ++k) {
                const KeyOut& K = p->keys[k];
                int64_t dk = (g / K.stride) % K.card;
                o[k] = K.dict ? K.dict[K.min + dk] : K.min + dk;
            }
            for (size_t c = 0; c < p->outcols.size(); ++c) o[nk + c] = rec[1 + p->outcols[c].first];
        }
        // canonical order: ascending by key tuple
        std::vector<int64_t> idx(nrec);
        for (int64_t r = 0; r < nrec; ++r) idx[r] = r;
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            return std::lexicographical_compare(out.begin() + a * nout, out.begin() + a * nout + nk,
                                                out.begin() + b * nout, out.begin() + b * nout + nk);
        });
        std::vector<int64_t> sorted((size_t)nrec * nout);
        for (int64_t r = 0; r < nrec; ++r)
            std::copy(out.begin() + idx[r] * nout, out.begin() + (idx[r] + 1) * nout, sorted.begin() + r * nout);
        out.swap(sorted);
        res->ncols[i] = nout;
        res->read[i] = 1;
    }
    *ngroups = nrec;
    *ncols = nout;
    *rows = res->rows[i].data();
    return DPF_OK;
}

// ---------------------------------------------------------------------------
// Measurement helper: read bandwidth from HBM or from pinned host memory
// ---------------------------------------------------------------------------
extern "C" dpf_status dpf_measure_read(dpf_ctx ctx, int32_t kind, size_t bytes, int32_t grid, int32_t reps,
                                       dpf_stream stream, float* ms) {
    if (!ctx || !ms) return fail(DPF_ERR_INVALID_ARG, "NULL argument");
    if (ctx->device < 0) return fail(DPF_ERR_INVALID_ARG, "measurement needs a device context");
    if (kind != DPF_MEM_HBM && kind != DPF_MEM_HOST_MAPPED) return fail(DPF_ERR_INVALID_ARG, "unknown memory kind");
    if (bytes < 16 || bytes % 16 || reps < 1 || reps > 1000 || grid < 0)
        return fail(DPF_ERR_INVALID_ARG, "bytes: a positive multiple of 16; reps: 1..1000; grid >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (grid == 0) grid = ctx->ncu * 8;
    uint8_t* buf = (uint8_t*)ctx->alloc_mem(bytes, kind);
    uint32_t* sink = (uint32_t*)ctx->alloc_mem(256, DPF_MEM_HBM);
    std::vector<hipEvent_t> ev((size_t)reps + 1, nullptr);
    dpf_status st = DPF_OK;
    const void* src = buf;
    if (!buf || !sink) {
        st = fail(DPF_ERR_OOM, "measurement buffer");
    } else if (kind == DPF_MEM_HOST_MAPPED) {
        std::memset(buf, 0x5A, bytes);
        src = ctx->device_ptr(buf);
        if (!src) st = fail(DPF_ERR_HIP, "hipHostGetDevicePointer(measurement buffer)");
    } else {
        hipError_t e = hipMemsetAsync(buf, 0x5A, bytes, s);
        if (e != hipSuccess) st = hip_fail(e, "hipMemsetAsync(measurement buffer)");
    }
    for (size_t i = 0; st == DPF_OK && i < ev.size(); ++i) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) { ev[i] = nullptr; st = hip_fail(e, "hipEventCreate"); }
    }
    if (st == DPF_OK) {
        hipError_t e = hipEventRecord(ev[0], s);
        for (int32_t r = 0; e == hipSuccess && r < reps; ++r) {
            e = launch_stream_read(src, bytes, 0x9E3779B9u, sink, grid, s);
            if (e == hipSuccess) e = hipEventRecord(ev[(size_t)r + 1], s);
            ctx->launches++;
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[(size_t)reps]);
        for (int32_t r = 0; e == hipSuccess && r < reps; ++r) e = hipEventElapsedTime(&ms[r], ev[(size_t)r], ev[(size_t)r + 1]);
        if (e != hipSuccess) st = hip_fail(e, "measurement launch");
    }
    (void)hipStreamSynchronize(s);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (buf) ctx->free_mem(buf, kind);
    if (sink) ctx->free_mem(sink, DPF_MEM_HBM);
    return st;
}

extern "C" void dpf_result_release(dpf_result res) {
    if (!res) return;
    if (res->done) {
        // the plans' memory may be recycled below: wait for the launch
        (void)hipEventSynchronize(res->done);
        (void)hipEventDestroy(res->done);
    }
    for (dpf_plan p : res->plans) dpf_plan_release(p);
    delete res;
}

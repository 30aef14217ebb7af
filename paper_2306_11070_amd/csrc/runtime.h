// Host runtime internals shared by the C ABI (api.cpp) and the request
// server (server.cpp): the context, batch plans, and small helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>

#include <utility>
#include <vector>

#include "common.h"

struct huff_ctx {
    int device = 0;
    int num_cus = 256;
    huff_params params{};
    huff::HistState* hist_st = nullptr;
    // encode tile workspaces, sized for tile_cap tiles
    uint16_t* tile_hist = nullptr;        // [tile_cap][256]
    uint32_t* tile_bits = nullptr;        // [tile_cap]
    uint32_t* tile_local = nullptr;       // [tile_cap]
    unsigned long long* blk_tail = nullptr;   // [tile_cap / 1024 + 1]
    unsigned long long* blk_carry = nullptr;  // [tile_cap / 1024 + 1]
    uint64_t tile_cap = 0;
    int32_t* status = nullptr;
    void* scratch = nullptr;  // this device's fixed workspace (huff_compress_noalloc)
    // kernel timing (huff_ctx_set_timing): event pairs per kernel id
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spans[HUFF_K_COUNT];
    std::vector<hipEvent_t> spare_events;
};

// A batch plan: device file tables and per-tile workspaces for a set of
// files.  Built by huff_batch_create (own allocations) or by the server
// (slices of its arena).
struct huff_batch {
    huff_ctx* ctx = nullptr;
    int device = 0;              // ctx's device (destroy may run after the context is gone)
    uint32_t nfiles = 0, chunk_size = 0, sub_size = 0;
    uint64_t ntiles = 0, nitems = 0;
    bool aligned = true;         // every input 16-byte aligned
    bool can_decode = false;     // every non-empty file has an output buffer
    huff::FileDesc* d_enc = nullptr;   // [nfiles], first = first tile
    huff::FileDesc* d_dec = nullptr;   // [nfiles], first = first decode lane (256-aligned)
    uint32_t* d_tile_file = nullptr;
    uint32_t* d_blk_file = nullptr;    // [nitems / kDecBatchBlock] decode block -> file, or null (search)
    uint8_t* d_blk_mode = nullptr;     // [nitems / kDecBatchBlock] 1: the block's codes pass the peek table
    uint16_t* d_tile_hist = nullptr;
    uint32_t* d_tile_local = nullptr;
    unsigned long long* d_blk_tail = nullptr;
    unsigned long long* d_blk_carry = nullptr;
    unsigned long long* d_file_hist = nullptr;  // [nfiles][256] histogram totals of a compress
    hipStream_t cap = nullptr;   // capture stream
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    bool owns = true;            // device tables were allocated by the plan
};

namespace huff {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
inline uint32_t log2u(uint64_t x) { return 63 - __builtin_clzll(x); }
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
// Device codebooks are read with 16-byte transfers: 16-byte alignment is required.
inline bool dcb_ok(const void* p) { return p && ((uintptr_t)p & 15u) == 0; }

inline huff_status hip_status(hipError_t e) { return e == hipSuccess ? HUFF_OK : HUFF_E_HIP; }

constexpr uint32_t kDecBatchBlock = 256;  // decode lanes per workgroup in batches (files start on a workgroup)

// Host-side tables of a batch plan.
struct BatchTables {
    std::vector<FileDesc> enc;       // first = first tile of the file
    std::vector<FileDesc> dec;       // first = first decode lane (kDecBatchBlock-aligned)
    std::vector<uint32_t> tile_file; // tile -> file
    std::vector<uint32_t> blk_file;  // block of kDecBatchBlock decode lanes -> file
    uint64_t ntiles = 0, nitems = 0;
    bool aligned = true;             // every input 16-byte aligned
    bool can_decode = true;          // every non-empty file has an output buffer
};

// Validates `files` and fills `t`.  HUFF_E_INVAL on a bad file or sizes.
// With decode_only the inputs (`in`) are not needed.
huff_status batch_tables(const huff_file* files, uint32_t nfiles, uint32_t chunk_size, uint32_t sub_size,
                         BatchTables& t, bool decode_only = false);
// Queues the launches of one batch operation on `s` (no allocation, no sync).
huff_status batch_launch(huff_batch* b, int op, hipStream_t s);
// Device bytes of a plan's per-tile workspaces for `ntiles` tiles.
uint64_t batch_workspace_bytes(uint64_t ntiles);

}  // namespace huff

// C ABI of the codec: argument checks, context workspaces, launch shapes.
// Every call validates before it launches and returns a huff_status.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "runtime.h"

using namespace huff;

namespace {


huff_params defaults(int num_cus) {
    huff_params p;
    // LDS lets four encode workgroups share a CU; a grid of one workgroup per
    // 16 KiB tile (what 256 per CU gives up to 1 GiB) beats a persistent one
    // (markov 1 GiB: 409 us against 432-447 us for four per CU)
    p.enc_blocks_per_cu = 256;
    p.hist_blocks = (uint32_t)num_cus * 16;  // 270 us against 284 us for four per CU
    p.hist_depth = 16;
    p.dec_block = 256;
    return p;
}

huff_status check_params(const huff_params& p) {
    if (p.enc_blocks_per_cu > 1024) return HUFF_E_INVAL;
    if (p.hist_depth && (!is_pow2(p.hist_depth) || p.hist_depth > (uint32_t)kHistMaxDepth)) return HUFF_E_INVAL;
    if (p.dec_block && (p.dec_block < 64 || p.dec_block > 256 || p.dec_block % 64)) return HUFF_E_INVAL;
    return HUFF_OK;
}

void merge_params(huff_params& dst, const huff_params& src) {
    if (src.hist_blocks) dst.hist_blocks = src.hist_blocks;
    if (src.hist_depth) dst.hist_depth = src.hist_depth;
    if (src.dec_block) dst.dec_block = src.dec_block;
    if (src.enc_blocks_per_cu) dst.enc_blocks_per_cu = src.enc_blocks_per_cu;
}

// Grows the per-tile workspaces to hold `tiles` tiles.  Waits for the
// device first: kernels queued earlier may still use the old buffers.
huff_status ensure_tiles(huff_ctx* ctx, uint64_t tiles) {
    if (tiles <= ctx->tile_cap) return HUFF_OK;
    uint64_t cap = std::max<uint64_t>(tiles, 4096);
    cap = std::max(cap, ctx->tile_cap * 2);
    if (hipDeviceSynchronize() != hipSuccess) return HUFF_E_HIP;
    (void)hipFree(ctx->tile_hist);
    (void)hipFree(ctx->tile_bits);
    (void)hipFree(ctx->tile_local);
    (void)hipFree(ctx->blk_tail);
    (void)hipFree(ctx->blk_carry);
    ctx->tile_hist = nullptr;
    ctx->tile_bits = ctx->tile_local = nullptr;
    ctx->blk_tail = ctx->blk_carry = nullptr;
    ctx->tile_cap = 0;
    const uint64_t blocks = cap / kScanTilesPerBlock + 1;
    if (hipMalloc(&ctx->tile_hist, cap * 256 * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&ctx->tile_bits, cap * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&ctx->tile_local, cap * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&ctx->blk_tail, blocks * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx->blk_carry, blocks * sizeof(unsigned long long)) != hipSuccess)
        return HUFF_E_NOMEM;
    ctx->tile_cap = cap;
    return HUFF_OK;
}

// Event pair around the launches made during its lifetime, kept per kernel
// id while the context's timing is on (huff_ctx_set_timing).  A stream being
// captured into a graph records nothing.
hipEvent_t take_event(huff_ctx* c) {
    if (!c->spare_events.empty()) {
        hipEvent_t e = c->spare_events.back();
        c->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

class KernelTimer {
public:
    KernelTimer(huff_ctx* c, int kernel, hipStream_t s) : c_(c), k_(kernel), s_(s) {
        if (!c_->timing) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        a_ = take_event(c_);
        if (a_ && hipEventRecord(a_, s_) != hipSuccess) {
            c_->spare_events.push_back(a_);
            a_ = nullptr;
        }
    }
    ~KernelTimer() {
        if (!a_) return;
        hipEvent_t b = take_event(c_);
        if (b && hipEventRecord(b, s_) == hipSuccess) {
            c_->spans[k_].push_back({a_, b});
            return;
        }
        c_->spare_events.push_back(a_);
        if (b) c_->spare_events.push_back(b);
    }
    KernelTimer(const KernelTimer&) = delete;
    KernelTimer& operator=(const KernelTimer&) = delete;

private:
    huff_ctx* c_;
    int k_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

void drop_spans(huff_ctx* c, int k) {
    for (auto& p : c->spans[k]) {
        c->spare_events.push_back(p.first);
        c->spare_events.push_back(p.second);
    }
    c->spans[k].clear();
}

}  // namespace

extern "C" {

const char* huff_strerror(huff_status s) {
    switch (s) {
        case HUFF_OK: return "ok";
        case HUFF_E_INVAL: return "invalid argument";
        case HUFF_E_CAPACITY: return "output buffer too small";
        case HUFF_E_CORRUPT: return "corrupt stream";
        case HUFF_E_NOMEM: return "out of device memory / over budget";
        case HUFF_E_AGAIN: return "pending";
        case HUFF_E_HIP: return "HIP runtime error";
        case HUFF_E_CODELEN: return "code longer than 63 bits";
        case HUFF_E_NOTFOUND: return "unknown ticket or handle";
        case HUFF_E_MISMATCH: return "result differs from the expected result";
        default: return "unknown status";
    }
}

huff_status huff_ctx_create(int device, const huff_params* params, huff_ctx** out) {
    if (!out) return HUFF_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HUFF_E_INVAL;
    DeviceGuard g(device);
    huff_ctx* c = new (std::nothrow) huff_ctx();
    if (!c) return HUFF_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    c->params = defaults(c->num_cus);
    if (params) {
        if (check_params(*params) != HUFF_OK) { delete c; return HUFF_E_INVAL; }
        merge_params(c->params, *params);
    }
    // the fixed workspace of huff_compress_noalloc: its address on this device
    // (looked up once per device; kept null if the lookup fails)
    if (scratch_address(device, &c->scratch) != hipSuccess) c->scratch = nullptr;
    bool ok = hipMalloc(&c->hist_st, sizeof(HistState)) == hipSuccess &&
              hipMalloc(&c->status, 256) == hipSuccess;
    if (ok) ok = hipMemset(c->hist_st, 0, sizeof(HistState)) == hipSuccess &&
                 hipMemset(c->status, 0, 256) == hipSuccess;
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (!ok) { huff_ctx_destroy(c); return HUFF_E_NOMEM; }
    *out = c;
    return HUFF_OK;
}

void huff_ctx_destroy(huff_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    if (c->hist_st) (void)hipFree(c->hist_st);
    (void)hipFree(c->tile_hist);
    (void)hipFree(c->tile_bits);
    (void)hipFree(c->tile_local);
    (void)hipFree(c->blk_tail);
    (void)hipFree(c->blk_carry);
    if (c->status) (void)hipFree(c->status);
    for (int k = 0; k < HUFF_K_COUNT; ++k) drop_spans(c, k);
    for (hipEvent_t e : c->spare_events) (void)hipEventDestroy(e);
    delete c;
}

huff_status huff_ctx_set_params(huff_ctx* c, const huff_params* p) {
    if (!c || !p || check_params(*p) != HUFF_OK) return HUFF_E_INVAL;
    merge_params(c->params, *p);
    return HUFF_OK;
}

huff_status huff_ctx_get_params(const huff_ctx* c, huff_params* out) {
    if (!c || !out) return HUFF_E_INVAL;
    *out = c->params;
    return HUFF_OK;
}

huff_status huff_ctx_set_timing(huff_ctx* c, int enable) {
    if (!c) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    if (!enable)
        for (int k = 0; k < HUFF_K_COUNT; ++k) drop_spans(c, k);
    c->timing = enable != 0;
    return HUFF_OK;
}

huff_status huff_ctx_kernel_time(huff_ctx* c, int kernel, double* total_ms, uint64_t* launches, int reset) {
    if (!c || kernel < 0 || kernel >= HUFF_K_COUNT || !total_ms || !launches) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    double sum = 0.0;
    for (auto& p : c->spans[kernel]) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            return HUFF_E_HIP;
        sum += ms;
    }
    *total_ms = sum;
    *launches = c->spans[kernel].size();
    if (reset) drop_spans(c, kernel);
    return HUFF_OK;
}

huff_status huff_ctx_status(huff_ctx* c, int32_t* out, int reset) {
    if (!c || !out) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    if (hipDeviceSynchronize() != hipSuccess) return HUFF_E_HIP;
    if (hipMemcpy(out, c->status, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return HUFF_E_HIP;
    if (reset && hipMemset(c->status, 0, sizeof(int32_t)) != hipSuccess) return HUFF_E_HIP;
    if (reset && hipDeviceSynchronize() != hipSuccess) return HUFF_E_HIP;
    return HUFF_OK;
}

namespace {
// Device workspaces of one compress or encode: the context's own (grown by
// ensure_tiles) or, for huff_compress_noalloc, slices of the fixed array.
struct Workspace {
    HistState* hist_st;
    uint16_t* tile_hist;
    uint32_t* tile_bits;
    uint32_t* tile_local;
    unsigned long long* blk_tail;
    unsigned long long* blk_carry;
};

Workspace ctx_workspace(huff_ctx* c) {
    return {c->hist_st, c->tile_hist, c->tile_bits, c->tile_local, c->blk_tail, c->blk_carry};
}

huff_status launch_hist_only(huff_ctx* c, HistState* hist_st, const uint8_t* d_in, uint64_t n, uint16_t* tile_hist,
                             hipStream_t s) {
    const uint64_t ntiles = (n + kEncTile - 1) / kEncTile;
    uint64_t blocks = std::min<uint64_t>(c->params.hist_blocks, ntiles);
    blocks = std::max<uint64_t>(blocks, (n >> 31) + 1);  // < 2^31 bytes per workgroup: u32 LDS counters
    const uint64_t tpb = (ntiles + blocks - 1) / blocks;
    blocks = (ntiles + tpb - 1) / tpb;
    HistArgs a;
    memset(&a, 0, sizeof(a));
    a.in = d_in;
    a.n = n;
    a.st = hist_st;
    a.tile_hist = tile_hist;
    a.depth_log2 = log2u(c->params.hist_depth);
    a.tiles_per_block = tpb;
    KernelTimer kt(c, HUFF_K_HIST, s);
    return hip_status(launch_histogram(a, (uint32_t)blocks, s));
}

huff_status check_encode_args(uint64_t n, const void* d_in, const void* d_words, const void* d_chunk_off,
                              uint32_t chunk_size, uint32_t sub_size, const void* d_sub_lo) {
    if (!d_chunk_off || n >= kMaxN) return HUFF_E_INVAL;
    if (!is_pow2(chunk_size) || chunk_size < 1024 || chunk_size > (64u << 20)) return HUFF_E_INVAL;
    if (sub_size && (!is_pow2(sub_size) || sub_size < 16 || sub_size > chunk_size || !d_sub_lo)) return HUFF_E_INVAL;
    if (n && (!d_in || !d_words)) return HUFF_E_INVAL;
    return HUFF_OK;
}

// Tile offsets (from the per-tile histograms when `from_hist`, else from a
// bit-counting pass over the input), then the encode itself.
huff_status launch_encode_one(huff_ctx* c, const Workspace& ws, const uint8_t* d_in, uint64_t n, const huff_dcb* d_cb,
                              uint32_t chunk_size, uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off,
                              uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status, bool from_hist, hipStream_t s) {
    if (n == 0) return hip_status(launch_encode_empty(d_chunk_off, sub_size ? d_sub_lo : nullptr, s));
    const uint64_t ntiles = (n + kEncTile - 1) / kEncTile;
    huff_status st = HUFF_OK;
    {
        // code bits per tile (from the tile histograms, or counted from the
        // input), then their scan
        KernelTimer kt(c, HUFF_K_SCAN, s);
        if (from_hist) {
            TileBitsArgs ta;
            memset(&ta, 0, sizeof(ta));
            ta.tile_hist = ws.tile_hist;
            ta.cb = d_cb;
            ta.ntiles = ntiles;
            ta.tile_bits = ws.tile_bits;
            ta.status = d_status;
            ta.err = c->status;
            st = hip_status(launch_tile_bits_hist(ta, s));
        } else {
            st = hip_status(launch_tile_bits(d_in, n, d_cb, ws.tile_bits, d_status, c->status, s));
        }
        if (st == HUFF_OK) {
            ScanArgs sa;
            memset(&sa, 0, sizeof(sa));
            sa.tile_bits = ws.tile_bits;
            sa.ntiles = ntiles;
            sa.tile_local = ws.tile_local;
            sa.blk_tail = ws.blk_tail;
            sa.blk_carry = ws.blk_carry;
            st = hip_status(launch_tile_scan(sa, s));
        }
    }
    if (st != HUFF_OK) return st;
    EncArgs a;
    memset(&a, 0, sizeof(a));
    a.files = nullptr;
    a.one.in = d_in;
    a.one.n = n;
    a.one.cb = d_cb;
    a.one.words = d_words;
    a.one.nwords = cap_words;
    a.one.chunk_off = d_chunk_off;
    a.one.sub_lo = sub_size ? d_sub_lo : nullptr;
    a.one.status = d_status;
    a.one.first = 0;
    a.nfiles = 1;
    a.chunk_log2 = log2u(chunk_size);
    a.sub_log2 = sub_size ? log2u(sub_size) : kNoSub;
    a.aligned = ((uintptr_t)d_in & 15u) == 0;
    a.ntiles = ntiles;
    a.tile_local = ws.tile_local;
    a.blk_carry = ws.blk_carry;
    a.err = c->status;
    const uint64_t grid = std::min<uint64_t>(ntiles, (uint64_t)c->num_cus * c->params.enc_blocks_per_cu);
    KernelTimer kt(c, HUFF_K_ENCODE, s);
    return hip_status(launch_encode(a, (uint32_t)grid, s));
}
}  // namespace

huff_status huff_histogram(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint64_t* d_hist, void* stream) {
    if (!c || !d_hist || (n && !d_in) || n >= kMaxN) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    hipStream_t s = as_stream(stream);
    if (n) {
        huff_status st = launch_hist_only(c, c->hist_st, d_in, n, nullptr, s);
        if (st != HUFF_OK) return st;
    }
    return hip_status(launch_hist_finalize(c->hist_st, d_hist, s));
}

// ---- host codebook: tie-ruled Huffman lengths, then canonical codes -------
huff_status huff_build_codebook(const uint64_t hist[256], huff_codebook* out) {
    if (!hist || !out) return HUFF_E_INVAL;
    memset(out, 0, sizeof(*out));
    // present bytes in (count, value) order
    uint16_t order[256];
    int k = 0;
    for (int v = 0; v < 256; ++v)
        if (hist[v]) order[k++] = (uint16_t)v;
    std::stable_sort(order, order + k, [&](uint16_t a, uint16_t b) { return hist[a] < hist[b]; });
    if (k == 1) out->len[order[0]] = 1;
    if (k >= 2) {
        // node ids: leaves 0..k-1 in that order, internal nodes k.. in creation order
        uint64_t w[511];
        uint16_t parent[511];
        for (int i = 0; i < k; ++i) w[i] = hist[order[i]];
        int leaf = 0, inner = k, made = k;
        auto take = [&]() -> int {
            const bool use_leaf = leaf < k && (inner == made || w[leaf] <= w[inner]);
            return use_leaf ? leaf++ : inner++;
        };
        for (int m = 0; m < k - 1; ++m) {
            const int a = take();
            const int b = take();
            w[made] = w[a] + w[b];
            parent[a] = parent[b] = (uint16_t)made;
            ++made;
        }
        uint16_t depth[511];
        const int root = made - 1;
        depth[root] = 0;
        for (int id = root - 1; id >= 0; --id) depth[id] = depth[parent[id]] + 1;
        for (int i = 0; i < k; ++i) {
            if (depth[i] > HUFF_MAX_CODE_LEN) { memset(out, 0, sizeof(*out)); return HUFF_E_CODELEN; }
            out->len[order[i]] = (uint8_t)depth[i];
        }
    }
    // canonical codes: per length, consecutive values in byte order
    uint32_t count[HUFF_MAX_CODE_LEN + 1] = {0};
    for (int v = 0; v < 256; ++v)
        if (out->len[v]) count[out->len[v]]++;
    uint64_t next[HUFF_MAX_CODE_LEN + 2] = {0};
    uint64_t code = 0;
    for (int l = 1; l <= HUFF_MAX_CODE_LEN; ++l) {
        code = (code + count[l - 1]) << 1;
        next[l] = code;
    }
    for (int v = 0; v < 256; ++v) {
        const uint8_t l = out->len[v];
        if (!l) continue;
        out->code[v] = next[l]++;
        out->nsym++;
        out->max_len = std::max<uint32_t>(out->max_len, l);
    }
    return HUFF_OK;
}

uint64_t huff_encoded_bits(const uint64_t hist[256], const huff_codebook* cb) {
    if (!hist || !cb) return 0;
    uint64_t t = 0;
    for (int v = 0; v < 256; ++v) t += hist[v] * cb->len[v];
    return t;
}

huff_status huff_build_codebook_device(huff_ctx* c, const uint64_t* d_hist, huff_dcb* d_cb, int32_t* d_status,
                                       void* stream) {
    if (!c || !d_hist || !dcb_ok(d_cb)) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    CbArgs a;
    memset(&a, 0, sizeof(a));
    a.hist = d_hist;
    a.out = d_cb;
    a.err = d_status ? d_status : c->status;
    a.from_lengths = 0;
    KernelTimer kt(c, HUFF_K_CODEBOOK, as_stream(stream));
    return hip_status(launch_codebook(a, 1, as_stream(stream)));
}

huff_status huff_codebook_upload(huff_ctx* c, const huff_codebook* cb, huff_dcb* d_cb, void* stream) {
    if (!c || !cb || !dcb_ok(d_cb)) return HUFF_E_INVAL;
    // lengths must describe a prefix code: Kraft sum <= 1, exactly
    unsigned __int128 kraft = 0;
    const unsigned __int128 one = (unsigned __int128)1 << HUFF_MAX_CODE_LEN;
    for (int v = 0; v < 256; ++v) {
        if (cb->len[v] > HUFF_MAX_CODE_LEN) return HUFF_E_CODELEN;
        if (cb->len[v]) kraft += one >> cb->len[v];
    }
    if (kraft > one) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    CbArgs a;
    memset(&a, 0, sizeof(a));
    a.out = d_cb;
    a.err = c->status;
    a.from_lengths = 1;
    memcpy(a.len, cb->len, 256);
    KernelTimer kt(c, HUFF_K_CODEBOOK, as_stream(stream));
    return hip_status(launch_codebook(a, 1, as_stream(stream)));
}

huff_status huff_encode(huff_ctx* c, const uint8_t* d_in, uint64_t n, const huff_dcb* d_cb, uint32_t chunk_size,
                        uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off, uint32_t sub_size,
                        uint32_t* d_sub_lo, int32_t* d_status, void* stream) {
    if (!c || !dcb_ok(d_cb)) return HUFF_E_INVAL;
    huff_status st = check_encode_args(n, d_in, d_words, d_chunk_off, chunk_size, sub_size, d_sub_lo);
    if (st != HUFF_OK) return st;
    DeviceGuard g(c->device);
    if (n) {
        st = ensure_tiles(c, (n + kEncTile - 1) / kEncTile);
        if (st != HUFF_OK) return st;
    }
    return launch_encode_one(c, ctx_workspace(c), d_in, n, d_cb, chunk_size, d_words, cap_words, d_chunk_off, sub_size,
                             d_sub_lo, d_status, false, as_stream(stream));
}

namespace {
// The compress path (histogram, device codebook, encode) over workspace ws.
huff_status compress_with(huff_ctx* c, const Workspace& ws, const uint8_t* d_in, uint64_t n, uint32_t chunk_size,
                          huff_dcb* d_cb, uint64_t* d_hist, uint32_t* d_words, uint64_t cap_words,
                          uint64_t* d_chunk_off, uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status,
                          hipStream_t s) {
    huff_status st = HUFF_OK;
    if (n) {
        st = launch_hist_only(c, ws.hist_st, d_in, n, ws.tile_hist, s);
        if (st != HUFF_OK) return st;
    }
    CbArgs a;
    memset(&a, 0, sizeof(a));
    a.acc = ws.hist_st;
    a.hist_out = d_hist;
    a.out = d_cb;
    a.err = d_status ? d_status : c->status;
    {
        KernelTimer kt(c, HUFF_K_CODEBOOK, s);
        st = hip_status(launch_codebook(a, 1, s));
    }
    if (st != HUFF_OK) return st;
    return launch_encode_one(c, ws, d_in, n, d_cb, chunk_size, d_words, cap_words, d_chunk_off, sub_size, d_sub_lo,
                             d_status, true, s);
}
}  // namespace

huff_status huff_compress(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint32_t chunk_size, huff_dcb* d_cb,
                          uint64_t* d_hist, uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off,
                          uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status, void* stream) {
    if (!c || !dcb_ok(d_cb)) return HUFF_E_INVAL;
    huff_status st = check_encode_args(n, d_in, d_words, d_chunk_off, chunk_size, sub_size, d_sub_lo);
    if (st != HUFF_OK) return st;
    DeviceGuard g(c->device);
    if (n) {
        st = ensure_tiles(c, (n + kEncTile - 1) / kEncTile);
        if (st != HUFF_OK) return st;
    }
    return compress_with(c, ctx_workspace(c), d_in, n, chunk_size, d_cb, d_hist, d_words, cap_words, d_chunk_off,
                         sub_size, d_sub_lo, d_status, as_stream(stream));
}

huff_status huff_compress_noalloc(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint32_t chunk_size, huff_dcb* d_cb,
                                  uint64_t* d_hist, uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off,
                                  uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status, void* stream) {
    if (!c || !dcb_ok(d_cb)) return HUFF_E_INVAL;
    if (n > HUFF_NOALLOC_MAX_N) return HUFF_E_INVAL;  // the fixed workspace holds at most this many bytes' tiles
    huff_status st = check_encode_args(n, d_in, d_words, d_chunk_off, chunk_size, sub_size, d_sub_lo);
    if (st != HUFF_OK) return st;
    if (!c->scratch) return HUFF_E_HIP;  // its address was not found when the context was created
    DeviceGuard g(c->device);
    hipStream_t s = as_stream(stream);
    const ScratchLayout& L = scratch_layout();
    uint8_t* base = static_cast<uint8_t*>(c->scratch);
    Workspace ws;
    ws.hist_st = reinterpret_cast<HistState*>(base + L.hist_st);
    ws.tile_hist = reinterpret_cast<uint16_t*>(base + L.tile_hist);
    ws.tile_bits = reinterpret_cast<uint32_t*>(base + L.tile_bits);
    ws.tile_local = reinterpret_cast<uint32_t*>(base + L.tile_local);
    ws.blk_tail = reinterpret_cast<unsigned long long*>(base + L.blk_tail);
    ws.blk_carry = reinterpret_cast<unsigned long long*>(base + L.blk_carry);
    // the accumulator must start at zero; whatever the previous call on this
    // device left there is cleared by a fill kernel (no memset node, so a
    // graph that captures this call replays correctly)
    st = hip_status(launch_fill_u64(reinterpret_cast<unsigned long long*>(ws.hist_st),
                                    sizeof(HistState) / sizeof(unsigned long long), 0ull, s));
    if (st != HUFF_OK) return st;
    return compress_with(c, ws, d_in, n, chunk_size, d_cb, d_hist, d_words, cap_words, d_chunk_off, sub_size, d_sub_lo,
                         d_status, s);
}

huff_status huff_decode(huff_ctx* c, const uint32_t* d_words, uint64_t nwords, const uint64_t* d_chunk_off,
                        uint64_t n, uint32_t chunk_size, const uint32_t* d_sub_lo, uint32_t sub_size,
                        const huff_dcb* d_cb, uint8_t* d_out, int32_t* d_status, void* stream) {
    if (!c || !dcb_ok(d_cb) || !d_chunk_off || n >= kMaxN) return HUFF_E_INVAL;
    if (!is_pow2(chunk_size) || chunk_size < 1024 || chunk_size > (64u << 20)) return HUFF_E_INVAL;
    if (sub_size && (!is_pow2(sub_size) || sub_size < 16 || sub_size > chunk_size || !d_sub_lo)) return HUFF_E_INVAL;
    if (n == 0) return HUFF_OK;
    if (!d_out || !d_words || ((uintptr_t)d_words & 15u)) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    const uint32_t item = sub_size ? sub_size : chunk_size;
    DecArgs a;
    memset(&a, 0, sizeof(a));
    a.files = nullptr;
    a.one.n = n;
    a.one.cb = d_cb;
    a.one.words = const_cast<uint32_t*>(d_words);
    a.one.nwords = nwords;
    a.one.chunk_off = const_cast<uint64_t*>(d_chunk_off);
    a.one.sub_lo = const_cast<uint32_t*>(d_sub_lo);
    a.one.out = d_out;
    a.one.status = d_status;
    a.one.first = 0;
    a.nfiles = 1;
    a.chunk_log2 = log2u(chunk_size);
    a.item_log2 = log2u(item);
    a.use_sub = sub_size ? 1 : 0;
    a.nitems = (n + item - 1) / item;
    a.err = c->status;
    KernelTimer kt(c, HUFF_K_DECODE, as_stream(stream));
    return hip_status(launch_decode(a, c->params.dec_block, ((uintptr_t)d_out & 15u) == 0, as_stream(stream)));
}

namespace {
huff_status check_bwt_args(uint64_t n, uint32_t block, uint32_t every) {
    if (n >= kMaxN || !is_pow2(block) || block < 1024 || block > HUFF_BWT_MAX_BLOCK) return HUFF_E_INVAL;
    if (!is_pow2(every) || every < 16 || every > block) return HUFF_E_INVAL;
    return HUFF_OK;
}
}  // namespace

huff_status huff_bwt(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint32_t block, uint32_t every, uint8_t* d_last,
                     uint16_t* d_rows, void* stream) {
    if (!c || check_bwt_args(n, block, every) != HUFF_OK || (n && (!d_in || !d_last || !d_rows))) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    return hip_status(launch_bwt(d_in, n, block, log2u(every), d_last, d_rows, as_stream(stream)));
}

huff_status huff_unbwt(huff_ctx* c, const uint8_t* d_last, uint64_t n, uint32_t block, uint32_t every,
                       const uint16_t* d_rows, uint8_t* d_out, int32_t* d_status, void* stream) {
    if (!c || check_bwt_args(n, block, every) != HUFF_OK || (n && (!d_last || !d_rows || !d_out))) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    return hip_status(launch_unbwt(d_last, n, block, log2u(every), d_rows, d_out, d_status ? d_status : c->status,
                                   as_stream(stream)));
}

huff_status huff_mtf(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint32_t block, uint8_t* d_out, void* stream) {
    if (!c || n >= kMaxN || !is_pow2(block) || block < 64 || block > (1u << 24) || (n && (!d_in || !d_out)))
        return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    return hip_status(launch_mtf(d_in, n, block, d_out, false, as_stream(stream)));
}

huff_status huff_unmtf(huff_ctx* c, const uint8_t* d_in, uint64_t n, uint32_t block, uint8_t* d_out, void* stream) {
    if (!c || n >= kMaxN || !is_pow2(block) || block < 64 || block > (1u << 24) || (n && (!d_in || !d_out)))
        return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    return hip_status(launch_mtf(d_in, n, block, d_out, true, as_stream(stream)));
}

huff_status huff_copy(huff_ctx* c, const void* d_src, void* d_dst, uint64_t bytes, void* stream) {
    if (!c || (bytes && (!d_src || !d_dst))) return HUFF_E_INVAL;
    if (bytes == 0) return HUFF_OK;
    if (((uintptr_t)d_src & 15u) || ((uintptr_t)d_dst & 15u)) return HUFF_E_INVAL;
    DeviceGuard g(c->device);
    return hip_status(launch_copy(d_src, d_dst, bytes, as_stream(stream)));
}

}  // extern "C"

extern "C" uint64_t huff_abi_sizeof(int which) {
    switch (which) {
        case 0: return sizeof(huff_dcb);
        case 1: return sizeof(huff_codebook);
        case 2: return sizeof(huff_params);
        case 3: return sizeof(huff_file);
        case 4: return sizeof(huff_server_cfg);
        case 5: return sizeof(huff_request);
        case 6: return sizeof(huff_result);
        case 7: return sizeof(huff_stream_info);
        default: return 0;
    }
}

// =============================================================== batches
namespace huff {

huff_status batch_tables(const huff_file* files, uint32_t nfiles, uint32_t chunk_size, uint32_t sub_size,
                         BatchTables& t, bool decode_only) {
    if (nfiles && !files) return HUFF_E_INVAL;
    if (!is_pow2(chunk_size) || chunk_size < 1024 || chunk_size > (64u << 20)) return HUFF_E_INVAL;
    if (sub_size && (!is_pow2(sub_size) || sub_size < 16 || sub_size > chunk_size)) return HUFF_E_INVAL;
    t.enc.assign(nfiles, FileDesc{});
    t.dec.assign(nfiles, FileDesc{});
    t.ntiles = t.nitems = 0;
    t.aligned = true;
    t.can_decode = true;
    const uint32_t item = sub_size ? sub_size : chunk_size;
    for (uint32_t i = 0; i < nfiles; ++i) {
        const huff_file& f = files[i];
        if (f.n >= kMaxN || !dcb_ok(f.cb) || !f.chunk_off || (sub_size && !f.sub_lo)) return HUFF_E_INVAL;
        if (f.n && ((!decode_only && !f.in) || !f.words || ((uintptr_t)f.words & 15u))) return HUFF_E_INVAL;
        if (f.n && decode_only && !f.out) return HUFF_E_INVAL;
        if (f.n && f.out && ((uintptr_t)f.out & 15u)) return HUFF_E_INVAL;
        if (f.n && !f.out) t.can_decode = false;
        if (f.n && ((uintptr_t)f.in & 15u)) t.aligned = false;
        FileDesc d;
        memset(&d, 0, sizeof(d));
        d.in = f.in;
        d.n = f.n;
        d.cb = f.cb;
        d.words = f.words;
        d.nwords = f.cap_words;
        d.chunk_off = f.chunk_off;
        d.sub_lo = sub_size ? f.sub_lo : nullptr;
        d.out = f.out;
        d.status = f.status;
        d.hist = f.hist;
        d.first = t.ntiles;
        t.enc[i] = d;
        d.first = t.nitems;
        t.dec[i] = d;
        t.ntiles += (f.n + kEncTile - 1) / kEncTile;
        const uint64_t items = (f.n + item - 1) / item;
        t.nitems += (items + kDecBatchBlock - 1) / kDecBatchBlock * kDecBatchBlock;
    }
    if (t.ntiles >= (1ull << 32)) return HUFF_E_INVAL;
    t.tile_file.resize(t.ntiles);
    for (uint32_t i = 0; i < nfiles; ++i) {
        const uint64_t t0 = t.enc[i].first, t1 = t0 + (files[i].n + kEncTile - 1) / kEncTile;
        for (uint64_t k = t0; k < t1; ++k) t.tile_file[k] = i;
    }
    t.blk_file.resize(t.nitems / kDecBatchBlock);
    for (uint32_t i = 0; i < nfiles; ++i) {
        const uint64_t b1 = i + 1 < nfiles ? t.dec[i + 1].first : t.nitems;
        for (uint64_t k = t.dec[i].first / kDecBatchBlock; k < b1 / kDecBatchBlock; ++k) t.blk_file[k] = i;
    }
    return HUFF_OK;
}

uint64_t batch_workspace_bytes(uint64_t ntiles) {
    const uint64_t nblk = ntiles / kScanTilesPerBlock + 1;
    return ntiles * (4 + 512 + 4) + nblk * 16;
}

huff_status batch_launch(huff_batch* b, int op, hipStream_t s) {
    huff_ctx* c = b->ctx;
    if (op == HUFF_OP_DECODE) {
        if (b->nitems == 0) return HUFF_OK;
        const uint32_t item = b->sub_size ? b->sub_size : b->chunk_size;
        DecArgs a;
        memset(&a, 0, sizeof(a));
        a.files = b->d_dec;
        a.nfiles = b->nfiles;
        a.chunk_log2 = log2u(b->chunk_size);
        a.item_log2 = log2u(item);
        a.use_sub = b->sub_size ? 1 : 0;
        a.nitems = b->nitems;
        a.err = c->status;
        a.blk_file = b->d_blk_file;
        if (b->d_blk_file && b->d_blk_mode) {
            // which of the two staged launches takes each block, read by both
            // with one load (the codebooks exist by now: built by a compress
            // earlier on the stream, or given)
            const hipError_t e = launch_blk_mode(b->d_blk_file, b->d_dec, b->d_blk_mode, b->nitems / kDecBatchBlock, s);
            if (e != hipSuccess) return HUFF_E_HIP;
            a.blk_mode = b->d_blk_mode;
        }
        return hip_status(launch_decode(a, kDecBatchBlock, true, s));
    }
    if (b->ntiles > 0) {
        // per-tile histograms of every file
        HistArgs h;
        memset(&h, 0, sizeof(h));
        h.files = b->d_enc;
        h.tile_file = b->d_tile_file;
        h.ntiles = b->ntiles;
        h.tile_hist = b->d_tile_hist;
        h.depth_log2 = log2u(c->params.hist_depth);
        if (op == HUFF_OP_COMPRESS && b->d_file_hist) {
            // every file's histogram, added up by the histogram launch
            h.file_hist = b->d_file_hist;
            huff_status st0 = hip_status(launch_fill_u64(b->d_file_hist, (uint64_t)b->nfiles * 256, 0, s));
            if (st0 != HUFF_OK) return st0;
        }
        uint64_t blocks = std::min<uint64_t>(c->params.hist_blocks, b->ntiles);
        const uint64_t tpb = (b->ntiles + blocks - 1) / blocks;
        h.tiles_per_block = tpb;
        blocks = (b->ntiles + tpb - 1) / tpb;
        huff_status st = hip_status(launch_histogram(h, (uint32_t)blocks, s));
        if (st != HUFF_OK) return st;
    }
    if (op == HUFF_OP_COMPRESS && b->nfiles) {
        // one codebook per file from its tiles' histograms (empty files too)
        CbArgs a;
        memset(&a, 0, sizeof(a));
        a.files = b->d_enc;
        a.tile_hist = b->d_tile_hist;
        a.file_hist = b->ntiles > 0 ? b->d_file_hist : nullptr;
        a.err = c->status;
        huff_status st = hip_status(launch_codebook(a, b->nfiles, s));
        if (st != HUFF_OK) return st;
    }
    if (b->ntiles == 0) return HUFF_OK;
    // tile bits into d_tile_local, scanned there in place
    TileBitsArgs ta;
    memset(&ta, 0, sizeof(ta));
    ta.tile_hist = b->d_tile_hist;
    ta.files = b->d_enc;
    ta.tile_file = b->d_tile_file;
    ta.ntiles = b->ntiles;
    ta.tile_bits = b->d_tile_local;
    ta.err = c->status;
    huff_status st = hip_status(launch_tile_bits_hist(ta, s));
    if (st != HUFF_OK) return st;
    ScanArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.tile_bits = b->d_tile_local;
    sa.files = b->d_enc;
    sa.tile_file = b->d_tile_file;
    sa.ntiles = b->ntiles;
    sa.tile_local = b->d_tile_local;
    sa.blk_tail = b->d_blk_tail;
    sa.blk_carry = b->d_blk_carry;
    st = hip_status(launch_tile_scan(sa, s));  // block scans, then the carries across blocks
    if (st != HUFF_OK) return st;
    EncArgs e;
    memset(&e, 0, sizeof(e));
    e.files = b->d_enc;
    e.nfiles = b->nfiles;
    e.aligned = b->aligned ? 1u : 0u;
    e.chunk_log2 = log2u(b->chunk_size);
    e.sub_log2 = b->sub_size ? log2u(b->sub_size) : kNoSub;
    e.ntiles = b->ntiles;
    e.tile_file = b->d_tile_file;
    e.tile_local = b->d_tile_local;
    e.blk_carry = b->d_blk_carry;
    e.err = c->status;
    const uint64_t grid = std::min<uint64_t>(b->ntiles, (uint64_t)c->num_cus * c->params.enc_blocks_per_cu);
    return hip_status(launch_encode(e, (uint32_t)grid, s));
}

}  // namespace huff

namespace {
void batch_free(huff_batch* b) {
    for (int i = 0; i < 3; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->owns) {
        (void)hipFree(b->d_enc);
        (void)hipFree(b->d_dec);
        (void)hipFree(b->d_tile_file);
        (void)hipFree(b->d_blk_file);
        (void)hipFree(b->d_blk_mode);
        (void)hipFree(b->d_tile_hist);
        (void)hipFree(b->d_tile_local);
        (void)hipFree(b->d_blk_tail);
        (void)hipFree(b->d_blk_carry);
        (void)hipFree(b->d_file_hist);
    }
    delete b;
}
}  // namespace

extern "C" {

huff_status huff_batch_create(huff_ctx* c, const huff_file* files, uint32_t nfiles, uint32_t chunk_size,
                              uint32_t sub_size, huff_batch** out) {
    if (!out) return HUFF_E_INVAL;
    *out = nullptr;
    if (!c) return HUFF_E_INVAL;
    BatchTables t;
    const huff_status vst = batch_tables(files, nfiles, chunk_size, sub_size, t);
    if (vst != HUFF_OK) return vst;
    DeviceGuard g(c->device);
    huff_batch* b = new (std::nothrow) huff_batch();
    if (!b) return HUFF_E_NOMEM;
    b->ctx = c;
    b->device = c->device;
    b->nfiles = nfiles;
    b->chunk_size = chunk_size;
    b->sub_size = sub_size;
    b->ntiles = t.ntiles;
    b->nitems = t.nitems;
    b->can_decode = t.can_decode;
    b->aligned = t.aligned;
    const uint64_t ntiles = t.ntiles;
    const uint64_t nblk = ntiles / kScanTilesPerBlock + 1;
    const size_t fbytes = std::max<size_t>(1, nfiles) * sizeof(FileDesc);
    bool ok = hipMalloc(&b->d_enc, fbytes) == hipSuccess && hipMalloc(&b->d_dec, fbytes) == hipSuccess &&
              hipMalloc(&b->d_tile_file, std::max<uint64_t>(1, ntiles) * 4) == hipSuccess &&
              hipMalloc(&b->d_tile_hist, std::max<uint64_t>(1, ntiles) * 512) == hipSuccess &&
              hipMalloc(&b->d_tile_local, std::max<uint64_t>(1, ntiles) * 4) == hipSuccess &&
              hipMalloc(&b->d_blk_tail, nblk * 8) == hipSuccess && hipMalloc(&b->d_blk_carry, nblk * 8) == hipSuccess &&
              hipMalloc(&b->d_file_hist, std::max<size_t>(1, nfiles) * 2048) == hipSuccess &&
              hipMalloc(&b->d_blk_file, std::max<size_t>(1, t.blk_file.size()) * 4) == hipSuccess &&
              hipMalloc(&b->d_blk_mode, std::max<size_t>(1, t.blk_file.size())) == hipSuccess;
    if (!ok) { batch_free(b); return HUFF_E_NOMEM; }
    if ((nfiles && (hipMemcpy(b->d_enc, t.enc.data(), nfiles * sizeof(FileDesc), hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(b->d_dec, t.dec.data(), nfiles * sizeof(FileDesc), hipMemcpyHostToDevice) != hipSuccess)) ||
        (ntiles && hipMemcpy(b->d_tile_file, t.tile_file.data(), ntiles * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        (!t.blk_file.empty() &&
         hipMemcpy(b->d_blk_file, t.blk_file.data(), t.blk_file.size() * 4, hipMemcpyHostToDevice) != hipSuccess)) {
        batch_free(b);
        return HUFF_E_HIP;
    }
    *out = b;
    return HUFF_OK;
}

void huff_batch_destroy(huff_batch* b) {
    if (!b) return;
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
}

huff_status huff_batch_run(huff_batch* b, int op, int use_graph, void* stream) {
    if (!b || op < HUFF_OP_COMPRESS || op > HUFF_OP_DECODE) return HUFF_E_INVAL;
    if (op == HUFF_OP_DECODE && !b->can_decode) return HUFF_E_INVAL;  // a non-empty file has no output buffer
    DeviceGuard g(b->device);
    hipStream_t s = as_stream(stream);
    if (!use_graph) return batch_launch(b, op, s);
    if (!b->exec[op]) {
        if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return HUFF_E_HIP;
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return HUFF_E_HIP;
        const huff_status st = batch_launch(b, op, b->cap);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &gr);
        if (st != HUFF_OK || e != hipSuccess || !gr) {
            if (gr) (void)hipGraphDestroy(gr);
            return st != HUFF_OK ? st : HUFF_E_HIP;
        }
        if (hipGraphInstantiate(&b->exec[op], gr, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(gr);
            b->exec[op] = nullptr;
            return HUFF_E_HIP;
        }
        b->graph[op] = gr;
    }
    return hip_status(hipGraphLaunch(b->exec[op], s));
}

huff_status huff_compress_batch(huff_batch* b, void* stream) { return huff_batch_run(b, HUFF_OP_COMPRESS, 0, stream); }
huff_status huff_encode_batch(huff_batch* b, void* stream) { return huff_batch_run(b, HUFF_OP_ENCODE, 0, stream); }
huff_status huff_decode_batch(huff_batch* b, void* stream) { return huff_batch_run(b, HUFF_OP_DECODE, 0, stream); }

}  // extern "C"

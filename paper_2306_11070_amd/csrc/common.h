// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "huff.h"

namespace huff {

constexpr int kEncThreads = 256;                 // encode workgroup
constexpr int kEncUnit = 64;                     // input bytes per encode thread
constexpr int kEncTile = kEncThreads * kEncUnit; // 16 KiB per tile
constexpr int kCbThreads = 256;                  // codebook workgroup (one per file)
constexpr int kHistThreads = 512;
constexpr int kScanTilesPerBlock = 1024;         // tiles per k_tile_scan block
constexpr int kHistMaxDepth = 32;
constexpr uint32_t kNoSub = 0xFFFFFFFFu;         // sub_log2 when there is no sub index
constexpr uint64_t kMaxN = 1ull << 38;

// Histogram accumulator (device).  Workgroup w adds into copy
// w % kHistCopies, which spreads same-address atomics; the kernel that
// consumes the counts (finalize or codebook) sums the copies and zeroes them
// for the next launch.
constexpr int kHistCopies = 16;
struct HistState {
    unsigned long long acc[kHistCopies][256];
};

// One stream / file as the kernels see it.  Single calls pass one by value;
// batched calls pass a device table sorted by the first-work-item fields.
struct FileDesc {
    const uint8_t* in;        // encode input / decode: unused
    uint64_t n;               // bytes
    const huff_dcb* cb;       // codebook read by encode / decode
    uint32_t* words;          // encode output / decode input
    uint64_t nwords;          // encode: capacity; decode: valid words
    uint64_t* chunk_off;      // nchunks + 1
    uint32_t* sub_lo;         // nsub + 1 or null
    uint8_t* out;             // decode output
    int32_t* status;          // per-file status word (may be null)
    uint64_t* hist;           // batch codebook: optional histogram output
    uint64_t first;           // first global work item (tile / sub-block) of this file
};

struct EncArgs {
    const FileDesc* files;  // null: single file in `one`
    FileDesc one;
    uint32_t nfiles;
    uint32_t chunk_log2;
    uint32_t sub_log2;      // kNoSub if no sub index
    uint32_t aligned;       // every input is 16-byte aligned
    uint64_t ntiles;        // total over all files
    const uint32_t* tile_file;             // batch: file index of every tile
    const uint32_t* tile_local;            // tile's first bit inside its scan block (and, batch, its file)
    const unsigned long long* blk_carry;   // bits of the file open at a block's start, before the block
    int32_t* err;           // fallback status word
    uint32_t split;         // set by launch_encode: 1 a single stream, 2 a batch, split between the compact kernel
                            // (codes of at most kEncCompactMaxLen bits) and the full kernel (longer codes)
};

// Tile offsets are a scan in two levels.  A short stream: k_tile_scan scans
// the tiles of each 1024-tile block and sums the bits of all earlier tiles
// into the block's carry.  A batch, or a longer stream (one segment):
// k_tile_scan_seg scans each block restarting at every file, and k_blk_scan
// carries the open file's running total from block to block; blk_tail packs,
// per block, the bits of its last segment (low 62 bits) with two flags.
// launch_tile_scan queues both levels.
constexpr unsigned long long kTailStarts = 1ull << 63;  // the block's last segment starts inside the block
constexpr unsigned long long kTailHead = 1ull << 62;    // a file starts at the block's first tile
constexpr unsigned long long kTailBits = kTailHead - 1;

// Per-tile code bits from the per-tile histograms (k_tile_bits_hist).
struct TileBitsArgs {
    const uint16_t* tile_hist;  // [ntiles][256] u16 counts
    const huff_dcb* cb;         // single file: its codebook
    const FileDesc* files;      // batch: file table (codebook per file) ...
    const uint32_t* tile_file;  // ... and file index of every tile
    uint64_t ntiles;
    uint32_t* tile_bits;        // out: code bits of each tile
    int32_t* status;            // single file: its status word (or null) ...
    int32_t* err;               // ... fallback: the context's (batch: files[i].status, else this)
};

struct ScanArgs {
    const uint32_t* tile_bits;  // code bits of each tile
    const FileDesc* files;      // batch: file table ...
    const uint32_t* tile_file;  // ... and file index of every tile
    uint64_t ntiles;
    uint32_t* tile_local;
    unsigned long long* blk_tail;   // last segment of each block, with flags (segmented scan)
    unsigned long long* blk_carry;  // out: bits of the open segment before each block
};

struct DecArgs {
    const FileDesc* files;
    FileDesc one;
    uint32_t nfiles;
    uint32_t chunk_log2;
    uint32_t item_log2;     // log2 of bytes per decode lane (sub_size or chunk_size)
    uint32_t use_sub;       // 1: start bits from sub_lo, else from chunk_off
    uint64_t nitems;        // total lanes over all files (files padded to whole blocks)
    int32_t* err;
    const uint32_t* blk_file;  // batch, optional: file of every block of 256 lanes (else a search over `files`)
    const uint8_t* blk_mode;   // batch, optional: 1 where a block's codebook has codes past its peek table
};

struct HistArgs {
    const uint8_t* in;          // single input ...
    uint64_t n;
    const FileDesc* files;      // ... or a batch: file table, tile -> file map, tile count
    const uint32_t* tile_file;
    uint64_t ntiles;
    HistState* st;
    uint16_t* tile_hist;    // optional per-16 KiB-tile histograms, [ntiles][256]
    uint32_t depth_log2;
    uint64_t tiles_per_block;
    unsigned long long* file_hist;  // batch, optional: [nfiles][256] totals, added to (cleared by the caller)
};

struct CbArgs {
    const FileDesc* files;      // batch: one workgroup per file, histogram summed from ...
    const uint16_t* tile_hist;  // ... the per-tile histograms (or their totals, file_hist); output into files[i].cb
    const unsigned long long* file_hist;  // batch, optional: [nfiles][256] histograms
    const uint64_t* hist;   // histogram input (from-histogram mode) ...
    HistState* acc;         // ... or the histogram accumulator, summed and zeroed here
    uint64_t* hist_out;     // optional copy of the summed histogram (accumulator mode)
    huff_dcb* out;
    int32_t* err;
    uint32_t from_lengths;
    uint8_t len[256];
};

// One result check of the request server: `bytes` bytes at `got` against
// `want`, and (got_bits non-null) the stream length *got_bits against
// want_bits; a difference sets *status to HUFF_E_MISMATCH.
struct CmpJob {
    const uint8_t* got;
    const uint8_t* want;
    uint64_t bytes;
    const uint64_t* got_bits;
    uint64_t want_bits;
    int32_t* status;
    uint32_t first_block;  // the job's first workgroup of the launch (set by launch_compare's caller)
    uint32_t nblocks;      // and how many it has
};

// The fixed device workspace of huff_compress_noalloc (kernels.hip): byte
// offsets of its parts, sized for HUFF_NOALLOC_MAX_N input bytes.
struct ScratchLayout {
    uint64_t hist_st, tile_hist, tile_bits, tile_local, blk_tail, blk_carry, bytes;
};
const ScratchLayout& scratch_layout();
// Address of the workspace on `device` (looked up on the first call for each
// device, with that device current).
hipError_t scratch_address(int device, void** out);

// Launchers (kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_histogram(const HistArgs& a, uint32_t blocks, hipStream_t s);
hipError_t launch_hist_finalize(HistState* st, uint64_t* out, hipStream_t s);
hipError_t launch_codebook(const CbArgs& a, uint32_t nblocks, hipStream_t s);
hipError_t launch_tile_bits(const uint8_t* in, uint64_t n, const huff_dcb* cb, uint32_t* tile_bits, int32_t* status,
                            int32_t* err, hipStream_t s);
hipError_t launch_tile_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_tile_bits_hist(const TileBitsArgs& a, hipStream_t s);
hipError_t launch_blk_scan(const unsigned long long* blk_tail, unsigned long long* blk_carry, uint64_t nblk,
                           hipStream_t s);
hipError_t launch_encode(const EncArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_encode_empty(uint64_t* chunk_off, uint32_t* sub_lo, hipStream_t s);
// out_aligned: every output is 16-byte aligned (the staged decoder requires it)
hipError_t launch_decode(const DecArgs& a, uint32_t block, bool out_aligned, hipStream_t s);
// Fills mode[b] for the nblk decode blocks of a batch (from blk_file and the files' codebooks).
hipError_t launch_blk_mode(const uint32_t* blk_file, const FileDesc* files, uint8_t* mode, uint64_t nblk,
                           hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);
hipError_t launch_gather_u64(const uint64_t* const* src, uint64_t* dst, uint32_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s);
// Workgroups a compare job of `bytes` bytes takes (first_block / nblocks).
uint32_t compare_blocks(uint64_t bytes);
hipError_t launch_compare(const CmpJob* jobs, uint32_t njobs, uint32_t total_blocks, hipStream_t s);
// Method 3's block transform (bwt.hip).
hipError_t launch_bwt(const uint8_t* in, uint64_t n, uint32_t block, uint32_t every_log2, uint8_t* last,
                      uint16_t* rows, hipStream_t s);
hipError_t launch_unbwt(const uint8_t* last, uint64_t n, uint32_t block, uint32_t every_log2, const uint16_t* rows,
                        uint8_t* out, int32_t* status, hipStream_t s);
hipError_t launch_mtf(const uint8_t* in, uint64_t n, uint32_t block, uint8_t* out, bool inverse, hipStream_t s);

}  // namespace huff

// HIP kernels of the Huffman codec for gfx950 (CDNA4, wave64).
//
//   k_hist            byte histogram over 16 KiB tiles: replicated LDS
//                     counters, a u16 histogram per tile (what the tile
//                     offsets come from), totals added into accumulator
//                     copies that the consumer sums and clears.
//   k_hist_finalize   sums the accumulator copies (histogram-only calls).
//   k_codebook        tie-ruled Huffman code lengths, canonical codes and
//                     decode tables, one workgroup per file.
//   k_tile_bits_hist  code bits of each tile from its histogram.
//   k_tile_scan       exclusive scan of the tile bits (block carries summed in
//                     the same launch up to eight scan blocks);
//   k_tile_scan_seg,  otherwise, or per file in a batch: segmented block scans
//   k_blk_scan        and a scan of the block totals with resets.
//   k_encode          one workgroup per tile: per-thread code packing, a
//                     workgroup scan of the bit counts, words assembled in LDS
//                     and stored coalesced, segment and decode index entries.
//   k_decode_lds      one lane per sub-block, the wave's stream staged in LDS,
//                     table-driven decode, bytes stored through LDS.
//   k_decode          one lane per sub-block or chunk read from memory.
//   k_copy            plain copy, the bandwidth probe and counter calibration.
//   k_compare         device comparison of results with expected bytes.
#include "common.h"

#include <mutex>
#include <type_traits>

namespace huff {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int l = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (l >= d) x += y;
    }
    return x;
}

// Inclusive prefix sum of a u64 across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)x, d, 64), hi = __shfl_up((uint32_t)(x >> 32), d, 64);
        if (lane >= (uint32_t)d) x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wave (it is a workgroup
// release/acquire on all memory), which would drain the next tile's prefetch
// and the current tile's stores at each barrier.  Used where the threads of
// a workgroup share data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders the LDS accesses of one wave: what its lanes wrote before is seen
// by all of its lanes after.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, d, 64);
        uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

__device__ __forceinline__ uint32_t byte_of(const uint4& x, int i) {
    const uint32_t w = i < 4 ? x.x : i < 8 ? x.y : i < 12 ? x.z : x.w;
    return (w >> (8 * (i & 3))) & 0xffu;
}

__device__ __forceinline__ void report(int32_t* primary, int32_t* fallback, int32_t code) {
    atomicMin(primary ? primary : fallback, code);
}

__device__ __forceinline__ uint32_t find_file(const FileDesc* files, uint32_t nfiles, uint64_t item) {
    // last file whose first work item is <= item (files sorted by `first`)
    uint32_t lo = 0, hi = nfiles - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (files[mid].first <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// File of decode lane `item` of a batch (files start on a block of 256
// lanes): one read of the block table when the plan has one.
__device__ __forceinline__ uint32_t dec_file(const DecArgs& a, uint64_t item) {
    return a.blk_file ? a.blk_file[item >> 8] : find_file(a.files, a.nfiles, item);
}

// ============================================================== histogram
__device__ __forceinline__ uint32_t byte32(const uint4& x0, const uint4& x1, int i) {
    return i < 16 ? byte_of(x0, i) : byte_of(x1, i - 16);
}

// Unaligned-safe 16-byte load; bytes at or past n read as zero.
__device__ __forceinline__ uint4 load16(const uint8_t* in, uint64_t q, uint64_t n, bool aligned) {
    if (aligned && q + 16 <= n) return *reinterpret_cast<const uint4*>(in + q);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t b = q + i < n ? (uint32_t)in[q + i] : 0u;
        const uint32_t sh = 8 * (i & 3);
        if (i < 4) w0 |= b << sh;
        else if (i < 8) w1 |= b << sh;
        else if (i < 12) w2 |= b << sh;
        else w3 |= b << sh;
    }
    return make_uint4(w0, w1, w2, w3);
}

// Persistent histogram over 16 KiB tiles (the encode tile).  Workgroup b
// takes a contiguous run of tiles; each thread counts 2 x 16 bytes per tile
// into LDS replicas laid out [value][replica] (the lanes of a wave hit
// different banks), with the next tile's loads issued before the current
// tile is counted.  With a tile_hist buffer the replicas are flushed after
// every tile into a u16 per-tile histogram (what the encoder's tile offsets
// are computed from).  Each workgroup adds its totals into accumulator copy
// b % kHistCopies; the consumer sums and zeroes the copies.
//
// Batched (kBatch): the tiles of all files form one sequence (a tile belongs
// to one file, tile_file maps it); only per-tile histograms are written, the
// per-file totals are summed from them by the codebook kernel.
template <bool kBatch>
__global__ __launch_bounds__(kHistThreads) void k_hist(HistArgs a) {
    __shared__ uint32_t sh[256 * kHistMaxDepth];
    const uint32_t dl = a.depth_log2, depth = 1u << dl;
    const uint32_t tid = threadIdx.x;
    // with per-tile histograms and room for two replica sets, tiles count into
    // the sets in turn: a set is read after its tile while the next tile
    // counts into the other one, so a tile needs one barrier, not two
    const bool dbl = a.tile_hist != nullptr && 2 * depth <= (uint32_t)kHistMaxDepth;
    for (uint32_t i = tid; i < (dbl ? 512u : 256u) * depth; i += kHistThreads) sh[i] = 0;
    const uint32_t rep = tid & (depth - 1);
    // reading a value's replicas: thread tid's row starts at bank
    // (tid * depth) mod 32, shared by the 32/depth-apart threads of a half
    // wave; starting each of them at a different replica makes the 32 reads
    // of a half wave fall on 32 different banks
    const uint32_t rot = dl <= 5 ? tid >> (5 - dl) : tid;
    uint32_t* set = sh;
    const uint64_t ntiles = kBatch ? a.ntiles : (a.n + kEncTile - 1) / kEncTile;
    const uint64_t t0 = (uint64_t)blockIdx.x * a.tiles_per_block;
    const uint64_t t1 = min(ntiles, t0 + a.tiles_per_block);
    // tile t's bytes: in[base .. min(base + kEncTile, n))
    struct Src {
        const uint8_t* in;
        uint64_t n, base;
    };
    auto src = [&](uint64_t t) -> Src {
        if constexpr (kBatch) {
            const FileDesc& d = a.files[a.tile_file[t]];
            return {d.in, d.n, (t - d.first) * (uint64_t)kEncTile};
        } else {
            return {a.in, a.n, t * (uint64_t)kEncTile};
        }
    };
    // counter of value b in this thread's replica: one shift-add per byte
    // from the replica's column base
    uint32_t* col = set + rep;
    auto count = [&](uint32_t b) { atomicAdd(col + (b << dl), 1u); };
    auto count4 = [&](uint32_t w) {
        count(w & 0xffu);
        count((w >> 8) & 0xffu);
        count((w >> 16) & 0xffu);
        count(w >> 24);
    };
    auto count16 = [&](const uint4 q, uint64_t at, uint64_t n) {
        if (at + 16 <= n) {
            count4(q.x); count4(q.y); count4(q.z); count4(q.w);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (at + i < n) count(byte_of(q, i));
        }
    };
    auto load2 = [&](const Src& sr, uint4& y0, uint4& y1) {
        const bool al = ((uintptr_t)sr.in & 15u) == 0;
        const uint64_t off = (uint64_t)tid * 16;
        y0 = load16(sr.in, sr.base + off, sr.n, al);
        y1 = load16(sr.in, sr.base + kEncTile / 2 + off, sr.n, al);
    };
    unsigned long long total = 0;
    uint32_t run = 0, run2 = 0;  // with tile_hist: each set's sum for byte value tid after its previous tile
    uint32_t curFile = 0xffffffffu;  // batch with file_hist: the file whose totals `total` holds
    const uint64_t off = (uint64_t)tid * 16;
    uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
    Src cur = {nullptr, 0, 0};
    if (t0 < t1) {
        cur = src(t0);
        load2(cur, q0, q1);
    }
    __syncthreads();
    for (uint64_t t = t0; t < t1; ++t) {
        const uint4 c0 = q0, c1 = q1;
        const Src sr = cur;
        if (t + 1 < t1) {
            cur = src(t + 1);
            load2(cur, q0, q1);
        }
        const bool odd = dbl && ((t - t0) & 1);
        set = odd ? sh + 256 * depth : sh;
        col = set + rep;
        count16(c0, sr.base + off, sr.n);
        count16(c1, sr.base + kEncTile / 2 + off, sr.n);
        if (a.tile_hist) {
            // the replicas keep counting across tiles: a tile's count is the
            // growth of their set's sum since that set's previous tile
            lds_barrier();
            if (tid < 256) {
                uint32_t s = 0;  // modulo 2^32: the growth over one tile is exact
                for (uint32_t r = 0; r < depth; ++r) s += set[(tid << dl) | ((r + rot) & (depth - 1))];
                const uint32_t c = s - (odd ? run2 : run);
                a.tile_hist[t * 256 + tid] = (uint16_t)c;
                if (odd) run2 = s; else run = s;
                if constexpr (kBatch) {
                    // a file's totals go out when its tiles in this run end
                    if (a.file_hist) {
                        const uint32_t fi = a.tile_file[t];
                        if (fi != curFile) {
                            if (curFile != 0xffffffffu && total) atomicAdd(&a.file_hist[curFile * 256ull + tid], total);
                            total = 0;
                            curFile = fi;
                        }
                    }
                }
                total += c;
            }
            // one set: no thread may count the next tile before every thread
            // has read this one (two sets: the next tile counts into the other
            // set, and the barrier after it orders this set's reads before the
            // tile after that counts here again)
            if (!dbl) lds_barrier();
        }
    }
    if constexpr (!kBatch) {
        if (!a.tile_hist) {
            __syncthreads();
            if (tid < 256)
                for (uint32_t r = 0; r < depth; ++r) total += sh[(tid << dl) | ((r + rot) & (depth - 1))];
        }
        if (tid < 256 && total) atomicAdd(&a.st->acc[blockIdx.x % kHistCopies][tid], total);
    } else {
        if (a.file_hist && tid < 256 && curFile != 0xffffffffu && total)
            atomicAdd(&a.file_hist[curFile * 256ull + tid], total);
    }
}

// Sums the accumulator copies into d_hist and zeroes them for the next launch.
__global__ __launch_bounds__(256) void k_hist_finalize(HistState* st, uint64_t* out) {
    const uint32_t v = threadIdx.x;
    unsigned long long t = 0;
    for (int c = 0; c < kHistCopies; ++c) {
        t += st->acc[c][v];
        st->acc[c][v] = 0;
    }
    out[v] = t;
}

hipError_t launch_histogram(const HistArgs& a, uint32_t blocks, hipStream_t s) {
    if (a.files) hipLaunchKernelGGL(k_hist<true>, dim3(blocks), dim3(kHistThreads), 0, s, a);
    else hipLaunchKernelGGL(k_hist<false>, dim3(blocks), dim3(kHistThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hist_finalize(HistState* st, uint64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_finalize, dim3(1), dim3(256), 0, s, st, out);
    return hipGetLastError();
}

// =============================================================== codebook
// One workgroup of 256 threads; thread v owns byte value v.
//
// Code lengths follow the merge rule (two smallest (weight, id) nodes ->
// one node of their summed weight), computed in rounds instead of one merge
// at a time: with s0 the sum of the two smallest queued nodes, every queued
// node of weight <= s0 precedes all nodes this round creates, so the first
// 2*floor(c/2) of those c nodes, taken in merged (weight, id) order, pair up
// exactly as the one-at-a-time merge pairs them.  Leaves are queued in
// (count, value) order, internal nodes in creation order (never decreasing),
// and on equal weight a leaf precedes an internal node and an older node a
// newer one.
__global__ __launch_bounds__(kCbThreads) void k_codebook(CbArgs a) {
    __shared__ unsigned long long s_w[512];  // node weights: sorted leaves [0,K), internal nodes [K, 2K-1)
    __shared__ __align__(16) unsigned long long s_tmp[256];  // sort keys
    __shared__ uint16_t s_par[512], s_m[512];
    __shared__ uint16_t s_d[512], s_p[512];
    __shared__ uint8_t s_sym[256];            // leaf rank -> byte
    __shared__ uint8_t s_len[256];
    __shared__ uint8_t s_sorted[256];
    __shared__ uint32_t s_cnt[64], s_fidx[64];
    __shared__ unsigned long long s_first[64];
    __shared__ uint32_t s_wcnt[64][kCbThreads / 64];  // bytes of each length, per wave
    __shared__ unsigned long long s_red_t[kCbThreads / 64], s_red_n[kCbThreads / 64];
    __shared__ uint32_t s_red_m[kCbThreads / 64];
    __shared__ uint32_t s_rc[kCbThreads / 64][2];  // per-wave counts of a merge round
    const uint32_t v = threadIdx.x;
    uint64_t h = 0;
    uint32_t myLen = 0;
    int32_t status = HUFF_OK;
    huff_dcb* d = a.out;
    int32_t* err = a.err;
    if (!a.from_lengths) {
        if (a.files) {
            // one workgroup per file: its histogram is the sum of its tiles'
            const FileDesc& f = a.files[blockIdx.x];
            d = const_cast<huff_dcb*>(f.cb);  // the batch builds the codebooks it then reads
            if (f.status) err = f.status;
            if (a.file_hist) {
                h = a.file_hist[(uint64_t)blockIdx.x * 256 + v];  // summed by the histogram launch
            } else {
                const uint64_t t0 = f.first, t1 = f.first + (f.n + kEncTile - 1) / kEncTile;
                uint64_t acc4[4] = {0, 0, 0, 0};
                uint64_t t = t0;
                for (; t + 4 <= t1; t += 4)
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc4[k] += a.tile_hist[(t + k) * 256 + v];
                for (; t < t1; ++t) acc4[0] += a.tile_hist[t * 256 + v];
                h = acc4[0] + acc4[1] + acc4[2] + acc4[3];
            }
            if (f.hist) f.hist[v] = h;
            if (f.n == 0 && v == 0) {  // an empty file's offset index is [0]
                f.chunk_off[0] = 0;
                if (f.sub_lo) f.sub_lo[0] = 0;
            }
        } else if (a.acc) {
            // all copies in flight at once, then summed, then cleared
            unsigned long long part[kHistCopies];
#pragma unroll
            for (int c = 0; c < kHistCopies; ++c) part[c] = a.acc->acc[c][v];
#pragma unroll
            for (int c = 0; c < kHistCopies; ++c) h += part[c];
#pragma unroll
            for (int c = 0; c < kHistCopies; ++c) a.acc->acc[c][v] = 0;
            if (a.hist_out) a.hist_out[v] = h;
        } else {
            h = a.hist[v];
        }
        if (__syncthreads_or(h >> 56)) status = HUFF_E_INVAL;  // counts must fit the sort key
        // leaves in (count, value) order: the present keys are gathered into
        // LDS (keys are distinct), and a present byte's rank is the number of
        // smaller keys among them
        const uint32_t lane = v & 63, wave = v >> 6;
        const bool present = h && status == HUFF_OK;
        const uint64_t key = present ? (h << 8) | v : 0ull;
        {
            const uint64_t bal = __ballot(present);
            if (lane == 0) s_rc[wave][0] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t off = 0;
            for (uint32_t w = 0; w < wave; ++w) off += s_rc[w][0];
            if (present) s_tmp[off + (uint32_t)__popcll(bal & ((1ull << lane) - 1))] = key;
        }
        const uint32_t K = s_rc[0][0] + s_rc[1][0] + s_rc[2][0] + s_rc[3][0];
        __syncthreads();
        if (present) {
            uint32_t r0 = 0, r1 = 0;
            const ulonglong2* k2 = reinterpret_cast<const ulonglong2*>(s_tmp);
            uint32_t u = 0;
#pragma unroll 16
            for (; u < K / 2; ++u) {  // independent broadcast reads: many in flight
                const ulonglong2 p = k2[u];
                r0 += p.x < key ? 1u : 0u;
                r1 += p.y < key ? 1u : 0u;
            }
            if (K & 1) r0 += s_tmp[K - 1] < key ? 1u : 0u;
            const uint32_t i = r0 + r1;
            s_w[i] = h;
            s_sym[i] = (uint8_t)v;
        }
        __syncthreads();
        if (status != HUFF_OK) {
            // leave every length 0
        } else if (K == 1) {
            myLen = h ? 1u : 0u;
        } else if (K >= 2) {
            uint32_t li = 0, qi = 0, m = 0;  // leaf head, internal head, internal nodes made
            uint32_t rounds = 0;
            while (m < K - 1) {
                // s0: sum of the two smallest queued nodes (leaf first on ties)
                const uint64_t kInf = ~0ull;
                const uint64_t l0 = li < K ? s_w[li] : kInf, l1 = li + 1 < K ? s_w[li + 1] : kInf;
                const uint64_t i0 = qi < m ? s_w[K + qi] : kInf, i1 = qi + 1 < m ? s_w[K + qi + 1] : kInf;
                uint64_t s0;
                if (l0 <= i0) s0 = l0 + (l1 <= i0 ? l1 : i0);
                else s0 = i0 + (l0 <= i1 ? l0 : i1);
                const bool leafIn = li + v < K && s_w[li + v] <= s0;
                const bool intIn = qi + v < m && s_w[K + qi + v] <= s0;
                // both counts with one barrier: per-wave ballots, then a sum
                {
                    const uint64_t bl = __ballot(leafIn), bi = __ballot(intIn);
                    if (lane == 0) {
                        s_rc[wave][0] = (uint32_t)__popcll(bl);
                        s_rc[wave][1] = (uint32_t)__popcll(bi);
                    }
                }
                __syncthreads();
                uint32_t cL = 0, cI = 0;
#pragma unroll
                for (int w = 0; w < kCbThreads / 64; ++w) {
                    cL += s_rc[w][0];
                    cI += s_rc[w][1];
                }
                const uint32_t pairs = (cL + cI) >> 1;
                if (cL == 0 || cI == 0) {
                    // one queue alone takes part: its nodes pair up in queue order
                    const uint32_t base = cI == 0 ? li : K + qi;
                    if (v < pairs) {
                        const uint32_t x = base + 2 * v, y = x + 1, id = K + m + v;
                        s_w[id] = s_w[x] + s_w[y];
                        s_par[x] = (uint16_t)id;
                        s_par[y] = (uint16_t)id;
                    }
                    __syncthreads();
                    if (cI == 0) li += 2 * pairs;
                    else qi += 2 * pairs;
                    m += pairs;
                    ++rounds;
                    continue;
                }
                // merged position of each node taking part
                // both binary searches in one loop, so that their LDS reads overlap:
                // for the leaf, internal nodes strictly lighter; for the internal
                // node, leaves at most as heavy
                const uint64_t keyL = leafIn ? s_w[li + v] : 0ull, keyI = intIn ? s_w[K + qi + v] : 0ull;
                uint32_t loL = 0, hiL = leafIn ? cI : 0u, loI = 0, hiI = intIn ? cL : 0u;
                while (loL < hiL || loI < hiI) {
                    const uint32_t mL = (loL + hiL) >> 1, mI = (loI + hiI) >> 1;
                    const uint64_t wL = s_w[K + qi + mL], wI = s_w[li + mI];
                    if (loL < hiL) {
                        if (wL < keyL) loL = mL + 1; else hiL = mL;
                    }
                    if (loI < hiI) {
                        if (wI <= keyI) loI = mI + 1; else hiI = mI;
                    }
                }
                const uint32_t posL = leafIn ? v + loL : ~0u;
                if (posL < 2 * pairs) s_m[posL] = (uint16_t)(li + v);
                if (intIn && v + loI < 2 * pairs) s_m[v + loI] = (uint16_t)(K + qi + v);
                const uint32_t nl = (uint32_t)__syncthreads_count(posL < 2 * pairs);
                if (v < pairs) {
                    const uint32_t x = s_m[2 * v], y = s_m[2 * v + 1];
                    const uint32_t id = K + m + v;
                    s_w[id] = s_w[x] + s_w[y];
                    s_par[x] = (uint16_t)id;
                    s_par[y] = (uint16_t)id;
                }
                __syncthreads();
                li += nl;
                qi += 2 * pairs - nl;
                m += pairs;
                ++rounds;
            }
            // depths by pointer jumping: d = distance to p, p -> p's ancestor
            const uint32_t nodes = 2 * K - 1, root = nodes - 1;
            for (uint32_t i = v; i < nodes; i += 256) {
                s_d[i] = i == root ? 0 : 1;
                s_p[i] = i == root ? root : s_par[i];
            }
            __syncthreads();
            // the tree is at most `rounds` deep (a round pairs only nodes made
            // before it), so ceil(log2(rounds + 1)) doublings reach the root
            const int jumps = 32 - __clz(rounds);
            for (int it = 0; it < jumps; ++it) {
                uint16_t nd[2] = {0, 0}, np[2] = {0, 0};
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t i = v + 256 * t;
                    if (i < nodes) {
                        const uint16_t p = s_p[i];
                        nd[t] = s_d[i] + s_d[p];
                        np[t] = s_p[p];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t i = v + 256 * t;
                    if (i < nodes) { s_d[i] = nd[t]; s_p[i] = np[t]; }
                }
                __syncthreads();
            }
            s_len[v] = 0;
            __syncthreads();
            if (v < K) s_len[s_sym[v]] = (uint8_t)s_d[v];
            __syncthreads();
            myLen = h ? s_len[v] : 0u;
        }
    } else {
        myLen = a.len[v];
    }
    // totals by wave reductions (no same-address atomics): n = sum h,
    // T = sum h * len, longest code
    const uint32_t lane = v & 63, wave = v >> 6;
    {
        const uint64_t wt = wave_sum_u64(h * myLen), wn = wave_sum_u64(h);
        uint32_t wm = myLen;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wm = max(wm, (uint32_t)__shfl_xor(wm, o, 64));
        if (lane == 0) {
            s_red_t[wave] = wt;
            s_red_n[wave] = wn;
            s_red_m[wave] = wm;
        }
    }
    s_sorted[v] = 0;
    __syncthreads();
    uint64_t tot = 0, nn = 0;
    uint32_t maxLen = 0;
#pragma unroll
    for (int w = 0; w < kCbThreads / 64; ++w) {
        tot += s_red_t[w];
        nn += s_red_n[w];
        maxLen = max(maxLen, s_red_m[w]);
    }
    if (maxLen > HUFF_MAX_CODE_LEN) status = HUFF_E_CODELEN;
    // counting sort of the present bytes by (length, value): per wave, one
    // ballot per length gives that length's count and each byte's rank among
    // the bytes of its length in lower lanes (lower byte values)
    const uint32_t lmax = maxLen < 64 ? maxLen : 63;
    uint32_t rank = 0;
    const uint64_t below = (1ull << lane) - 1;
    for (uint32_t l = 1; l <= lmax; ++l) {
        const uint64_t m = __ballot(myLen == l);
        if (myLen == l) rank = (uint32_t)__popcll(m & below);
        if (lane == 0) s_wcnt[l][wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (v < 64) {
        uint32_t c = 0;
        if (v >= 1 && v <= lmax)
            for (int w = 0; w < kCbThreads / 64; ++w) c += s_wcnt[v][w];
        s_cnt[v] = c;
    }
    __syncthreads();
    if (v < 64) {
        // wave 0, lane v = length v: fidx = bytes with shorter codes; first
        // canonical code of length v = sum over j < v of count[j] * 2^(v-j),
        // taken from the Kraft sums F(v) = sum over j < v of count[j] * 2^(63-j)
        // (at most 2^63: every code reaching here satisfies Kraft's inequality)
        const uint32_t c = s_cnt[v];
        s_fidx[v] = wave_incl_scan(c) - c;
        const uint64_t kv = v >= 1 ? (uint64_t)c << (63 - v) : 0ull;
        s_first[v] = (wave_incl_scan_u64(kv) - kv) >> (63 - v);
    }
    __syncthreads();
    // the byte's place in (length, value) order and its canonical code
    uint64_t code = 0;
    if (myLen && myLen < 64) {
        uint32_t r = rank;
        for (uint32_t w = 0; w < wave; ++w) r += s_wcnt[myLen][w];
        code = s_first[myLen] + r;
        s_sorted[s_fidx[myLen] + r] = (uint8_t)v;
    }
    const uint32_t K2 = (uint32_t)__syncthreads_count(myLen != 0 && myLen < 64);
    const uint32_t lutBits = maxLen < HUFF_LUT_BITS ? maxLen : HUFF_LUT_BITS;
    d->len[v] = (uint8_t)myLen;
    d->code[v] = code;
    d->enc[v] = (maxLen <= 24 && myLen) ? (uint32_t)((code << 8) | myLen) : 0u;
    d->sorted_sym[v] = s_sorted[v];
    if (v < 64) {
        d->first_code[v] = s_first[v];
        d->first_index[v] = s_fidx[v];
        d->count[v] = s_cnt[v];
    }
    // peek table: the codes of length l, left-justified to lutBits bits, fill
    // [lo[l], lo[l] + cnt[l] << (lutBits - l)); the ranges are read once into
    // registers and every entry finds its length by comparisons
    {
        uint32_t lo[HUFF_LUT_BITS + 1], span[HUFF_LUT_BITS + 1];
#pragma unroll
        for (uint32_t l = 1; l <= HUFF_LUT_BITS; ++l) {
            const bool on = l <= lutBits && s_cnt[l] != 0;
            lo[l] = on ? (uint32_t)(s_first[l] << (lutBits - l)) : 0u;
            span[l] = on ? s_cnt[l] << (lutBits - l) : 0u;
        }
#pragma unroll
        for (uint32_t p = v; p < (1u << HUFF_LUT_BITS); p += 256) {  // four independent entries in flight
            uint32_t len = 0;
#pragma unroll
            for (uint32_t l = 1; l <= HUFF_LUT_BITS; ++l) len = p - lo[l] < span[l] ? l : len;
            uint16_t e = 0;
            if (len) {
                const uint32_t c = p >> (lutBits - len);
                e = (uint16_t)(s_sorted[s_fidx[len] + (uint32_t)(c - s_first[len])] | (len << 8));
            }
            d->lut[p] = e;
        }
    }
    if (v == 0) {
        d->nsym = K2;
        d->max_len = maxLen;
        d->lut_bits = lutBits;
        d->status = status;
        d->total_bits = a.from_lengths ? 0 : tot;
        d->n = a.from_lengths ? 0 : nn;
        if (status != HUFF_OK) atomicMin(err, status);
    }
}

hipError_t launch_codebook(const CbArgs& a, uint32_t nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_codebook, dim3(nblocks), dim3(kCbThreads), 0, s, a);
    return hipGetLastError();
}

// ================================================================= encode
// Tile offsets.  A tile's code bits are known before it is encoded: from its
// u16 histogram (sum of count x length, written by k_hist) or, for a
// standalone encode, counted by k_tile_bits.  One stream: k_tile_scan turns
// them into an exclusive prefix inside blocks of kScanTiles tiles, and each
// block sums the bits of all earlier tiles into its carry.  A batch: the scan
// restarts at every file; k_tile_scan_seg
// scans inside the blocks and k_blk_scan carries the running total of the
// file that is open across a block boundary, so a tile's first bit is
// tile_local + (carry of its block if its file began before the block).
// Either way k_encode never waits on another workgroup.
constexpr int kScanTiles = kScanTilesPerBlock;

__global__ __launch_bounds__(kEncThreads) void k_tile_bits(const uint8_t* in, uint64_t n, const huff_dcb* cb,
                                                            uint32_t* tile_bits, int32_t* status, int32_t* err) {
    __shared__ uint8_t s_len[256];
    __shared__ uint32_t s_sum[kEncThreads / 64];
    const uint32_t tid = threadIdx.x;
    const uint64_t g = blockIdx.x;
    s_len[tid] = cb->len[tid];
    const bool aligned = ((uintptr_t)in & 15u) == 0;
    const uint64_t q = g * kEncTile + (uint64_t)tid * kEncUnit;
    uint4 x[kEncUnit / 16];
#pragma unroll
    for (int k = 0; k < kEncUnit / 16; ++k) x[k] = load16(in, q + 16 * k, n, aligned);
    __syncthreads();
    uint32_t sum = 0, missing = 0;
    const uint32_t nv = q >= n ? 0u : (uint32_t)min<uint64_t>(kEncUnit, n - q);
#pragma unroll
    for (int i = 0; i < kEncUnit; ++i) {
        const uint32_t l = (uint32_t)i < nv ? s_len[byte_of(x[i >> 4], i & 15)] : 1u;
        sum += (uint32_t)i < nv ? l : 0u;
        missing |= l == 0 ? 1u : 0u;
    }
    // a byte that has no code (the encoder itself does not check)
    if (missing) report(status, err, HUFF_E_INVAL);
    sum = (uint32_t)wave_sum_u64(sum);
    if ((tid & 63) == 0) s_sum[tid >> 6] = sum;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kEncThreads / 64; ++w) t += s_sum[w];
        tile_bits[g] = t;
    }
}

// Code bits of every tile from its u16 histogram: sum over byte values of
// count x code length.  One wave per kTbTiles consecutive tiles; lane l takes
// values 4l..4l+3, so a tile's 512-byte histogram is one coalesced 8-byte
// load per lane, and the wave issues the loads of all its tiles before it
// uses any.  A batch takes each tile's lengths from its file's codebook.
constexpr uint32_t kTbTiles = 4;

template <bool kBatch>
__global__ __launch_bounds__(256) void k_tile_bits_hist(TileBitsArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t t0 = ((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kTbTiles;
    if (t0 >= a.ntiles) return;  // the whole wave
    uint2 h[kTbTiles];
    uint32_t l4[kTbTiles];
#pragma unroll
    for (uint32_t k = 0; k < kTbTiles; ++k) {
        const uint64_t t = t0 + k < a.ntiles ? t0 + k : t0;
        const huff_dcb* cb = a.cb;
        if constexpr (kBatch) cb = a.files[a.tile_file[t]].cb;
        h[k] = reinterpret_cast<const uint2*>(a.tile_hist + t * 256)[lane];
        l4[k] = reinterpret_cast<const uint32_t*>(cb->len)[lane];
    }
#pragma unroll
    for (uint32_t k = 0; k < kTbTiles; ++k) {
        const uint64_t t = t0 + k;
        if (t >= a.ntiles) break;  // the whole wave
        const uint2 hk = h[k];
        const uint32_t lk = l4[k];
        uint32_t bits = (hk.x & 0xffffu) * (lk & 0xffu) + (hk.x >> 16) * ((lk >> 8) & 0xffu) +
                        (hk.y & 0xffffu) * ((lk >> 16) & 0xffu) + (hk.y >> 16) * (lk >> 24);
        // a byte that occurs but has no code (the encoder itself does not check)
        const bool missing = ((hk.x & 0xffffu) && !(lk & 0xffu)) || ((hk.x >> 16) && !(lk & 0xff00u)) ||
                             ((hk.y & 0xffffu) && !(lk & 0xff0000u)) || ((hk.y >> 16) && !(lk & 0xff000000u));
        if (missing) report(kBatch ? a.files[a.tile_file[t]].status : a.status, a.err, HUFF_E_INVAL);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) bits += __shfl_xor(bits, d, 64);
        if (lane == 0) a.tile_bits[t] = bits;
    }
}

hipError_t launch_tile_bits_hist(const TileBitsArgs& a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    const uint64_t blocks = (a.ntiles + 4 * kTbTiles - 1) / (4 * kTbTiles);
    if (a.files) hipLaunchKernelGGL(k_tile_bits_hist<true>, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_tile_bits_hist<false>, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// One stream of at most kInlineCarryBlocks scan blocks: exclusive scan of
// the tile bits inside blocks of kScanTiles tiles, one thread per tile, and
// each block's carry summed from the tile counts of all earlier blocks (at
// most (kInlineCarryBlocks - 1) x kScanTiles reads per block, so one launch
// does both levels).  tile_local must not alias tile_bits: a block reads the
// counts of earlier blocks while those blocks write their offsets.  Longer
// streams take the segmented scan below (a single segment) and k_blk_scan,
// whose cost grows linearly with the tile count.
constexpr uint64_t kInlineCarryBlocks = 8;

__global__ __launch_bounds__(kScanTiles) void k_tile_scan(ScanArgs a) {
    __shared__ uint32_t s_wsum[kScanTiles / 64];
    __shared__ unsigned long long s_wcar[kScanTiles / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanTiles;
    const uint64_t t = b0 + tid;
    const uint32_t bits = t < a.ntiles ? a.tile_bits[t] : 0u;
    // the block's carry: the bits of every earlier tile, summed here from the
    // tile counts (a strided read of at most ntiles words per block), so that
    // one stream needs no separate scan of block totals
    unsigned long long car = 0;
    for (uint64_t u = tid; u < b0; u += kScanTiles) car += a.tile_bits[u];
    car = wave_sum_u64(car);
    const uint32_t incl = wave_incl_scan(bits);
    if (lane == 63) s_wsum[wave] = incl;
    if (lane == 0) s_wcar[wave] = car;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < (int)wave; ++w) before += s_wsum[w];
    if (t < a.ntiles) a.tile_local[t] = before + incl - bits;
    if (tid == 0) {
        unsigned long long c = 0;
        for (int w = 0; w < kScanTiles / 64; ++w) c += s_wcar[w];
        a.blk_carry[blockIdx.x] = c;
    }
}

// Batch: the same scan restarted at every file (without a file table the
// whole stream is one file).  One workgroup per block of kScanTiles tiles,
// one thread per tile; tile_local may be the tile_bits buffer itself (each
// thread reads only its own tile's count, before it writes that tile's
// offset).
__global__ __launch_bounds__(kScanTiles) void k_tile_scan_seg(ScanArgs a) {
    __shared__ uint32_t s_wsum[kScanTiles / 64];
    __shared__ uint32_t s_excl[kScanTiles];
    __shared__ uint32_t s_head;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanTiles;
    const uint64_t t = b0 + tid;
    const uint64_t last = min<uint64_t>(a.ntiles, b0 + kScanTiles) - 1;
    uint32_t bits = 0;
    uint64_t first = 0;  // first tile of the tile's file
    if (t < a.ntiles) {
        if (a.files) first = a.files[a.tile_file[t]].first;
        bits = a.tile_bits[t];
    }
    const uint32_t incl = wave_incl_scan(bits);
    if (lane == 63) s_wsum[wave] = incl;
    if (tid == 0) s_head = first == b0 ? 1u : 0u;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < (int)wave; ++w) before += s_wsum[w];
    const uint32_t excl = before + incl - bits;
    s_excl[tid] = excl;
    __syncthreads();
    // the tile's segment starts at its file's first tile or at the block start
    const uint32_t seg = first > b0 ? (uint32_t)(first - b0) : 0u;
    if (t < a.ntiles) a.tile_local[t] = excl - s_excl[seg];
    if (t == last) {
        unsigned long long tail = (unsigned long long)(excl + bits - s_excl[seg]);
        if (first >= b0) tail |= kTailStarts;
        if (s_head) tail |= kTailHead;
        a.blk_tail[blockIdx.x] = tail;
    }
}

// Block carries, one workgroup: carry[B] = 0 if a file starts at block B's
// first tile; else tail[B-1] if the segment that ends block B-1 began inside
// it; else carry[B-1] + tail[B-1].  A scan with resets, 1024 blocks per pass.
__global__ __launch_bounds__(1024) void k_blk_scan(const unsigned long long* tail, unsigned long long* carry,
                                                   uint64_t nblk) {
    __shared__ unsigned long long s_v[2][1024];
    __shared__ uint32_t s_r[2][1024];
    const uint32_t tid = threadIdx.x;
    unsigned long long run = 0;  // carry of the last block of the previous pass
    for (uint64_t base = 0; base < nblk; base += 1024) {
        const uint64_t B = base + tid;
        unsigned long long v = 0;
        uint32_t r = 1;
        if (B < nblk && B > 0) {
            const unsigned long long cur = tail[B], prev = tail[B - 1];
            const bool head = (cur & kTailHead) != 0;
            r = head || (prev & kTailStarts) ? 1u : 0u;
            v = head ? 0ull : (prev & kTailBits);
        }
        if (tid == 0 && !r) v += run;  // continues the previous pass
        r |= tid == 0 ? 1u : 0u;
        // inclusive scan with resets (Hillis-Steele, double buffered)
        int cur = 0;
        s_v[0][tid] = v;
        s_r[0][tid] = r;
        __syncthreads();
        // only as many steps as this pass has blocks (every later block has r = 1)
        const uint32_t span = (uint32_t)min<uint64_t>(1024, nblk - base);
        for (uint32_t d = 1; d < span; d <<= 1) {
            unsigned long long nv = s_v[cur][tid];
            uint32_t nr = s_r[cur][tid];
            if (tid >= d && !nr) {
                nv += s_v[cur][tid - d];
                nr = s_r[cur][tid - d];
            }
            s_v[cur ^ 1][tid] = nv;
            s_r[cur ^ 1][tid] = nr;
            cur ^= 1;
            __syncthreads();
        }
        if (B < nblk) carry[B] = s_v[cur][tid];
        run = s_v[cur][1023];
        __syncthreads();
    }
}

hipError_t launch_tile_bits(const uint8_t* in, uint64_t n, const huff_dcb* cb, uint32_t* tile_bits, int32_t* status,
                            int32_t* err, hipStream_t s) {
    const uint64_t ntiles = (n + kEncTile - 1) / kEncTile;
    hipLaunchKernelGGL(k_tile_bits, dim3((uint32_t)ntiles), dim3(kEncThreads), 0, s, in, n, cb, tile_bits, status, err);
    return hipGetLastError();
}

hipError_t launch_tile_scan(const ScanArgs& a, hipStream_t s) {
    const uint64_t blocks = (a.ntiles + kScanTiles - 1) / kScanTiles;
    if (blocks == 0) return hipSuccess;
    if (!a.files && blocks <= kInlineCarryBlocks) {
        hipLaunchKernelGGL(k_tile_scan, dim3((uint32_t)blocks), dim3(kScanTiles), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_tile_scan_seg, dim3((uint32_t)blocks), dim3(kScanTiles), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_blk_scan(a.blk_tail, a.blk_carry, blocks, s);
}

hipError_t launch_blk_scan(const unsigned long long* blk_tail, unsigned long long* blk_carry, uint64_t nblk,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_blk_scan, dim3(1), dim3(1024), 0, s, blk_tail, blk_carry, nblk);
    return hipGetLastError();
}

// Persistent encode over 16 KiB tiles (256 threads x 64 bytes); workgroup w
// takes tiles w, w + G, w + 2G, ... and requests the next tile's bytes while
// it encodes the current one.  Each thread packs its 64 bytes into a private
// LDS slot with one table lookup per byte; the workgroup scans the
// per-thread bit counts; the tile's first stream bit is its block prefix
// plus its offset inside the block.
//
// Output words are owned by the thread whose bit range holds the word's last
// bit; the bits of the owner's first word that precede its range belong to
// the previous thread (read from that thread's LDS slot) or, for the first
// thread of a tile, are re-derived from the 32 input bytes before the tile.
// The final partial word of a stream is written by its last thread.  No two
// threads write the same word.
constexpr int kSlotWords = kEncUnit * 16 / 32 + 1;  // 64 bytes x 16 bits, plus a zero word
constexpr int kSlotStride = kEncThreads + 1;           // word k of thread t at [k*stride + t]: banks differ along k
// With codes of at most 8 bits a thread's slot needs rows 0..16 (64 x 8 bits
// and the zero word); rows kLinRow.. then hold a whole tile's output words
// (at most 16 KiB x 8 bits / 32 + 1 = 4097 of them).
constexpr int kLinRow = kEncUnit * 8 / 32 + 1;
static_assert((kSlotWords - kLinRow) * kSlotStride >= kEncTile * 8 / 32 + 1, "tile words fit above the slots");
constexpr int kEncWaves = kEncThreads / 64;
// The compact encode kernel: codes of at most 10 bits, so a slot needs 21
// words and the zero word, and a tile at most 16 KiB x 10 / 32 + 1 words,
// which the whole slot region holds once the threads have taken their words
// into registers.  Its LDS (about 26.8 KB against 38.4 KB) lets a CU hold six
// workgroups instead of four, so more tiles' loads are in flight.
constexpr int kEncCompactMaxLen = 10;
constexpr int kCompactRows = kEncUnit * kEncCompactMaxLen / 32 + 2;
static_assert(kCompactRows * kSlotStride >= kEncTile * kEncCompactMaxLen / 32 + 1, "a tile's words fit the slots");

__device__ __forceinline__ uint32_t byte64(const uint4& a, const uint4& b, const uint4& c, const uint4& d, int i) {
    return i < 16 ? byte_of(a, i) : i < 32 ? byte_of(b, i - 16) : i < 48 ? byte_of(c, i - 32) : byte_of(d, i - 48);
}

// Packs one thread's 64 bytes (codes of at most 16 bits) into its LDS slot,
// left-aligned and followed by a zero word: G codes at a time are joined
// into one 32-bit group (so G codes of at most 32/G bits) before the group is
// appended to a 64-bit accumulator.  Every group stores the accumulator's
// current top word and moves to the next slot word only once that word is
// full, so there is no branch.  G = 4 (codes of at most 8 bits) reads the
// length and the code from two byte tables (s_len, s_code8: the lanes of a
// wave then meet fewer LDS bank conflicts than in one 16-bit table); G <= 3
// reads both from one table read of s_cl32 (code in the low half, length in
// the high half).  G = 1 handles a partial unit of nv bytes.
template <int G>
__device__ __forceinline__ void pack_unit(const uint4 x0, const uint4 x1, const uint4 x2, const uint4 x3,
                                            const uint8_t* s_len, const uint8_t* s_code8, const uint32_t* s_cl32,
                                            uint32_t* slot, uint32_t& L, uint32_t& nwp, uint32_t nv = kEncUnit) {
    uint64_t acc = 0;
    uint32_t na = 0, wi = 0;
    auto emit = [&]() {
        const uint32_t sh = na >= 32 ? na - 32 : 0;
        slot[wi * kSlotStride] = (uint32_t)(acc >> sh);
        const uint32_t full = na >= 32 ? 1u : 0u;
        wi += full;
        na -= full << 5;
    };
    if constexpr (G == 1) {
        for (uint32_t i = 0; i < nv; ++i) {
            const uint32_t e = s_cl32[byte64(x0, x1, x2, x3, (int)i)];
            const uint32_t l = e >> 16;
            acc = (acc << l) | (e & 0xffffu);
            na += l;
            emit();
        }
    } else {
#pragma unroll
        for (int i0 = 0; i0 < kEncUnit; i0 += G) {
            uint32_t g = 0, gl = 0;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (i0 + k < kEncUnit) {
                    const uint32_t v = byte64(x0, x1, x2, x3, i0 + k);
                    uint32_t l, c;
                    if constexpr (G == 4) {
                        l = s_len[v];
                        c = s_code8[v];
                    } else {
                        const uint32_t e = s_cl32[v];
                        l = e >> 16;
                        c = e & 0xffffu;
                    }
                    g = (g << l) | c;
                    gl += l;
                }
            }
            acc = (acc << gl) | g;
            na += gl;
            emit();
        }
    }
    L = wi * 32 + na;
    nwp = wi;
    if (na) {
        slot[wi * kSlotStride] = (uint32_t)(acc << (32 - na));
        ++nwp;
    }
    slot[nwp * kSlotStride] = 0;
}

// kRows = kSlotWords: every code length (the full kernel); kRows =
// kCompactRows: codes of at most kEncCompactMaxLen bits.
template <bool kBatch, bool kAligned, int kRows>
__device__ __forceinline__ void encode_tiles(const EncArgs& a) {
    constexpr bool kCompact = kRows < kSlotWords;
    __shared__ uint32_t s_slot[kRows * kSlotStride];  // private slots; tile bytes (generic path)
    // code | length << 16, and (codes of at most 8 bits) the code alone, per
    // byte value; the full kernel also keeps the whole codes for longer ones
    __shared__ unsigned long long s_code[kCompact ? 1 : 256];
    __shared__ uint32_t s_cl32[256];
    __shared__ uint8_t s_code8[256];
    __shared__ uint8_t s_len[256];
    __shared__ uint32_t s_prev4[8];  // the 32 input bytes before the tile
    __shared__ uint32_t s_L[kEncThreads];
    __shared__ uint32_t s_wsum[kEncWaves];
    const uint8_t* s_prev = reinterpret_cast<const uint8_t*>(s_prev4);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (!kBatch) {
        // a split launch: the stream's codes are the compact kernel's or the
        // full kernel's, never both (the same value for the whole grid)
        if (a.split && kCompact != (a.one.cb->max_len <= (uint32_t)kEncCompactMaxLen)) return;
    }
    const huff_dcb* loaded = nullptr;
    bool fast = true;
    uint32_t group = 1;

    auto fileOf = [&](uint64_t tile) -> const FileDesc& {
        if constexpr (kBatch) return a.files[a.tile_file[tile]];
        else return a.one;
    };
    // Everything a tile needs from memory is requested one tile ahead, by a
    // fixed sequence of loads with no branch: the thread's 64 bytes, the 32
    // bytes before the tile (lanes 0..7), the tile's offset inside its scan
    // block and the carry of its block.  They are first used in the next
    // iteration, so the wait for them does not fall right behind their issue.
    struct Pre {
        uint4 x0, x1, x2, x3;
        uint32_t before, local;
        unsigned long long carry;
    };
    auto fetch = [&](uint64_t tile, Pre& p) {
        const FileDesc& d = fileOf(tile);
        const uint64_t j = tile - d.first;
        const uint64_t q = j * (uint64_t)kEncTile + (uint64_t)tid * kEncUnit;
        if constexpr (kAligned) {
            // whole aligned 16-byte blocks: a block that holds a byte of the
            // file lies in a page of the file; a block wholly past the end is
            // replaced by block 0 (its bytes are not used)
            auto blk = [&](uint64_t at) { return *reinterpret_cast<const uint4*>(d.in + (at < d.n ? at : 0)); };
            p.x0 = blk(q);
            p.x1 = blk(q + 16);
            p.x2 = blk(q + 32);
            p.x3 = blk(q + 48);
            const uint64_t bo = j > 0 && tid < 8 ? j * (uint64_t)kEncTile - 32 + 4 * tid : 0;
            p.before = *reinterpret_cast<const uint32_t*>(d.in + bo);
        } else {
            p.x0 = load16(d.in, q, d.n, false);
            p.x1 = load16(d.in, q + 16, d.n, false);
            p.x2 = load16(d.in, q + 32, d.n, false);
            p.x3 = load16(d.in, q + 48, d.n, false);
            p.before = 0;
            if (j > 0 && tid < 8) {
                const uint8_t* bp = d.in + j * (uint64_t)kEncTile - 32 + 4 * tid;
                p.before = (uint32_t)bp[0] | (uint32_t)bp[1] << 8 | (uint32_t)bp[2] << 16 | (uint32_t)bp[3] << 24;
            }
        }
        // vector loads (an index the compiler cannot see is uniform): a
        // scalar load would share its wait counter with the LDS lookups
        uint32_t lane0 = (uint32_t)(tid >> 10);
        asm volatile("" : "+v"(lane0));
        const uint64_t blk = tile / kScanTiles;
        p.local = a.tile_local[tile + lane0];
        // blk_carry[0] is 0: it stands in when the file begins inside the block
        p.carry = a.blk_carry[(d.first <= blk * kScanTiles ? blk : 0) + lane0];
    };
    Pre cur;
    cur.x0 = cur.x1 = cur.x2 = cur.x3 = make_uint4(0, 0, 0, 0);
    cur.before = cur.local = 0;
    cur.carry = 0;
    // the compact kernel (one tile per workgroup at its usual grid) loads
    // each tile when it starts it: no registers held for the next one
    // so does either kernel of a split batch, each of which skips the other's
    // tiles (a prefetch could read a tile that this kernel then skips)
    const bool batchSplit = kBatch && a.split == 2;
    const bool early = kCompact || batchSplit;
    if (!early && (uint64_t)blockIdx.x < a.ntiles) fetch(blockIdx.x, cur);
    // the previous tile stored its words from the slot rows at and above
    // kLinRow: every read of LDS it still makes comes after its barriers, and
    // from those rows only, which the next tile (same codebook, codes of at
    // most 8 bits) writes only after its scan barrier
    bool prevLin = false;
    for (uint64_t g = blockIdx.x; g < a.ntiles; g += gridDim.x) {
        const FileDesc& f = fileOf(g);
        if constexpr (kBatch) {
            // a split batch: files with codes of at most kEncCompactMaxLen
            // bits are the compact kernel's, the others the full kernel's
            if (batchSplit && (f.cb->max_len <= (uint32_t)kEncCompactMaxLen) != kCompact) continue;
        }
        const uint64_t j = g - f.first;
        const uint64_t n = f.n;
        const uint64_t tstart = j * (uint64_t)kEncTile;
        const uint64_t q0 = tstart + (uint64_t)tid * kEncUnit;
        const uint32_t nv = q0 >= n ? 0u : (uint32_t)min<uint64_t>(kEncUnit, n - q0);
        if (early) fetch(g, cur);
        const uint4 x0 = cur.x0, x1 = cur.x1, x2 = cur.x2, x3 = cur.x3;
        const uint32_t prev4 = cur.before;
        const uint64_t S = cur.carry + cur.local;  // the tile's first stream bit
        // the next tile's loads (none after the workgroup's last tile)
        const uint64_t gn = g + gridDim.x;
        if (!early && gn < a.ntiles) fetch(gn, cur);
        if (!(prevLin && f.cb == loaded)) __syncthreads();  // the previous tile is done with the LDS slots and tables
        prevLin = false;
        if (tid < 8) s_prev4[tid] = prev4;
        if (f.cb != loaded) {
            const uint32_t maxLen = f.cb->max_len;
            fast = maxLen <= 16;
            group = maxLen <= 8 ? 4 : maxLen <= 10 ? 3 : 2;  // codes per 32-bit group
            {
                const uint64_t c = f.cb->code[tid];
                const uint32_t l = f.cb->len[tid];
                s_len[tid] = (uint8_t)l;
                s_cl32[tid] = (uint32_t)(c & 0xffffu) | l << 16;
                s_code8[tid] = (uint8_t)c;
                if constexpr (!kCompact) s_code[tid] = c;
            }
            loaded = f.cb;
            __syncthreads();
        }

        // 1) pack into the private slot (fast) or count bits (generic)
        uint32_t L = 0, nwp = 0;
        if (fast) {
            uint32_t* slot = s_slot + tid;  // stride kSlotStride
            if (nv == kEncUnit) {
                // opaque copies keep the variants from sharing (and hoisting)
                // their byte extraction and table reads
                uint4 z0 = x0, z1 = x1, z2 = x2, z3 = x3;
                asm volatile("" : "+v"(z0.x), "+v"(z0.y), "+v"(z0.z), "+v"(z0.w), "+v"(z1.x), "+v"(z1.y), "+v"(z1.z), "+v"(z1.w)::"memory");
                asm volatile("" : "+v"(z2.x), "+v"(z2.y), "+v"(z2.z), "+v"(z2.w), "+v"(z3.x), "+v"(z3.y), "+v"(z3.z), "+v"(z3.w)::"memory");
                if (group == 4) {
                    pack_unit<4>(z0, z1, z2, z3, s_len, s_code8, s_cl32, slot, L, nwp);
                } else if (kCompact || group == 3) {  // the compact kernel's codes: at most 10 bits
                    asm volatile("" : "+v"(z0.x), "+v"(z1.x), "+v"(z2.x), "+v"(z3.x)::"memory");
                    pack_unit<3>(z0, z1, z2, z3, s_len, s_code8, s_cl32, slot, L, nwp);
                } else {
                    asm volatile("" : "+v"(z0.y), "+v"(z1.y), "+v"(z2.y), "+v"(z3.y)::"memory");
                    pack_unit<2>(z0, z1, z2, z3, s_len, s_code8, s_cl32, slot, L, nwp);
                }
            } else {
                pack_unit<1>(x0, x1, x2, x3, s_len, s_code8, s_cl32, slot, L, nwp, nv);
            }
        } else {
            uint4* in4 = reinterpret_cast<uint4*>(s_slot) + 4 * tid;
            in4[0] = x0;
            in4[1] = x1;
            in4[2] = x2;
            in4[3] = x3;
            for (uint32_t i = 0; i < nv; ++i) L += s_len[byte64(x0, x1, x2, x3, (int)i)];
        }

        // 2) workgroup exclusive scan of per-thread bit counts
        s_L[tid] = L;
        const uint32_t incl = wave_incl_scan(L);
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, agg = 0;
#pragma unroll
        for (int w = 0; w < kEncWaves; ++w) {
            const uint32_t ws = s_wsum[w];
            agg += ws;
            before += w < wave ? ws : 0u;
        }
        const uint64_t b = S + before + incl - L, e = b + L;
        const uint32_t sh = (uint32_t)(b & 31);
        const bool lastThread = nv > 0 && q0 + kEncUnit >= n;

        // 3) segment index and decode index
        if (nv) {
            if ((q0 & ((1ull << a.chunk_log2) - 1)) == 0) f.chunk_off[q0 >> a.chunk_log2] = b;
            if (a.sub_log2 != kNoSub) {
                if (a.sub_log2 >= 6) {
                    if ((q0 & ((1ull << a.sub_log2) - 1)) == 0) f.sub_lo[q0 >> a.sub_log2] = (uint32_t)b;
                } else {
                    // sub-blocks of 16 or 32 bytes: bit offsets inside the unit
                    const uint32_t step = 1u << a.sub_log2;
                    uint32_t run = 0;
                    for (uint32_t at = 0; at < nv; at += step) {
                        f.sub_lo[(q0 + at) >> a.sub_log2] = (uint32_t)(b + run);
                        for (uint32_t i = at; i < at + step && i < nv; ++i) run += s_len[byte64(x0, x1, x2, x3, (int)i)];
                    }
                }
            }
        }
        if (lastThread) {
            f.chunk_off[(n + (1ull << a.chunk_log2) - 1) >> a.chunk_log2] = e;
            if (a.sub_log2 != kNoSub) f.sub_lo[(n + (1ull << a.sub_log2) - 1) >> a.sub_log2] = (uint32_t)e;
            if (((e + 31) >> 5) > f.nwords) report(f.status, a.err, HUFF_E_CAPACITY);
        }

        // 4) the bits before b that share b's word, right-aligned
        uint32_t prefix = 0;
        if (sh && nv) {
            if (tid > 0 && fast && s_L[tid - 1] >= sh) {
                const uint32_t Lp = s_L[tid - 1];
                const uint32_t q = Lp - sh, i = q >> 5, o = q & 31;
                const uint64_t hi = s_slot[i * kSlotStride + tid - 1];
                const uint64_t lo = s_slot[(i + 1) * kSlotStride + tid - 1];  // zero past the last word
                prefix = (uint32_t)((((hi << 32) | lo) << o) >> 32) >> (32 - sh);
            } else {
                // re-derive from the bytes just before this thread's unit
                uint64_t acc = 0;
                uint32_t nb = 0;
                for (int k = 31; k >= 0 && nb < sh; --k) {
                    const uint32_t v = tid == 0 ? s_prev[k]
                                                : reinterpret_cast<const uint8_t*>(s_slot)[(tid - 1) * kEncUnit + 32 + k];
                    if constexpr (kCompact) acc |= (uint64_t)(s_cl32[v] & 0xffffu) << nb;
                    else acc |= s_code[v] << nb;
                    nb += s_len[v];
                }
                prefix = (uint32_t)acc & ((1u << sh) - 1);
            }
        }

        // 5) write the owned words
        const uint64_t w0 = b >> 5;
        const uint64_t tileEnd = S + agg;
        const bool tileLast = tstart + kEncTile >= n;
        const bool capOK = ((tileEnd + 31) >> 5) <= f.nwords;  // the whole tile fits
        if (fast) {
            uint32_t nw = (uint32_t)((e >> 5) - w0);
            if (lastThread && (e & 31)) ++nw;
            uint32_t* wp = f.words + w0;
            const uint32_t* slot = s_slot + tid;
            uint32_t prevw = prefix;
            if (capOK && group == 4 && !kCompact) {
                // Codes of at most 8 bits fill only slot rows below kLinRow:
                // the tile's words are put together in order in the rows
                // above, then the whole workgroup stores them, 1 KB of
                // contiguous words per store instruction (group and capOK are
                // the same for every thread of the tile).
                const uint64_t ws = S >> 5;  // the tile's first word
                uint32_t* lin = s_slot + kLinRow * kSlotStride;
                const uint32_t at = (uint32_t)(w0 - ws);
                constexpr uint32_t kLinWords = (kSlotWords - kLinRow) * kSlotStride;
                for (uint32_t k = 0; k < nw; ++k) {
                    const uint32_t cur = slot[k * kSlotStride];
                    if (at + k < kLinWords) lin[at + k] = __builtin_amdgcn_alignbit(prevw, cur, sh);
                    prevw = cur;
                }
                __syncthreads();
                // the tile's words: those whose last bit lies in the tile, and
                // the stream's final partial word after the last tile
                const uint32_t nwt = (uint32_t)((tileEnd >> 5) - ws) + (tileLast && (tileEnd & 31) ? 1u : 0u);
                const uint32_t head = min(nwt, ((uint32_t)(0u - (uint32_t)(uintptr_t)(f.words + ws)) & 15u) >> 2);
                if ((uint32_t)tid < head) f.words[ws + tid] = lin[tid];
                const uint32_t body = (nwt - head) >> 2;
                uint4* g4 = reinterpret_cast<uint4*>(f.words + ws + head);
                for (uint32_t u = tid; u < body; u += kEncThreads) {
                    const uint32_t o = head + 4 * u;
                    g4[u] = make_uint4(lin[o], lin[o + 1], lin[o + 2], lin[o + 3]);
                }
                const uint32_t t0 = head + 4 * body;
                if ((uint32_t)tid < nwt - t0) f.words[ws + t0 + tid] = lin[t0 + tid];
                prevLin = true;
            } else if (capOK && (group == 3 || (kCompact && group == 4))) {
                // Codes of 9 or 10 bits (and, in the compact kernel, all
                // codes): the slots fill the rows that the assembled tile
                // would need, so each thread first takes its (at most
                // kWords3) words into registers; after a barrier the whole
                // slot region holds the tile's words in order, and the
                // workgroup stores them as above.
                constexpr uint32_t kWords3 = kEncUnit * 10 / 32 + 1;
                const uint64_t ws = S >> 5;
                const uint32_t at = (uint32_t)(w0 - ws);
                uint32_t wv[kWords3];
#pragma unroll
                for (uint32_t k = 0; k < kWords3; ++k) {
                    const uint32_t cur = k < nw ? slot[k * kSlotStride] : 0u;
                    wv[k] = __builtin_amdgcn_alignbit(prevw, cur, sh);
                    prevw = cur;
                }
                __syncthreads();  // every thread is done with its slot
                constexpr uint32_t kAllWords = kRows * kSlotStride;
#pragma unroll
                for (uint32_t k = 0; k < kWords3; ++k)
                    if (k < nw && at + k < kAllWords) s_slot[at + k] = wv[k];
                __syncthreads();
                const uint32_t nwt = (uint32_t)((tileEnd >> 5) - ws) + (tileLast && (tileEnd & 31) ? 1u : 0u);
                const uint32_t head = min(nwt, ((uint32_t)(0u - (uint32_t)(uintptr_t)(f.words + ws)) & 15u) >> 2);
                if ((uint32_t)tid < head) f.words[ws + tid] = s_slot[tid];
                const uint32_t body = (nwt - head) >> 2;
                uint4* g4 = reinterpret_cast<uint4*>(f.words + ws + head);
                for (uint32_t u = tid; u < body; u += kEncThreads) {
                    const uint32_t o = head + 4 * u;
                    g4[u] = make_uint4(s_slot[o], s_slot[o + 1], s_slot[o + 2], s_slot[o + 3]);
                }
                const uint32_t t0 = head + 4 * body;
                if ((uint32_t)tid < nwt - t0) f.words[ws + t0 + tid] = s_slot[t0 + tid];
            } else if (capOK && !kCompact) {
                // single words up to a 16-byte boundary, then 16-byte stores
                uint32_t k = 0;
                const uint32_t head = min(nw, ((uint32_t)(0u - (uint32_t)(uintptr_t)wp) & 15u) >> 2);
                for (; k < head; ++k) {
                    const uint32_t cur = slot[k * kSlotStride];
                    wp[k] = __builtin_amdgcn_alignbit(prevw, cur, sh);
                    prevw = cur;
                }
                for (; k + 4 <= nw; k += 4) {
                    const uint32_t c0 = slot[k * kSlotStride], c1 = slot[(k + 1) * kSlotStride];
                    const uint32_t c2 = slot[(k + 2) * kSlotStride], c3 = slot[(k + 3) * kSlotStride];
                    *reinterpret_cast<uint4*>(wp + k) =
                        make_uint4(__builtin_amdgcn_alignbit(prevw, c0, sh), __builtin_amdgcn_alignbit(c0, c1, sh),
                                   __builtin_amdgcn_alignbit(c1, c2, sh), __builtin_amdgcn_alignbit(c2, c3, sh));
                    prevw = c3;
                }
                for (; k < nw; ++k) {
                    const uint32_t cur = slot[k * kSlotStride];
                    wp[k] = __builtin_amdgcn_alignbit(prevw, cur, sh);
                    prevw = cur;
                }
            } else {
                for (uint32_t k = 0; k < nw; ++k) {
                    const uint32_t cur = slot[k * kSlotStride];
                    if (w0 + k < f.nwords) wp[k] = __builtin_amdgcn_alignbit(prevw, cur, sh);
                    prevw = cur;
                }
            }
        } else if (nv) {
            uint64_t acc = prefix;
            uint32_t na = sh;
            uint64_t w = w0;
            auto put = [&](uint64_t c, uint32_t len) {
                acc = (acc << len) | c;
                na += len;
                if (na >= 32) {
                    na -= 32;
                    if (w < f.nwords) f.words[w] = (uint32_t)(acc >> na);
                    ++w;
                }
            };
            for (uint32_t i = 0; i < nv; ++i) {
                const uint32_t v = byte64(x0, x1, x2, x3, (int)i);
                const uint32_t l = s_len[v];
                // codes past 16 bits never reach the compact kernel (its
                // launch takes only codebooks of at most 10 bits)
                const uint64_t c = kCompact ? (uint64_t)(s_cl32[v] & 0xffffu) : s_code[v];
                if (l > 32) {
                    put(c >> 32, l - 32);
                    put(c & 0xffffffffull, 32);
                } else {
                    put(c, l);
                }
            }
            if (lastThread && na && w < f.nwords) f.words[w] = (uint32_t)(acc << (32 - na));
        }
    }
}

template <bool kBatch, bool kAligned>
__global__ __launch_bounds__(kEncThreads) void k_encode(EncArgs a) {
    encode_tiles<kBatch, kAligned, kSlotWords>(a);
}

// At most 80 VGPRs, so that six workgroups (24 waves) fit a CU, as its LDS allows.
template <bool kBatch>
__global__ __launch_bounds__(kEncThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_encode_compact(EncArgs a) {
    encode_tiles<kBatch, true, kCompactRows>(a);
}

// A single stream's codebook is on the device when the encode is queued, so
// for a 16-byte aligned input both kernels are launched: the compact one on
// the full grid, then the full one on at most kEncLongGrid workgroups (a
// persistent grid over the tiles); the one whose codes these are not exits at
// once.  A batch of aligned files launches both on the full grid, each taking
// the tiles of the files whose codes are its own.
constexpr uint32_t kEncLongGrid = 1024;

hipError_t launch_encode(const EncArgs& a, uint32_t grid, hipStream_t s) {
    if (a.files) {
        if (a.aligned) {
            EncArgs b = a;
            b.split = 2;
            hipLaunchKernelGGL((k_encode_compact<true>), dim3(grid), dim3(kEncThreads), 0, s, b);
            hipLaunchKernelGGL((k_encode<true, true>), dim3(grid), dim3(kEncThreads), 0, s, b);
        } else {
            hipLaunchKernelGGL((k_encode<true, false>), dim3(grid), dim3(kEncThreads), 0, s, a);
        }
    } else if (a.aligned) {
        EncArgs b = a;
        b.split = 1;
        const uint32_t grid2 = grid < kEncLongGrid ? grid : kEncLongGrid;
        hipLaunchKernelGGL((k_encode_compact<false>), dim3(grid), dim3(kEncThreads), 0, s, b);
        hipLaunchKernelGGL((k_encode<false, true>), dim3(grid2), dim3(kEncThreads), 0, s, b);
    } else {
        // an unaligned input's byte-wise loads would make the compact kernel spill
        hipLaunchKernelGGL((k_encode<false, false>), dim3(grid), dim3(kEncThreads), 0, s, a);
    }
    return hipGetLastError();
}

__global__ void k_encode_empty(uint64_t* chunk_off, uint32_t* sub_lo) {
    chunk_off[0] = 0;
    if (sub_lo) sub_lo[0] = 0;
}

hipError_t launch_encode_empty(uint64_t* chunk_off, uint32_t* sub_lo, hipStream_t s) {
    hipLaunchKernelGGL(k_encode_empty, dim3(1), dim3(1), 0, s, chunk_off, sub_lo);
    return hipGetLastError();
}

// ================================================================= decode
// Per-lane bit reader: a 64-bit window fed from a four-word register queue
// that is refilled with 16-byte loads one vector ahead.
struct BitReader {
    const uint4* vec;
    const uint32_t* w;
    uint64_t nwords;
    uint32_t q0, q1, q2, q3;  // queued words, q0 next
    uint32_t left;            // valid words in the queue
    uint4 nxt;                // the following vector, already in flight
    uint64_t vnext;
    uint64_t win;
    uint32_t avail;

    __device__ __forceinline__ uint4 load_vec(uint64_t vi) const {
        if ((vi + 1) * 4 <= nwords) return vec[vi];
        const uint64_t b = vi * 4;
        return make_uint4(b < nwords ? w[b] : 0u, b + 1 < nwords ? w[b + 1] : 0u, b + 2 < nwords ? w[b + 2] : 0u,
                          b + 3 < nwords ? w[b + 3] : 0u);
    }
    __device__ __forceinline__ uint32_t take() {
        const uint32_t r = q0;
        q0 = q1;
        q1 = q2;
        q2 = q3;
        if (--left == 0) {
            q0 = nxt.x;
            q1 = nxt.y;
            q2 = nxt.z;
            q3 = nxt.w;
            left = 4;
            nxt = load_vec(vnext++);
        }
        return r;
    }
    __device__ __forceinline__ void init(const uint32_t* words, uint64_t nw, uint64_t bit) {
        vec = reinterpret_cast<const uint4*>(words);
        w = words;
        nwords = nw;
        const uint64_t fw = bit >> 5;
        const uint4 c = load_vec(fw >> 2);
        nxt = load_vec((fw >> 2) + 1);
        vnext = (fw >> 2) + 2;
        q0 = c.x; q1 = c.y; q2 = c.z; q3 = c.w;
        left = 4;
        for (uint32_t s = (uint32_t)(fw & 3); s; --s) take();
        win = (uint64_t)take() << 32;
        win |= take();
        const uint32_t skip = (uint32_t)(bit & 31);
        win <<= skip;
        avail = 64 - skip;
    }
    __device__ __forceinline__ void refill() {
        if (avail < 32) {
            win |= (uint64_t)take() << (32 - avail);
            avail += 32;
        }
    }
};

// bits [pos, pos+64) of the stream, zero past nwords
__device__ __forceinline__ uint64_t peek64(const uint32_t* w, uint64_t nwords, uint64_t pos) {
    const uint64_t i = pos >> 5;
    const uint64_t a0 = i < nwords ? w[i] : 0u, a1 = i + 1 < nwords ? w[i + 1] : 0u, a2 = i + 2 < nwords ? w[i + 2] : 0u;
    const uint32_t s = (uint32_t)(pos & 31);
    const uint64_t hi = (a0 << 32) | a1;
    return s ? (hi << s) | (a2 >> (32 - s)) : hi;
}

// Canonical tables of one codebook, staged in LDS by every decode workgroup.
// The peek table is split into a length table and a byte table, so that a
// lookup needs no address scaling or field extraction and the length, which
// the next lookup waits for, comes straight from its own load.
template <uint32_t B>
struct alignas(16) DecTablesT {  // 16-byte aligned: the tables are filled with 4- to 16-byte stores
    static constexpr uint32_t kBits = B;
    uint8_t len8[1 << B];  // peek -> code length; 0: no code of at most lutBits bits
    uint8_t sym8[1 << B];  // peek -> byte
    unsigned long long first[64];
    uint32_t cnt[64], fidx[64];
    uint8_t sorted[256];
};
using DecTables = DecTablesT<HUFF_LUT_BITS>;
// The longer-code decoders' table: 12-bit peeks, so that codes of 11 and 12
// bits (most of the longer codes a byte alphabet gets) decode from the table.
// Codes longer still decode from a second table.  In a canonical code the
// longer codes take the largest values, so every code longer than 12 bits
// starts with one of the last 12-bit prefixes, [P, 4096), where P counts the
// prefixes the codes of at most 12 bits cover; the second table is indexed by
// the maxLen-bit peek minus P << (maxLen - 12) and has
// (4096 - P) << (maxLen - 12) entries, kept when at most kL2Max.
constexpr uint32_t kWideLutBits = 12;
constexpr uint32_t kL2Max = 2048;
struct DecTablesWide : DecTablesT<kWideLutBits> {
    uint8_t len2[kL2Max];  // second table: code length (0: no code)
    uint8_t sym2[kL2Max];  // second table: byte
};
// Where a lane finds the second-table entry of the 32 window bits `top`:
// min((top >> sh) - base, last).
struct L2Index {
    uint32_t sh, base, last;
};

static_assert(offsetof(huff_dcb, lut) % 16 == 0, "the peek table is read with 8-byte loads");

// Lengths (byte 1 of each u16 entry) and bytes (byte 0) of four peek-table
// entries held in two words.
__device__ __forceinline__ uint32_t lut_lens4(uint2 e) {
    return ((e.x >> 8) & 0xffu) | ((e.x >> 24) << 8) | (((e.y >> 8) & 0xffu) << 16) | ((e.y >> 24) << 24);
}
__device__ __forceinline__ uint32_t lut_syms4(uint2 e) {
    return (e.x & 0xffu) | (((e.x >> 16) & 0xffu) << 8) | ((e.y & 0xffu) << 16) | (((e.y >> 16) & 0xffu) << 24);
}

template <class Tab>
__device__ __forceinline__ void load_tables(Tab& t, const huff_dcb* cb, uint32_t lutBits) {
    const uint32_t nl = 1u << min(lutBits, (uint32_t)HUFF_LUT_BITS);
    if (nl == 4 * blockDim.x) {
        // the full table: four entries per thread, one 8-byte load, one
        // 4-byte store per table (the codebook's table starts 16-byte aligned)
        const uint2 e = reinterpret_cast<const uint2*>(cb->lut)[threadIdx.x];
        reinterpret_cast<uint32_t*>(t.len8)[threadIdx.x] = lut_lens4(e);
        reinterpret_cast<uint32_t*>(t.sym8)[threadIdx.x] = lut_syms4(e);
    } else {
        for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) {
            const uint32_t e = cb->lut[i];
            t.len8[i] = (uint8_t)(e >> 8);
            t.sym8[i] = (uint8_t)e;
        }
    }
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) {
        t.first[i] = cb->first_code[i];
        t.cnt[i] = cb->count[i];
        t.fidx[i] = cb->first_index[i];
    }
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) t.sorted[i] = cb->sorted_sym[i];
}

// The wide table of a codebook whose codes are longer than its own peek
// table (cb->lut_bits = HUFF_LUT_BITS bits): entry i (wideBits bits) repeats
// the codebook's entry for its first lut_bits bits when that entry has a
// code; otherwise the code starting with i is longer than lut_bits, and a
// canonical search over the lengths up to wideBits finds it (0 if it is
// longer still).  For codes of 13 to 32 bits the second table is filled the
// same way over the lengths past wideBits; the return value says where its
// entries are, with last = 0 when it is not built (the code is too long, or
// the table would pass kL2Max), so that such codes take the canonical search
// at decode time.  The canonical tables are loaded as by load_tables.
__device__ __forceinline__ L2Index load_tables_wide(DecTablesWide& t, const huff_dcb* cb, uint32_t wideBits,
                                                    uint32_t maxLen) {
    // the canonical tables first, and the codebook's peek entries into
    // registers: after one barrier the searches below read LDS, not memory
    const uint32_t lb = cb->lut_bits, sh = wideBits - lb;
    const uint32_t lmax = min(wideBits, maxLen);
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) {
        t.first[i] = cb->first_code[i];
        t.cnt[i] = cb->count[i];
        t.fidx[i] = cb->first_index[i];
    }
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) t.sorted[i] = cb->sorted_sym[i];
    constexpr uint32_t kPer = (1u << HUFF_LUT_BITS) / 256;  // entries per thread (256-thread workgroups)
    uint32_t ev[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = threadIdx.x + 256 * k;
        ev[k] = j < (1u << lb) ? cb->lut[j] : 0u;
    }
    __syncthreads();
    auto search = [&](uint64_t code, uint32_t bits, uint32_t l0, uint32_t l1, uint32_t& len, uint32_t& sym) {
        // the code of l0..l1 bits that the `bits`-bit value `code` starts with
        for (uint32_t l = l0; l <= l1; ++l) {
            const uint64_t c = code >> (bits - l);
            if (c - t.first[l] < t.cnt[l]) {
                sym = t.sorted[t.fidx[l] + (uint32_t)(c - t.first[l])];
                len = l;
                return;
            }
        }
    };
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = threadIdx.x + 256 * k;
        if (j < (1u << lb)) {
            const uint32_t e = ev[k];
            for (uint32_t r = 0; r < (1u << sh); ++r) {
                const uint32_t i = (j << sh) | r;
                uint32_t len = e >> 8, sym = e & 0xffu;
                if (len == 0) search(i, wideBits, lb + 1, lmax, len, sym);
                t.len8[i] = (uint8_t)len;
                t.sym8[i] = (uint8_t)sym;
            }
        }
    }
    L2Index l2 = {0u, 0u, 0u};
    if (wideBits == kWideLutBits && maxLen > wideBits && maxLen <= 32) {
        const uint64_t P = cb->first_code[wideBits] + cb->count[wideBits];
        const uint32_t extra = maxLen - wideBits;
        const uint64_t n2 = P < (1ull << wideBits) ? ((1ull << wideBits) - P) << extra : 0ull;
        if (n2 > 0 && n2 <= kL2Max) {
            const uint64_t base = P << extra;  // maxLen-bit value of the second table's entry 0
            for (uint32_t i = threadIdx.x; i < (uint32_t)n2; i += blockDim.x) {
                uint32_t len = 0, sym = 0;
                search(base + i, maxLen, wideBits + 1, maxLen, len, sym);
                t.len2[i] = (uint8_t)len;
                t.sym2[i] = (uint8_t)sym;
            }
            l2 = {32u - maxLen, (uint32_t)base, (uint32_t)n2 - 1u};
        }
    }
    return l2;
}

// Codes longer than the table: canonical search on the top 32 window bits.
// Returns sym | len << 8, or 0 if no code matches.
template <class Tab>
__device__ __noinline__ uint32_t decode_long(const Tab& t, uint32_t top, uint32_t lutBits, uint32_t maxLen) {
    for (uint32_t l = lutBits + 1; l <= maxLen; ++l) {
        const uint64_t c = top >> (32 - l);
        if (c - t.first[l] < t.cnt[l]) return t.sorted[t.fidx[l] + (uint32_t)(c - t.first[l])] | (l << 8);
    }
    return 0;
}

// Reader over words staged in LDS (word 0 = the first staged stream word).
// The refill has no branch: `pre` always holds the word at index `nxt` and is
// re-read after every symbol, so the word a refill takes was loaded at least
// one symbol earlier and the refill never waits for LDS.  Indexes are clamped
// to the wave's buffer; words past a sub-block's end only ever fill the
// window's tail, which the table lookups of its last codes do not depend on.
struct LdsReader {
    const uint32_t* s;
    uint32_t last, nxt, pre;  // last: index of the buffer's last word
    uint64_t win;
    uint32_t avail;
    __device__ __forceinline__ uint32_t at(uint32_t i) const { return s[i < last ? i : last]; }
    __device__ __forceinline__ void init(const uint32_t* s_, uint32_t lim, uint32_t bit) {
        s = s_;
        last = lim - 1;
        const uint32_t wi = bit >> 5, sk = bit & 31;
        win = (((uint64_t)at(wi) << 32) | at(wi + 1)) << sk;
        avail = 64 - sk;
        nxt = wi + 2;
        pre = at(nxt);
    }
    __device__ __forceinline__ void refill() {
        const bool need = avail < 32;
        const uint64_t add = (uint64_t)pre << ((32u - avail) & 63u);
        win |= need ? add : 0ull;
        avail += need ? 32u : 0u;
        nxt += need ? 1u : 0u;
        pre = at(nxt);
    }
};

// One symbol from a reader whose window holds >= 32 valid bits after refill.
// Reader for the table-only decoder over words staged in LDS: every k
// symbols it re-reads the 64 stream bits at its position and otherwise only
// shifts.  A window read at most 31 bits into a word holds at least 33 bits
// ahead of the position, enough for k codes of at most maxLen bits and the
// lutBits peek of the last of them when (k - 1) * maxLen + lutBits <= 33.
struct WinReader {
    const uint32_t* s;
    uint32_t last;     // index of the buffer's last word
    uint32_t pos;      // bit position of the window's first bit
    uint32_t cons;     // bits consumed from the window
    uint32_t c, k;     // symbols taken from the window, symbols per window
    uint64_t win;
    __device__ __forceinline__ void init(const uint32_t* s_, uint32_t lim, uint32_t bit, uint32_t k_) {
        s = s_;
        last = lim - 1;
        pos = bit;
        cons = 0;
        c = k = k_;
        win = 0;
    }
    template <class Tab>
    __device__ __forceinline__ uint32_t next(const Tab& t, uint32_t lutBits, uint32_t& emin) {
        if (c == k) {
            pos += cons;
            const uint32_t w = min(pos >> 5, last - 1);
            win = (((uint64_t)s[w] << 32) | s[w + 1]) << (pos & 31);
            cons = 0;
            c = 0;
        }
        const uint32_t idx = (uint32_t)(win >> 32) >> (32 - lutBits);
        const uint32_t len = t.len8[idx];
        emin = min(emin, len);
        win <<= len;
        cons += len;
        ++c;
        return t.sym8[idx];
    }
    // The same with the second table for codes past the wide peek table
    // (k * maxLen <= 33, so that the window still holds maxLen bits at the
    // last of its k codes).
    __device__ __forceinline__ uint32_t next2(const DecTablesWide& t, uint32_t lutBits, const L2Index& l2,
                                              uint32_t& emin) {
        if (c == k) {
            pos += cons;
            const uint32_t w = min(pos >> 5, last - 1);
            win = (((uint64_t)s[w] << 32) | s[w + 1]) << (pos & 31);
            cons = 0;
            c = 0;
        }
        const uint32_t top = (uint32_t)(win >> 32);
        const uint32_t idx = top >> (32 - lutBits);
        uint32_t len = t.len8[idx], sym = t.sym8[idx];
        if (len == 0) {
            const uint32_t i2 = min((top >> l2.sh) - l2.base, l2.last);
            len = t.len2[i2];
            sym = t.sym2[i2];
        }
        emin = min(emin, len);
        win <<= len;
        cons += len;
        ++c;
        return sym;
    }
};

// kFits: every code is at most lutBits long, so the table alone decodes; a
// table length of 0 (no code matches) is then kept in emin (the least length
// seen) and reported by the caller instead of being branched on per symbol.
template <bool kFits, class Rd, typename U, class Tab>
__device__ __forceinline__ uint32_t dec1(Rd& r, const Tab& t, uint32_t lutBits, uint32_t maxLen, bool& bad,
                                         U& used, uint32_t& emin) {
    r.refill();
    const uint32_t top = (uint32_t)(r.win >> 32);
    const uint32_t idx = top >> (32 - lutBits);
    uint32_t len = t.len8[idx], sym = t.sym8[idx];
    if constexpr (kFits) {
        emin = min(emin, len);
    } else if (len == 0) {
        const uint32_t e = decode_long(t, top, lutBits, maxLen);
        if (e == 0) bad = true;
        len = e ? e >> 8 : 1u;
        sym = e & 0xffu;
    }
    r.win <<= len;
    r.avail -= len;
    used += len;
    return sym;
}

// The windowed reader decodes from the table alone; bits used are counted by
// its position, not here.
template <bool kFits, typename U, class Tab>
__device__ __forceinline__ uint32_t dec1(WinReader& r, const Tab& t, uint32_t lutBits, uint32_t maxLen, bool& bad,
                                         U& used, uint32_t& emin) {
    return r.next(t, lutBits, emin);
}

constexpr int kDecLine = 64;  // bytes a decode lane stores together

// 16 symbols, packed into 16 bytes in stream order.
template <bool kFits, class Rd, typename U, class Tab>
__device__ __forceinline__ uint4 dec16(Rd& r, const Tab& t, uint32_t lutBits, uint32_t maxLen, bool& bad, U& used,
                                       uint32_t& emin) {
    uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        o[i >> 2] |= dec1<kFits>(r, t, lutBits, maxLen, bad, used, emin) << (8 * (i & 3));
        asm volatile("" : "+v"(o[i >> 2]), "+v"(emin));  // pack now: keeps table entries from staying live
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// Decodes nsym symbols into out (16-byte aligned).  Each lane writes its own
// region, so the lanes of one store instruction hit different cache lines; a
// line written 16 bytes at a time, far apart in time, leaves L2 in pieces.
// A lane therefore holds its last kLine / 16 groups of 16 decoded bytes in a
// register queue and stores them together once kLine bytes are complete, so
// that every kLine-byte piece of a line is written whole.
template <int kLine, bool kFits, class Rd, typename U, class Tab>
__device__ __forceinline__ void dec_run_k(Rd& r, const Tab& t, uint32_t lutBits, uint32_t maxLen, bool& bad,
                                          U& used, uint8_t* out, uint32_t nsym) {
    uint32_t emin = 0xffffffffu;
    constexpr uint32_t kG = kLine / 16;  // groups held before they are stored
    uint4* o4 = reinterpret_cast<uint4*>(out);
    const uint32_t groups = nsym >> 4;
    uint4 q[kG];  // q[kG - 1] is the newest group
#pragma unroll
    for (uint32_t k = 0; k < kG; ++k) q[k] = make_uint4(0, 0, 0, 0);
#pragma unroll 1
    for (uint32_t gi = 0; gi < groups; ++gi) {
        const uint4 v = dec16<kFits>(r, t, lutBits, maxLen, bad, used, emin);
#pragma unroll
        for (uint32_t k = 0; k + 1 < kG; ++k) q[k] = q[k + 1];
        q[kG - 1] = v;
        if (((gi + 1) & (kG - 1)) == 0) {
#pragma unroll
            for (uint32_t k = 0; k < kG; ++k) o4[gi + 1 - kG + k] = q[k];
        }
    }
    // groups left in the queue: the last (groups mod kG)
    const uint32_t rest = groups & (kG - 1);
#pragma unroll
    for (uint32_t k = 0; k < kG; ++k)
        if (k + rest >= kG) o4[groups - kG + k] = q[k];
    for (uint32_t i = groups << 4; i < nsym; ++i) out[i] = (uint8_t)dec1<kFits>(r, t, lutBits, maxLen, bad, used, emin);
    if (kFits && emin == 0u) bad = true;
}

// Picks the table-only decoder when every code fits the table.
template <int kLine, class Rd, typename U, class Tab>
__device__ __forceinline__ void dec_run(Rd& r, const Tab& t, uint32_t lutBits, uint32_t maxLen, bool& bad,
                                        U& used, uint8_t* out, uint32_t nsym) {
    if (maxLen <= lutBits) dec_run_k<kLine, true>(r, t, lutBits, maxLen, bad, used, out, nsym);
    else dec_run_k<kLine, false>(r, t, lutBits, maxLen, bad, used, out, nsym);
}

// Codes longer than 32 bits: canonical search on a 64-bit peek from memory.
template <class Tab>
__device__ void decode_generic(const FileDesc& f, const Tab& t, uint32_t maxLen, uint64_t start, uint64_t nsym,
                               uint8_t* out, bool& bad, uint64_t& used) {
    uint64_t pos = start;
    for (uint64_t i = 0; i < nsym; ++i) {
        const uint64_t top = peek64(f.words, f.nwords, pos);
        uint32_t len = 0, sym = 0;
        for (uint32_t l = 1; l <= maxLen; ++l) {
            const uint64_t c = top >> (64 - l);
            if (c - t.first[l] < t.cnt[l]) {
                sym = t.sorted[t.fidx[l] + (uint32_t)(c - t.first[l])];
                len = l;
                break;
            }
        }
        if (len == 0) { bad = true; len = 1; }
        out[i] = (uint8_t)sym;
        pos += len;
        used += len;
    }
}

// Start/end stream bits of decode item j (a sub-block, or a chunk without sub index).
__device__ __forceinline__ void item_bits(const FileDesc& f, const DecArgs& a, uint64_t j, uint64_t nitems,
                                          uint64_t& start, uint64_t& end) {
    const uint32_t il = a.item_log2, cl = a.chunk_log2;
    if (a.use_sub) {
        const uint64_t base = f.chunk_off[(j << il) >> cl];
        start = base + (uint32_t)(f.sub_lo[j] - (uint32_t)base);
        if (j + 1 == nitems) {
            end = f.chunk_off[(f.n + (1ull << cl) - 1) >> cl];
        } else {
            const uint64_t b2 = f.chunk_off[((j + 1) << il) >> cl];
            end = b2 + (uint32_t)(f.sub_lo[j + 1] - (uint32_t)b2);
        }
    } else {
        start = f.chunk_off[j];
        end = f.chunk_off[j + 1];
    }
}

// Direct decoder: one lane per item, words read straight from memory.  Used
// for chunk-only indexes and sub-blocks that the staged decoder (k_decode_lds)
// does not take.
template <bool kBatch>
__global__ __launch_bounds__(256) void k_decode(DecArgs a) {
    __shared__ DecTables t;
    const uint64_t item = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    FileDesc f;
    if constexpr (kBatch) f = a.files[dec_file(a, (uint64_t)blockIdx.x * blockDim.x)];
    else f = a.one;
    const huff_dcb* cb = f.cb;
    const uint32_t lutBits = cb->lut_bits, maxLen = cb->max_len;
    load_tables(t, cb, lutBits);
    __syncthreads();

    const uint64_t j = item - f.first;
    const uint64_t n = f.n;
    const uint32_t il = a.item_log2;
    const uint64_t nitems = (n + (1ull << il) - 1) >> il;
    if (j >= nitems) return;
    uint64_t start, end;
    item_bits(f, a, j, nitems, start, end);
    const uint64_t first = j << il;
    const uint64_t nsym = min<uint64_t>(1ull << il, n - first);
    uint8_t* out = f.out + first;
    bool bad = start > end || end > f.nwords * 32ull || maxLen == 0 || maxLen > HUFF_MAX_CODE_LEN;
    uint64_t used = 0;
    if (!bad && maxLen <= 32) {
        BitReader br;
        br.init(f.words, f.nwords, start);
        if ((((uintptr_t)out) & 15u) == 0) {
            dec_run<kDecLine>(br, t, lutBits, maxLen, bad, used, out, (uint32_t)nsym);
        } else {
            uint32_t emin = 0;  // unused by the general decoder
            for (uint64_t i = 0; i < nsym; ++i) out[i] = (uint8_t)dec1<false>(br, t, lutBits, maxLen, bad, used, emin);
        }
    } else if (!bad) {
        decode_generic(f, t, maxLen, start, nsym, out, bad, used);
    }
    if (bad || start + used != end) report(f.status, a.err, HUFF_E_CORRUPT);
}

// Lengths of a complete canonical code that spans at most three lengths,
// by comparison: the codes of length l, left-justified to 32 bits, fill one
// range that ends where those of length l + 1 begin, so the length of the
// code at the top of the window is `base` plus the number of the limits
// (left-justified first codes of the longer lengths) that the top 32 bits
// reach.  This keeps the table read off the chain from one code to the next.
struct LenCmp {
    uint32_t base, lim1, lim2;
};

// S symbols of one lane's sub-block into registers, 16 per uint4 in stream
// order, for codes that all fit the peek table.  The 64 stream bits at the
// position are re-read from LDS (three words, shifted) every K symbols, at
// positions fixed at compile time, so the unrolled run has no branch: the
// window holds 64 bits ahead, enough for K codes of at most maxLen bits and
// the peek of the last when (K - 1) * maxLen + lutBits <= 64.  NC = 0: lengths from the length table
// (a length of 0, no code, is kept in emin); NC = 3: the same for a complete
// code, where every table entry has a code and nothing is kept; NC = 1 or 2:
// lengths from NC comparisons (LenCmp); NC = 4: codes longer than the wide
// peek table from its second table (`l2`), with K * maxLen <= 64.  Each byte is packed as soon as it is
// decoded, so the table entries do not stay live.  pos: bit position in the
// buffer, advanced past the S codes.
template <int S, int K, int NC, class Tab>
__device__ __forceinline__ void dec_lane_fits(const uint32_t* s, uint32_t last, uint32_t& pos, const Tab& t,
                                              uint32_t lutBits, const LenCmp lc, uint4 (&o)[S / 16],
                                              uint32_t& emin, const L2Index l2 = {0u, 0u, 0u}) {
    uint64_t win = 0;
    uint32_t cons = 0;
#pragma unroll
    for (uint32_t g = 0; g < S / 16; ++g) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) {
            if ((g * 16 + i) % K == 0) {
                pos += cons;
                const uint32_t wi = min(pos >> 5, last - 2), sh = pos & 31;
                win = ((((uint64_t)s[wi] << 32) | s[wi + 1]) << sh) | (((uint64_t)s[wi + 2] << sh) >> 32);
                cons = 0;
            }
            const uint32_t top = (uint32_t)(win >> 32);
            const uint32_t idx = top >> (32 - lutBits);
            uint32_t len;
            if constexpr (NC == 4) {
                len = t.len8[idx];
                uint32_t sym = t.sym8[idx];
                if (len == 0) {
                    const uint32_t i2 = min((top >> l2.sh) - l2.base, l2.last);
                    len = t.len2[i2];
                    sym = t.sym2[i2];
                }
                emin = min(emin, len);
                win <<= len;
                cons += len;
                w[i >> 2] |= sym << (8 * (i & 3));
                if ((i & 3) == 3) asm volatile("" : "+v"(w[i >> 2]), "+v"(emin));
                continue;
            } else if constexpr (NC == 0) {
                len = t.len8[idx];
                emin = min(emin, len);
            } else if constexpr (NC == 3) {
                len = t.len8[idx];
            } else {
                len = lc.base + (top >= lc.lim1 ? 1u : 0u);
                if constexpr (NC == 2) len += top >= lc.lim2 ? 1u : 0u;
            }
            win <<= len;
            cons += len;
            w[i >> 2] |= (uint32_t)t.sym8[idx] << (8 * (i & 3));
            if ((i & 3) == 3) asm volatile("" : "+v"(w[i >> 2]), "+v"(emin));
        }
        o[g] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    pos += cons;
}

// Stores a whole wave's decoded sub-blocks (lane l holds bytes [l*S, l*S+S)
// of the wave's output) through the wave's LDS buffer, which the wave no
// longer reads: afterwards every store instruction writes 1 KB of
// contiguous output, so every output line is written whole at once.  A
// lane's g-th 16 bytes sit in LDS slot lane * G + ((g + lane) mod G), which
// spreads one instruction's lanes over the banks.
template <int S>
__device__ __forceinline__ void wave_store(const uint4 (&o)[S / 16], uint32_t* buf, uint8_t* wave_out, int lane) {
    constexpr uint32_t G = S / 16;
    wave_lds_sync();
    uint4* l4 = reinterpret_cast<uint4*>(buf);
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) l4[lane * G + ((g + lane) & (G - 1))] = o[g];
    wave_lds_sync();
    uint4* g4 = reinterpret_cast<uint4*>(wave_out);
#pragma unroll
    for (uint32_t i = 0; i < G; ++i) {
        const uint32_t e = i * 64 + lane, lp = e / G, g = e & (G - 1);
        g4[e] = l4[lp * G + ((g + lp) & (G - 1))];
    }
}

// 64-bit lane value of lane l (l uniform).
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, uint32_t l) {
    return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((uint32_t)v, l);
}

// Copies stream words [base, base + 4 * nv) into a wave's LDS buffer with
// 16-byte loads (nv <= kMaxV); words past the stream read as zero.  A lane
// issues its loads four at a time before it writes them to LDS, so the copy
// costs one memory round trip per four loads, not one per load, and holds
// only four of them in registers.
template <uint32_t kMaxV>
__device__ __forceinline__ void stage_words(const FileDesc& f, uint64_t base, uint32_t nv, uint32_t* buf, int lane) {
    constexpr uint32_t kPer = (kMaxV + 63) / 64, kBatch = 4;
    const uint4* src = reinterpret_cast<const uint4*>(f.words) + (base >> 2);
    uint4* dst = reinterpret_cast<uint4*>(buf);
#pragma unroll
    for (uint32_t r0 = 0; r0 < kPer; r0 += kBatch) {
        uint4 q[kBatch];
#pragma unroll
        for (uint32_t r = 0; r < kBatch; ++r) {
            const uint32_t v = lane + 64 * (r0 + r);
            const uint64_t wi = base + 4ull * v;
            q[r] = make_uint4(0, 0, 0, 0);
            if (r0 + r < kPer && v < nv) {
                if (wi + 4 <= f.nwords) {
                    q[r] = src[v];
                } else {
                    q[r].x = wi < f.nwords ? f.words[wi] : 0u;
                    q[r].y = wi + 1 < f.nwords ? f.words[wi + 1] : 0u;
                    q[r].z = wi + 2 < f.nwords ? f.words[wi + 2] : 0u;
                    q[r].w = wi + 3 < f.nwords ? f.words[wi + 3] : 0u;
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < kBatch; ++r)
            if (r0 + r < kPer && lane + 64 * (r0 + r) < nv) dst[lane + 64 * (r0 + r)] = q[r];
    }
}

// Which codebooks a staged decode launch takes: those whose codes all fit
// the peek table, the others, or both.  For sub-blocks of up to 64 bytes the
// first two are separate kernels, so that the registers of the longer-code
// path do not limit the occupancy of the table-only path (every block of a
// launch that its codebook does not belong to exits at once); from 128 bytes
// the LDS buffer limits occupancy first, and one kernel takes both.
enum : int { kDecFits = 0, kDecLong = 1, kDecBoth = 2 };

// Staged decoder for sub-blocks of S bytes (S = 32..256).  Each wave takes
// 64 consecutive sub-blocks, one per lane: their stream bits are contiguous,
// so the wave copies them once into its LDS buffer (sized for 8 bits per
// byte) with 16-byte loads, and every lane decodes its sub-block from LDS.
// A wave whose bits do not fit is staged in parts (halves, quarters, ... of
// its lanes, one part after another).
// Table-only codes: every whole sub-block is decoded into registers and the
// wave stores them at the end, through LDS when all 64 are whole; the short
// last sub-block of a stream is decoded byte by byte.  Longer codes: each
// lane decodes with a refilled window and stores 64 bytes at a time; codes
// longer than 32 bits are decoded straight from memory.
template <int S, class Tab>
struct StagedLds {
    uint32_t in[4][64 * S / 4 + 8];
    Tab t;
};
// The tables a staged launch takes: the longer-code launch (a kernel of its
// own below 128-byte sub-blocks) peeks 12 bits.
template <int S, int kMode>
using StagedLdsFor = StagedLds<S, typename std::conditional<kMode == kDecLong, DecTablesWide, DecTables>::type>;

// One block of 256 decode lanes (`blk`); every return below is either taken
// by the whole workgroup or comes after the workgroup's last barrier.
template <int S, bool kBatch, int kMode>
__device__ __forceinline__ void dec_staged_block(const DecArgs& a, uint64_t blk, StagedLdsFor<S, kMode>& sm) {
    constexpr uint32_t kInWords = 64 * S / 4 + 8;
    constexpr uint32_t G = S / 16;
    constexpr int kLine = S < kDecLine ? S : kDecLine;
    auto& s_in = sm.in;
    auto& t = sm.t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    FileDesc f;
    if constexpr (kBatch) {
        // the other launch's block: one load of its mode, no file or codebook reads
        if (kMode != kDecBoth && a.blk_mode && (a.blk_mode[blk] != 0) != (kMode == kDecLong)) return;
        f = a.files[dec_file(a, blk * 256)];
    } else {
        f = a.one;
    }
    const huff_dcb* cb = f.cb;
    const uint32_t cbBits = cb->lut_bits, maxLen = cb->max_len;
    if (kMode != kDecBoth && (maxLen <= cbBits) != (kMode == kDecFits)) return;  // the other launch decodes this block
    if (maxLen == 0 || maxLen > HUFF_MAX_CODE_LEN || cbBits == 0 || cbBits > HUFF_LUT_BITS) {
        if (tid == 0) report(f.status, a.err, HUFF_E_CORRUPT);
        return;
    }
    // the longer-code launch peeks up to kWideLutBits bits: codes that fit
    // them decode from the table alone, like the first launch's
    uint32_t lutBits = cbBits;
    L2Index l2 = {0u, 0u, 0u};
    if constexpr (kMode == kDecLong) {
        lutBits = min(maxLen, kWideLutBits);
        l2 = load_tables_wide(t, cb, lutBits, maxLen);
    } else {
        load_tables(t, cb, lutBits);
    }
    const bool fits = maxLen <= lutBits;
    const bool two = !fits && l2.last != 0;  // longer codes from the second table (the table has >= 2 entries)

    const uint64_t n = f.n;
    const uint64_t nitems = (n + S - 1) / S;
    const uint64_t j0 = blk * 256 + wave * 64 - f.first;  // first item of this wave
    const uint64_t j = j0 + lane;
    const bool active = j < nitems;
    uint64_t start = 0, end = 0;
    if (active) item_bits(f, a, j, nitems, start, end);
    const uint32_t nsym = active ? (uint32_t)min<uint64_t>(S, n - j * S) : 0;
    bool bad = start > end || end > f.nwords * 32ull;
    const bool direct = !fits && maxLen > 32;  // codes past the readers' 32-bit window

    // parts: the smallest power of two P such that every run of 64 / P lanes fits the buffer
    const bool wave_on = j0 < nitems;
    const uint32_t la = wave_on ? (uint32_t)min<uint64_t>(63, nitems - 1 - j0) : 0;  // last active lane
    uint32_t P = 1;
    if (wave_on && !direct) {
        for (;;) {
            bool ok = true;
            for (uint32_t l0 = 0; l0 <= la && ok; l0 += 64 / P) {
                const uint64_t ws = read_lane_u64(start, l0), we = read_lane_u64(end, min(l0 + 64 / P - 1, la));
                ok = we < ws || ((we + 31) >> 5) - ((ws >> 5) & ~3ull) + 4 <= kInWords;
            }
            if (ok || P == 64) break;
            P *= 2;
        }
    }

    // the first part (the whole wave when P = 1) is staged before the barrier
    // that also publishes the tables
    const uint32_t l1 = min(64 / P - 1, la);
    uint64_t base = 0;
    if (wave_on && !direct) {
        const uint64_t ws = read_lane_u64(start, 0), we = read_lane_u64(end, l1);
        base = (ws >> 5) & ~3ull;
        const uint64_t cnt = we >= ws ? ((we + 31) >> 5) - base : 0;
        stage_words<kInWords / 4>(f, base, (uint32_t)min<uint64_t>((cnt + 3) >> 2, kInWords / 4), s_in[wave], lane);
    }
    __syncthreads();

    uint32_t used = 0;
    if (P == 1) {
        if (active && !direct) {
            const uint32_t bit0 = (uint32_t)(start - (base << 5));
            if (fits) {
                const uint32_t k = (33u - lutBits) / maxLen + 1;  // symbols a re-read 33-bit window covers
                const uint32_t k64 = (64u - lutBits) / maxLen + 1;  // ... and a 64-bit one
                uint32_t emin = 0xffffffffu;
                if (nsym == S) {
                    uint4 o[G];
                    uint32_t pos = bit0;
                    // a complete code of at most three lengths: lengths by comparison
                    uint32_t minLen = maxLen;
                    for (uint32_t l = maxLen; l >= 1; --l)
                        if (t.cnt[l]) minLen = l;
                    const uint32_t span = maxLen - minLen;
                    const bool complete = t.first[maxLen] + t.cnt[maxLen] == (1ull << maxLen);
                    // Comparisons take the table read off the chain from one
                    // code to the next but cost more VALU per symbol: they pay
                    // where the LDS buffer of larger sub-blocks keeps few waves
                    // on a SIMD; with 64-byte sub-blocks (8 waves per SIMD) the
                    // decoder is bound by VALU issue and reads the table.
                    const bool cmp = S >= 128 && span <= 2 && k >= 4 && complete;
                    LenCmp lc = {0u, 0u, 0u};
                    if (span == 0) {
                        lc.base = minLen - 1;  // one length: the comparison with 0 always adds 1
                    } else {
                        lc.base = minLen;
                        lc.lim1 = (uint32_t)(t.first[minLen + 1] << (32 - (minLen + 1)));
                        if (span == 2) lc.lim2 = (uint32_t)(t.first[minLen + 2] << (32 - (minLen + 2)));
                    }
                    uint32_t* sb = s_in[wave];
                    if (cmp && span == 2) {
                        if (k64 >= 8) dec_lane_fits<S, 8, 2>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                        else dec_lane_fits<S, 4, 2>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    } else if (cmp) {
                        if (k64 >= 8) dec_lane_fits<S, 8, 1>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                        else dec_lane_fits<S, 4, 1>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    } else if (complete) {
                        if (k64 >= 8) dec_lane_fits<S, 8, 3>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                        else if (k64 >= 6) dec_lane_fits<S, 6, 3>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                        else dec_lane_fits<S, 4, 3>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    } else if (k64 >= 8) {  // k64 >= 5 here: maxLen <= lutBits <= 12
                        dec_lane_fits<S, 8, 0>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    } else if (k64 >= 6) {
                        dec_lane_fits<S, 6, 0>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    } else {
                        dec_lane_fits<S, 4, 0>(sb, kInWords - 1, pos, t, lutBits, lc, o, emin);
                    }
                    used = pos - bit0;
                    if ((j0 + 64) * S <= n) {
                        wave_store<S>(o, s_in[wave], f.out + j0 * S, lane);
                    } else {
                        uint4* o4 = reinterpret_cast<uint4*>(f.out + j * S);
#pragma unroll
                        for (uint32_t g = 0; g < G; ++g) o4[g] = o[g];
                    }
                } else {
                    WinReader rd;
                    rd.init(s_in[wave], kInWords, bit0, k);
                    uint8_t* out = f.out + j * S;
                    for (uint32_t i = 0; i < nsym; ++i) out[i] = (uint8_t)rd.next(t, lutBits, emin);
                    used = rd.pos + rd.cons - bit0;
                }
                if (emin == 0u) bad = true;
            } else if (two) {
                if constexpr (kMode == kDecLong) {
                    const uint32_t k2 = 33u / maxLen;  // codes a re-read 33-bit window covers: 1 or 2
                    const uint32_t k64 = 64u / maxLen;  // ... and a 64-bit one: 2 to 4
                    uint32_t emin = 0xffffffffu;
                    if (nsym == S) {
                        uint4 o[G];
                        uint32_t pos = bit0;
                        const LenCmp lc = {0u, 0u, 0u};
                        if (k64 >= 4) dec_lane_fits<S, 4, 4>(s_in[wave], kInWords - 1, pos, t, lutBits, lc, o, emin, l2);
                        else if (k64 >= 3) dec_lane_fits<S, 3, 4>(s_in[wave], kInWords - 1, pos, t, lutBits, lc, o, emin, l2);
                        else dec_lane_fits<S, 2, 4>(s_in[wave], kInWords - 1, pos, t, lutBits, lc, o, emin, l2);
                        used = pos - bit0;
                        if ((j0 + 64) * S <= n) {
                            wave_store<S>(o, s_in[wave], f.out + j0 * S, lane);
                        } else {
                            uint4* o4 = reinterpret_cast<uint4*>(f.out + j * S);
#pragma unroll
                            for (uint32_t g = 0; g < G; ++g) o4[g] = o[g];
                        }
                    } else {
                        WinReader rd;
                        rd.init(s_in[wave], kInWords, bit0, k2);
                        uint8_t* out = f.out + j * S;
                        for (uint32_t i = 0; i < nsym; ++i) out[i] = (uint8_t)rd.next2(t, lutBits, l2, emin);
                        used = rd.pos + rd.cons - bit0;
                    }
                    if (emin == 0u) bad = true;
                }
            } else {
                LdsReader rd;
                rd.init(s_in[wave], kInWords, bit0);
                dec_run_k<kLine, false>(rd, t, lutBits, maxLen, bad, used, f.out + j * S, nsym);
            }
        }
    } else {
        // parts of 64 / P lanes, one after another, each lane storing its own bytes
        for (uint32_t p = 0; p < P; ++p) {
            const uint32_t q0 = p * (64 / P), q1 = min(q0 + 64 / P - 1, la);
            if (q0 > la) break;
            if (p > 0) {
                wave_lds_sync();  // the previous part's lanes are done with the buffer
                const uint64_t ws = read_lane_u64(start, q0), we = read_lane_u64(end, q1);
                base = (ws >> 5) & ~3ull;
                const uint64_t cnt = we >= ws ? ((we + 31) >> 5) - base : 0;
                stage_words<kInWords / 4>(f, base, (uint32_t)min<uint64_t>((cnt + 3) >> 2, kInWords / 4), s_in[wave], lane);
                wave_lds_sync();
            }
            if (!active || lane < (int)q0 || lane > (int)q1) continue;
            const uint32_t bit0 = (uint32_t)(start - (base << 5));
            uint8_t* out = f.out + j * S;
            uint32_t emin = 0xffffffffu;
            if (fits) {
                WinReader rd;
                rd.init(s_in[wave], kInWords, bit0, (33u - lutBits) / maxLen + 1);
                for (uint32_t i = 0; i < nsym; ++i) out[i] = (uint8_t)rd.next(t, lutBits, emin);
                if (emin == 0u) bad = true;
                used = rd.pos + rd.cons - bit0;
            } else if (two) {
                if constexpr (kMode == kDecLong) {
                    WinReader rd;
                    rd.init(s_in[wave], kInWords, bit0, 33u / maxLen);
                    for (uint32_t i = 0; i < nsym; ++i) out[i] = (uint8_t)rd.next2(t, lutBits, l2, emin);
                    if (emin == 0u) bad = true;
                    used = rd.pos + rd.cons - bit0;
                }
            } else {
                LdsReader rd;
                rd.init(s_in[wave], kInWords, bit0);
                for (uint32_t i = 0; i < nsym; ++i) out[i] = (uint8_t)dec1<false>(rd, t, lutBits, maxLen, bad, used, emin);
            }
        }
    }
    if (!active) return;
    if (direct) {
        if (!bad) {
            uint64_t u = 0;
            decode_generic(f, t, maxLen, start, nsym, f.out + j * S, bad, u);
            if (start + u != end) bad = true;
        }
    } else if (start + used != end) {
        bad = true;
    }
    if (bad) report(f.status, a.err, HUFF_E_CORRUPT);
}

// One workgroup per block of 256 lanes.
template <int S, bool kBatch, int kMode>
__global__ __launch_bounds__(256) void k_decode_lds(DecArgs a) {
    __shared__ StagedLdsFor<S, kMode> sm;
    dec_staged_block<S, kBatch, kMode>(a, blockIdx.x, sm);
}

// The longer-code launch of one stream below 128 bytes: workgroup b takes blocks b,
// b + grid, ...  (kept apart from k_decode_lds: the loop costs the
// table-only path registers, about 64 -> 124 VGPRs at 64 bytes, held to
// four waves per SIMD).
template <int S, bool kBatch>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_decode_lds_long(DecArgs a) {
    __shared__ StagedLdsFor<S, kDecLong> sm;
    if constexpr (!kBatch) {
        // one codebook: if its codes all fit the peek table, the first launch
        // decodes every block (the check each block would make, made once)
        const huff_dcb* cb = a.one.cb;
        if (cb->max_len <= cb->lut_bits) return;
    }
    const uint64_t nblk = (a.nitems + 255) / 256;
    for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        dec_staged_block<S, kBatch, kDecLong>(a, blk, sm);
        __syncthreads();  // the block's tables and buffers are free for the next
    }
}

// Staged decode launches for one sub-block size.  Below 128 bytes the codes
// that fit the peek table and the longer ones are two launches.  For one
// stream, every block of the second launch exits at once unless the whole
// stream has long codes, so it runs a small grid that loops over the blocks
// (a full grid of workgroups that only exit costs ~16 us at 1 GiB); a batch
// mixes codebooks and keeps one workgroup per block in both.
constexpr uint32_t kDecSecondGrid = 1024;

template <int SZ>
hipError_t launch_staged(const DecArgs& a, hipStream_t s) {
    const uint64_t nblk = (a.nitems + 255) / 256;
    const dim3 grid((uint32_t)nblk), block(256);
    const dim3 grid2((uint32_t)(nblk < kDecSecondGrid ? nblk : kDecSecondGrid));
    if constexpr (SZ >= 128) {
        if (a.files) hipLaunchKernelGGL((k_decode_lds<SZ, true, kDecBoth>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_decode_lds<SZ, false, kDecBoth>), grid, block, 0, s, a);
    } else if (a.files) {
        // a batch mixes codebooks: both launches have work, one block each
        hipLaunchKernelGGL((k_decode_lds<SZ, true, kDecFits>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_decode_lds<SZ, true, kDecLong>), grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_decode_lds<SZ, false, kDecFits>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_decode_lds_long<SZ, false>), grid2, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_decode(const DecArgs& a, uint32_t block, bool out_aligned, hipStream_t s) {
    const uint32_t sub = 1u << a.item_log2;
    if (a.use_sub && out_aligned) {
        if (sub == 32) return launch_staged<32>(a, s);
        if (sub == 64) return launch_staged<64>(a, s);
        if (sub == 128) return launch_staged<128>(a, s);
        if (sub == 256) return launch_staged<256>(a, s);
    }
    const uint64_t blocks = (a.nitems + block - 1) / block;
    if (a.files) hipLaunchKernelGGL(k_decode<true>, dim3((uint32_t)blocks), dim3(block), 0, s, a);
    else hipLaunchKernelGGL(k_decode<false>, dim3((uint32_t)blocks), dim3(block), 0, s, a);
    return hipGetLastError();
}

// =================================================================== misc
// dst[i] = *src[i]: one value from each of n places (the server reads the
// stream lengths of a batch back with one copy).
__global__ __launch_bounds__(256) void k_gather_u64(const uint64_t* const* src, uint64_t* dst, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = *src[i];
}

hipError_t launch_gather_u64(const uint64_t* const* src, uint64_t* dst, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u64, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

// The bandwidth probe: workgroup b copies the contiguous vectors
// [b * kCopyChunk, (b + 1) * kCopyChunk) of 16 bytes, each thread issuing
// its kCopyInFlight non-temporal loads before it stores them (the probe's
// data is never reused).  Of the variants measured on MI355X (persistent
// grids of 512-65536 workgroups with 1-8 loads in flight, contiguous chunks
// of 16-128 KiB per workgroup), one 16 KiB chunk per workgroup moved the
// most.  The bytes past the last whole vector are copied by the first
// workgroup.
constexpr int kCopyInFlight = 4;
constexpr uint64_t kCopyChunk = 256 * kCopyInFlight;  // vectors per workgroup
typedef uint32_t v4u32_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, uint64_t bytes) {
    const uint64_t nvec = bytes >> 4;
    const v4u32_t* s = reinterpret_cast<const v4u32_t*>(src);
    v4u32_t* d = reinterpret_cast<v4u32_t*>(dst);
    const uint64_t b0 = (uint64_t)blockIdx.x * kCopyChunk + threadIdx.x;
    v4u32_t v[kCopyInFlight];
#pragma unroll
    for (int k = 0; k < kCopyInFlight; ++k) {
        const uint64_t i = b0 + 256 * k;
        v[k] = i < nvec ? __builtin_nontemporal_load(s + i) : v4u32_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < kCopyInFlight; ++k) {
        const uint64_t i = b0 + 256 * k;
        if (i < nvec) __builtin_nontemporal_store(v[k], d + i);
    }
    if (blockIdx.x == 0)
        for (uint64_t b = (nvec << 4) + threadIdx.x; b < bytes; b += blockDim.x) dst[b] = src[b];
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
    uint64_t g = ((bytes >> 4) + kCopyChunk - 1) / kCopyChunk;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)g), dim3(256), 0, s, (const uint8_t*)src, (uint8_t*)dst, bytes);
    return hipGetLastError();
}

// mode[b] = 1 when the codebook of decode block b's file has codes longer
// than its peek table (the staged decoder's second launch takes the block).
__global__ void k_blk_mode(const uint32_t* blk_file, const FileDesc* files, uint8_t* mode, uint64_t nblk) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const huff_dcb* cb = files[blk_file[b]].cb;
    mode[b] = cb->max_len > cb->lut_bits ? 1u : 0u;
}

hipError_t launch_blk_mode(const uint32_t* blk_file, const FileDesc* files, uint8_t* mode, uint64_t nblk,
                           hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blk_mode, dim3((uint32_t)((nblk + 255) / 256)), dim3(256), 0, s, blk_file, files, mode, nblk);
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s) {
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

// ========================================================= fixed workspace
// The workspaces of huff_compress_noalloc live in one file-scope device
// array, sized for HUFF_NOALLOC_MAX_N input bytes: the histogram accumulator
// and the per-tile histograms, bit counts, offsets and block carries.  Every
// call on a device shares that device's copy (calls that overlap on one
// device race).  Host code never uses the array's name as an address: its
// address on each device comes from hipGetSymbolAddress.
namespace {
constexpr uint64_t kAlignWs = 256;
constexpr uint64_t up_ws(uint64_t x) { return (x + kAlignWs - 1) / kAlignWs * kAlignWs; }
constexpr uint64_t kWsTiles = (HUFF_NOALLOC_MAX_N + kEncTile - 1) / kEncTile;
constexpr uint64_t kWsBlocks = kWsTiles / kScanTilesPerBlock + 1;
constexpr ScratchLayout kLayout = {
    0,
    up_ws(sizeof(HistState)),
    up_ws(sizeof(HistState)) + up_ws(kWsTiles * 512),
    up_ws(sizeof(HistState)) + up_ws(kWsTiles * 512) + up_ws(kWsTiles * 4),
    up_ws(sizeof(HistState)) + up_ws(kWsTiles * 512) + 2 * up_ws(kWsTiles * 4),
    up_ws(sizeof(HistState)) + up_ws(kWsTiles * 512) + 2 * up_ws(kWsTiles * 4) + up_ws(kWsBlocks * 8),
    up_ws(sizeof(HistState)) + up_ws(kWsTiles * 512) + 2 * up_ws(kWsTiles * 4) + 2 * up_ws(kWsBlocks * 8),
};
}  // namespace

static __device__ __align__(256) uint8_t scratch[kLayout.bytes];

const ScratchLayout& scratch_layout() { return kLayout; }

hipError_t scratch_address(int device, void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices];
    static bool found[kMaxDevices];
    if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(mu);
    if (!found[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[device] = p;
        found[device] = true;
    }
    *out = ptr[device];
    return hipSuccess;
}

// Result checks of the request server: every workgroup takes a share of
// every job's bytes (16 bytes per lane at a time when both sides are
// 16-byte aligned, single bytes otherwise).
// Every job has its own run of workgroups (first_block, nblocks: about
// kCmpBytesPerBlock bytes each), so all jobs of a batch are compared at once.
constexpr uint64_t kCmpBytesPerBlock = 64 << 10;

uint32_t compare_blocks(uint64_t bytes) {
    const uint64_t b = (bytes + kCmpBytesPerBlock - 1) / kCmpBytesPerBlock;
    return (uint32_t)(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(256) void k_compare(const CmpJob* jobs, uint32_t njobs) {
    // this workgroup's job: the last whose first block is at most blockIdx.x
    uint32_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first_block <= blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const CmpJob c = jobs[lo];
    const uint64_t stride = (uint64_t)c.nblocks * blockDim.x;
    const uint64_t me = (uint64_t)(blockIdx.x - c.first_block) * blockDim.x + threadIdx.x;
    bool diff = false;
    if (me == 0 && c.got_bits && *c.got_bits != c.want_bits) diff = true;
    const bool vec = (((uintptr_t)c.got | (uintptr_t)c.want) & 15u) == 0;
    const uint64_t nv = vec ? c.bytes >> 4 : 0;
    const uint4* g4 = reinterpret_cast<const uint4*>(c.got);
    const uint4* w4 = reinterpret_cast<const uint4*>(c.want);
    for (uint64_t i = me; i < nv; i += stride) {
        const uint4 a = g4[i], b = w4[i];
        diff |= a.x != b.x || a.y != b.y || a.z != b.z || a.w != b.w;
    }
    for (uint64_t i = (nv << 4) + me; i < c.bytes; i += stride) diff |= c.got[i] != c.want[i];
    if (diff) atomicMin(c.status, (int32_t)HUFF_E_MISMATCH);
}

hipError_t launch_compare(const CmpJob* jobs, uint32_t njobs, uint32_t total_blocks, hipStream_t s) {
    if (njobs == 0 || total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compare, dim3(total_blocks), dim3(256), 0, s, jobs, njobs);
    return hipGetLastError();
}

}  // namespace huff

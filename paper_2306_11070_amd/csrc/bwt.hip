// HIP kernels of the block transform that Method 3 of the paper applies
// before the Huffman code (Section III.A), for gfx950 (wave64).
//
//   k_bwt    one workgroup per block: the block's cyclic rotations sorted by
//            prefix doubling (position-tagged rank keys sorted in LDS), the
//            last column out, and the row of every rotation that starts at a
//            multiple of `every` (the inverse starts its walks there).
//   k_mtf    one wave per block: move-to-front positions, the list's first
//            64 entries one per lane, the rest in LDS.
//   k_unmtf  one wave per block: the inverse.
//   k_unbwt  one workgroup per block: the last-to-first map from a stable
//            count of the last column (wave ballots), then one walker per
//            `every` bytes, each starting from its recorded row.
// All of this is integer work bound by LDS and the ALUs, not by HBM.
#include "common.h"

namespace huff {

namespace {

constexpr int kBwtThreads = 1024;
constexpr uint32_t kPosBits = 14;  // positions and ranks in a block of at most 2^14 bytes
constexpr uint64_t kPosMask = (1u << kPosBits) - 1;
constexpr uint32_t kKeyBytes = 6;  // the first sort's key: 6 bytes and the position (62 bits)
static_assert(8 * kKeyBytes + kPosBits < 64, "first keys stay below the padding key");
constexpr uint32_t kMaxPer = HUFF_BWT_MAX_BLOCK / kBwtThreads;  // sort slots per thread
static_assert(HUFF_BWT_MAX_BLOCK == 1u << kPosBits, "block positions fit kPosBits");

// LDS slot of sort entry i: one spare slot after every 16, so that the 64
// lanes of a wave reading runs of up to 16 consecutive 8-byte entries (one
// run per lane) spread over the LDS banks instead of meeting in a few.
__device__ __forceinline__ uint32_t kslot(uint32_t i) { return i + (i >> 4); }
constexpr uint32_t kKeySlots = HUFF_BWT_MAX_BLOCK + HUFF_BWT_MAX_BLOCK / 16;

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Stages j = jtop, jtop/2, ..., 1 (all below E) of bitonic merge k on the
// run r[0..E) of sort entries q0 .. q0+E-1 held in registers.
template <uint32_t E, typename K>
__device__ __forceinline__ void reg_merge(K (&r)[E], uint32_t q0, uint32_t k, uint32_t jtop) {
#pragma unroll
    for (uint32_t j = E / 2; j >= 1; j >>= 1) {
        if (j <= jtop) {
#pragma unroll
            for (uint32_t e = 0; e < E; ++e) {
                if ((e & j) == 0) {
                    const bool up = ((q0 + e) & k) == 0;
                    const K x = r[e], y = r[e | j];
                    const K lo = x < y ? x : y, hi = x < y ? y : x;
                    r[e] = up ? lo : hi;
                    r[e | j] = up ? hi : lo;
                }
            }
        }
    }
}

// Ascending bitonic sort of key[0..np) in LDS (entry i at kslot(i)) by the
// whole workgroup of kBwtThreads threads, np = E * kBwtThreads.  Thread t
// owns entries [t*E, t*E + E).  The merges of runs up to E long happen in
// registers, in one pass.  In every later merge, the stages whose pairs lie
// E or more entries apart exchange through LDS -- every thread issues the
// loads of all its E/2 pairs before it compares and stores them, so a stage
// costs one LDS round trip -- and the stages with pairs closer than E that
// close the merge run in registers with no barrier between them.
template <uint32_t E, typename K>
__device__ void lds_bitonic_sort_e(K* key) {
    constexpr uint32_t np = E * kBwtThreads;
    const uint32_t tid = threadIdx.x;
    const uint32_t q0 = tid * E;
    {
        K r[E];
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) r[e] = key[kslot(q0 + e)];
#pragma unroll
        for (uint32_t k = 2; k <= E; k <<= 1) reg_merge<E>(r, q0, k, k >> 1);
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) key[kslot(q0 + e)] = r[e];
    }
    lds_sync();
    for (uint32_t k = 2 * E; k <= np; k <<= 1) {
        for (uint32_t j = k >> 1; j >= E; j >>= 1) {
            K a[E / 2], b[E / 2];
            uint32_t ii[E / 2];
#pragma unroll
            for (uint32_t e = 0; e < E / 2; ++e) {
                const uint32_t p = tid + kBwtThreads * e;
                const uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                ii[e] = i;
                a[e] = key[kslot(i)];
                b[e] = key[kslot(i | j)];
            }
#pragma unroll
            for (uint32_t e = 0; e < E / 2; ++e) {
                const uint32_t i = ii[e];
                const bool up = (i & k) == 0;
                const K lo = a[e] < b[e] ? a[e] : b[e], hi = a[e] < b[e] ? b[e] : a[e];
                key[kslot(i)] = up ? lo : hi;
                key[kslot(i | j)] = up ? hi : lo;
            }
            lds_sync();
        }
        K r[E];
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) r[e] = key[kslot(q0 + e)];
        reg_merge<E>(r, q0, k, E >> 1);
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) key[kslot(q0 + e)] = r[e];
        lds_sync();
    }
}

// The sort for np = 2048, 4096, 8192 or 16384 entries.
template <typename K>
__device__ void lds_bitonic_sort_reg(K* key, uint32_t np) {
    switch (np / kBwtThreads) {
        case 2: lds_bitonic_sort_e<2>(key); break;
        case 4: lds_bitonic_sort_e<4>(key); break;
        case 8: lds_bitonic_sort_e<8>(key); break;
        default: lds_bitonic_sort_e<16>(key); break;
    }
}

// Exclusive prefix maximum of v over the threads of the workgroup, in thread
// order (0 for thread 0).
__device__ __forceinline__ uint32_t wg_excl_max(uint32_t v, uint32_t* s_red) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x = max(x, y);
    }
    if (lane == 63) s_red[wave] = x;
    lds_sync();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before = max(before, s_red[w]);
    lds_sync();
    const uint32_t incl = max(x, before);
    const uint32_t up = __shfl_up(incl, 1, 64);
    return lane ? up : before;
}

// Orders the LDS accesses of one wave: what its lanes wrote before is seen
// by all of its lanes after.
__device__ __forceinline__ void wave_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wg_sum(uint32_t v, uint32_t* s_red) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) s_red[wave] = v;
    lds_sync();
    uint32_t t = 0;
    for (uint32_t w = 0; w < blockDim.x / 64; ++w) t += s_red[w];
    lds_sync();
    return t;
}

}  // namespace

// ------------------------------------------------------------ forward
// One workgroup per block of m <= 16384 bytes, prefix doubling.  A key is
// (group value << 14) | position: first the rotation's first six bytes, then
// (rank, rank of the rotation h bytes further) -- so the sorted keys order the
// rotations by their first 6, 12, 24, ... bytes, with ties in start
// position.  After each sort every rotation's rank is the slot, in the order
// of all rotations, of the first rotation of its group; it is kept by start
// position (u16, in the upper part of the key array).  Rotations alone in
// their group are placed for good; the next round sorts only the others once
// they fit the lower part (at most kCompactMax), and each of their new ranks
// is the old rank plus the offset of its new group inside the old one.  The
// rounds stop when every group is alone, or when h >= m (rotations still tied
// are equal and take their start order).  Each thread owns a contiguous run
// of sort slots.
constexpr uint32_t kCompactMax = HUFF_BWT_MAX_BLOCK / 2;
constexpr uint32_t kRankSlot = kCompactMax + kCompactMax / 16;  // kslot(kCompactMax)
static_assert(kRankSlot + HUFF_BWT_MAX_BLOCK * 2 / 8 <= kKeySlots, "the rank array fits above the compact keys");

// Exclusive prefix sum of v over the threads of the workgroup, in thread order.
__device__ __forceinline__ uint32_t wg_excl_sum(uint32_t v, uint32_t* s_red) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) s_red[wave] = x;
    lds_sync();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before += s_red[w];
    lds_sync();
    return before + x - v;
}

__global__ __launch_bounds__(kBwtThreads) void k_bwt(const uint8_t* __restrict__ in, uint64_t n, uint32_t block,
                                                     uint32_t every_log2, uint8_t* __restrict__ last,
                                                     uint16_t* __restrict__ rows) {
    __shared__ unsigned long long s_key[kKeySlots];
    __shared__ uint8_t s_blk[HUFF_BWT_MAX_BLOCK];
    __shared__ uint32_t s_red[kBwtThreads / 64];
    uint16_t* s_rank = reinterpret_cast<uint16_t*>(s_key + kRankSlot);
    const uint32_t tid = threadIdx.x;
    const uint64_t lo = (uint64_t)blockIdx.x * block;
    const uint32_t m = (uint32_t)min<uint64_t>(block, n - lo);
    uint32_t np = 2 * kBwtThreads;
    while (np < m) np <<= 1;

    for (uint32_t i = tid; i < m; i += kBwtThreads) s_blk[i] = in[lo + i];
    lds_sync();
    {
        const uint32_t per = np / kBwtThreads, q0 = tid * per;
        for (uint32_t e = 0; e < per; ++e) {
            const uint32_t i = q0 + e;
            unsigned long long k = ~0ull;
            if (i < m) {
                unsigned long long c6 = 0;  // the rotation's first kKeyBytes bytes
                uint32_t j = i;
#pragma unroll
                for (uint32_t t = 0; t < kKeyBytes; ++t) {
                    c6 = (c6 << 8) | s_blk[j];
                    j = j + 1 == m ? 0 : j + 1;
                }
                k = (c6 << kPosBits) | i;
            }
            s_key[kslot(i)] = k;
        }
    }
    lds_sync();
    lds_bitonic_sort_reg(s_key, np);

    uint32_t cnt = m, npc = np;  // sorted entries, and the sorted array's size
    bool compact = false;        // the entries are the rotations still tied, keys (rank, rank h on, position)
    for (uint32_t h = kKeyBytes;; h <<= 1) {
        const uint32_t per = npc / kBwtThreads, c0 = tid * per;
        // group heads (same key but the position) and, in a compact round,
        // old-group heads (same rank), up to this thread's slots
        unsigned long long prev = c0 ? s_key[kslot(c0 - 1)] : 0ull;
        uint32_t lastSub = 0, lastGrp = 0;
        for (uint32_t e = 0; e < per; ++e) {
            const uint32_t c = c0 + e;
            const unsigned long long k = s_key[kslot(c)];
            if (c < cnt) {
                if (c == 0 || (k >> kPosBits) != (prev >> kPosBits)) lastSub = c;
                if (compact && (c == 0 || (k >> (2 * kPosBits)) != (prev >> (2 * kPosBits)))) lastGrp = c;
            }
            prev = k;
        }
        uint32_t sub = wg_excl_max(lastSub, s_red);
        uint32_t grp = compact ? wg_excl_max(lastGrp, s_red) : 0u;
        // new ranks (by start position) and the entries still tied
        const bool final_ties = h >= m;
        uint32_t pk[kMaxPer];  // position | new rank << 16
        uint32_t heads = 0;    // bit e: entry e starts a group; bit per: the entry after the last starts one
        prev = c0 ? s_key[kslot(c0 - 1)] : 0ull;
#pragma unroll
        for (uint32_t e = 0; e < kMaxPer; ++e) {
            pk[e] = 0;
            if (e < per) {
                const uint32_t c = c0 + e;
                const unsigned long long k = s_key[kslot(c)];
                if (c < cnt) {
                    const bool sh = c == 0 || (k >> kPosBits) != (prev >> kPosBits);
                    if (sh) sub = c;
                    if (compact && (c == 0 || (k >> (2 * kPosBits)) != (prev >> (2 * kPosBits)))) grp = c;
                    const uint32_t base = compact ? (uint32_t)(k >> (2 * kPosBits)) : 0u;
                    const uint32_t r = base + (final_ties ? c : sub) - grp;
                    pk[e] = (uint32_t)(k & kPosMask) | r << 16;
                    heads |= (sh ? 1u : 0u) << e;
                }
                prev = k;
            }
        }
        {
            // does the entry after this thread's last one start a group?
            const uint32_t c = c0 + per;
            const unsigned long long k = c < npc ? s_key[kslot(c)] : ~0ull;
            if (c >= cnt || (k >> kPosBits) != (prev >> kPosBits)) heads |= 1u << per;
        }
        uint32_t tied = 0, ntied = 0;  // bit e: entry e shares its group
#pragma unroll
        for (uint32_t e = 0; e < kMaxPer; ++e) {
            if (e < per && c0 + e < cnt && !(((heads >> e) & 1u) && ((heads >> (e + 1)) & 1u))) {
                tied |= 1u << e;
                ++ntied;
            }
        }
        const uint32_t U = wg_sum(ntied, s_red);  // also: every sorted key has been read
#pragma unroll
        for (uint32_t e = 0; e < kMaxPer; ++e)
            if (e < per && c0 + e < cnt) s_rank[pk[e] & 0xffffu] = (uint16_t)(pk[e] >> 16);
        lds_sync();
        if (U == 0 || final_ties) break;
        if (U <= kCompactMax) {
            // the tied rotations' next keys, packed into the lower part
            uint32_t c = wg_excl_sum(ntied, s_red);
#pragma unroll
            for (uint32_t e = 0; e < kMaxPer; ++e) {
                if ((tied >> e) & 1u) {
                    const uint32_t i = pk[e] & 0xffffu, r = pk[e] >> 16;
                    const uint32_t j = i + h < m ? i + h : i + h - m;  // h < m here
                    s_key[kslot(c)] = ((unsigned long long)r << (2 * kPosBits)) |
                                      ((unsigned long long)s_rank[j] << kPosBits) | i;
                    ++c;
                }
            }
            npc = 2 * kBwtThreads;
            while (npc < U) npc <<= 1;
            for (uint32_t q = U + tid; q < npc; q += kBwtThreads) s_key[kslot(q)] = ~0ull;
            cnt = U;
            compact = true;
        } else {
            // every rotation's next key, in position order (before any compact round)
            const uint32_t pf = np / kBwtThreads, q0 = tid * pf;
            unsigned long long nk[kMaxPer];
#pragma unroll
            for (uint32_t e = 0; e < kMaxPer; ++e) {
                const uint32_t i = q0 + e;
                nk[e] = ~0ull;
                if (e < pf && i < m) {
                    const uint32_t j = i + h < m ? i + h : i + h - m;
                    nk[e] = ((unsigned long long)s_rank[i] << (2 * kPosBits)) |
                            ((unsigned long long)s_rank[j] << kPosBits) | i;
                }
            }
            lds_sync();  // the ranks are read before the keys overwrite them
#pragma unroll
            for (uint32_t e = 0; e < kMaxPer; ++e)
                if (e < pf) s_key[kslot(q0 + e)] = nk[e];
            cnt = m;
            npc = np;
        }
        lds_sync();
        lds_bitonic_sort_reg(s_key, npc);
    }

    // s_rank[p]: the sorted row of the rotation starting at p.  The last
    // column is put together in LDS (below the ranks) and stored in order.
    uint8_t* s_out = reinterpret_cast<uint8_t*>(s_key);
    for (uint32_t p = tid; p < m; p += kBwtThreads) {
        const uint32_t r = s_rank[p];
        s_out[r] = s_blk[p ? p - 1 : m - 1];
        if ((p & ((1u << every_log2) - 1)) == 0) rows[(lo + p) >> every_log2] = (uint16_t)r;
    }
    lds_sync();
    for (uint32_t q = tid; q < m; q += kBwtThreads) last[lo + q] = s_out[q];
}

// ------------------------------------------------------- move to front
// One wave per block.  List positions 0..63 are held one per lane (lane l
// holds the byte at position l); positions 64..255 sit in a per-wave LDS
// array.  A lane reads 64 input bytes at a time; the wave then takes them in
// order, each as a uniform value.  Forward: a ballot of the lanes equal to
// the byte gives its position; the rare byte further back is found by three
// ballots over the LDS part.  Inverse: the position names the lane (or LDS
// entry) that holds the byte.  Then every entry before the position moves one
// place back (a DPP shift of the wave by one lane; with a position past 63,
// lane 63's entry and the LDS entries before the position move too) and the
// byte goes to the front.  After a block transform nearly every position is
// small, so a byte costs a few wave instructions.
template <bool kInverse>
__global__ __launch_bounds__(256) void k_mtf(const uint8_t* __restrict__ in, uint64_t n, uint32_t block,
                                             uint8_t* __restrict__ out) {
    __shared__ uint32_t s_tail[4][192];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t b = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint64_t lo = b * block;
    if (lo >= n) return;  // the whole wave
    const uint32_t m = (uint32_t)min<uint64_t>(block, n - lo);
    uint32_t* tail = s_tail[threadIdx.x >> 6];
    uint32_t w = lane;  // the list in value order
    for (uint32_t k = lane; k < 192; k += 64) tail[k] = 64 + k;
    wave_lds_barrier();
    for (uint32_t base = 0; base < m; base += 64) {
        const uint32_t cnt = min(64u, m - base);
        const uint32_t v = lane < cnt ? in[lo + base + lane] : 0u;
        uint32_t res = 0;
        for (uint32_t t = 0; t < cnt; ++t) {
            const uint32_t x = __builtin_amdgcn_readlane(v, t);
            uint32_t at, c;
            if constexpr (!kInverse) {
                c = x;
                const uint64_t hit = __ballot(w == c);
                if (hit) {
                    at = (uint32_t)__builtin_ctzll(hit);
                } else {
                    const uint64_t h0 = __ballot(tail[lane] == c), h1 = __ballot(tail[64 + lane] == c);
                    const uint64_t h2 = __ballot(tail[128 + lane] == c);
                    at = 64 + (h0 ? (uint32_t)__builtin_ctzll(h0)
                                  : h1 ? 64 + (uint32_t)__builtin_ctzll(h1) : 128 + (uint32_t)__builtin_ctzll(h2));
                }
            } else {
                at = x;
                c = at < 64 ? __builtin_amdgcn_readlane(w, at) : tail[at - 64];
            }
            if (at >= 64) {
                // LDS entries [0, at - 64] move one place back, lane 63's entry to the first of them
                const uint32_t p = at - 64, last = __builtin_amdgcn_readlane(w, 63);
                const uint32_t q0 = lane ? tail[lane - 1] : last, q1 = tail[63 + lane], q2 = tail[127 + lane];
                wave_lds_barrier();
                if (lane <= p) tail[lane] = q0;
                if (64 + lane <= p) tail[64 + lane] = q1;
                if (128 + lane <= p) tail[128 + lane] = q2;
                wave_lds_barrier();
            }
            // lanes up to the position (all of them past 63) take the previous
            // lane's entry by a DPP shift of the wave by one lane; lane 0 takes c
            const uint32_t sh = (uint32_t)__builtin_amdgcn_update_dpp((int)c, (int)w, 0x138 /* wave_shr:1 */, 0xf, 0xf,
                                                                      false);
            w = lane <= at ? sh : w;
            res = lane == t ? (kInverse ? c : at) : res;
        }
        if (lane < cnt) out[lo + base + lane] = (uint8_t)res;
    }
}

// ------------------------------------------------------------ inverse
// One workgroup per block.  The row that follows row r one position back in
// the block is lf[r] = (bytes of the last column smaller than L[r]) + (copies
// of L[r] before row r).  The second count is stable: each wave counts a
// contiguous part of the rows, the parts' counts are summed in wave order,
// and inside a part 64 rows at a time find the earlier equal bytes in their
// group from eight ballots (one per bit).  Then walker w rebuilds bytes
// [w*every, (w+1)*every) backwards from the recorded row of the rotation
// that starts right after them.
__global__ __launch_bounds__(kBwtThreads) void k_unbwt(const uint8_t* __restrict__ last, uint64_t n, uint32_t block,
                                                       uint32_t every_log2, const uint16_t* __restrict__ rows,
                                                       uint8_t* __restrict__ out, int32_t* status) {
    constexpr uint32_t kWaves = kBwtThreads / 64;
    __shared__ uint8_t s_L[HUFF_BWT_MAX_BLOCK];
    __shared__ uint16_t s_lf[HUFF_BWT_MAX_BLOCK];
    __shared__ uint8_t s_out[HUFF_BWT_MAX_BLOCK];
    __shared__ uint32_t s_cnt[kWaves][256];  // per wave: copies of each byte in its part, then its base
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lo = (uint64_t)blockIdx.x * block;
    const uint32_t m = (uint32_t)min<uint64_t>(block, n - lo);
    for (uint32_t i = tid; i < m; i += kBwtThreads) s_L[i] = last[lo + i];
    for (uint32_t i = tid; i < kWaves * 256; i += kBwtThreads) (&s_cnt[0][0])[i] = 0;
    lds_sync();
    // each wave's part: rows [p0, p1), whole groups of 64
    const uint32_t span = ((m + kWaves - 1) / kWaves + 63) & ~63u;
    const uint32_t p0 = min(m, wave * span), p1 = min(m, p0 + span);
    for (uint32_t r = p0 + lane; r < p1; r += 64) atomicAdd(&s_cnt[wave][s_L[r]], 1u);
    lds_sync();
    __shared__ uint32_t s_tot[256], s_wtot[4];
    if (tid < 256) {
        // byte value tid: its copies in the earlier parts, and its total
        uint32_t run = 0;
        for (uint32_t w = 0; w < kWaves; ++w) {
            const uint32_t c = s_cnt[w][tid];
            s_cnt[w][tid] = run;
            run += c;
        }
        s_tot[tid] = run;
    }
    lds_sync();
    uint32_t x = 0;
    if (tid < 256) {
        // the copies of all smaller byte values: exclusive scan of the totals
        x = s_tot[tid];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= (uint32_t)d) x += y;
        }
        if (lane == 63) s_wtot[wave] = x;
    }
    lds_sync();
    if (tid < 256) {
        uint32_t before = 0;
        for (uint32_t w = 0; w < wave; ++w) before += s_wtot[w];
        const uint32_t smaller = before + x - s_tot[tid];
        for (uint32_t w = 0; w < kWaves; ++w) s_cnt[w][tid] += smaller;
    }
    lds_sync();
    // stable ranks inside the part, 64 rows at a time
    for (uint32_t r0 = p0; r0 < p1; r0 += 64) {
        const uint32_t r = r0 + lane;
        const bool on = r < p1;
        const uint32_t c = on ? s_L[r] : 0u;
        uint64_t eq = __ballot(on);
        for (uint32_t bit = 0; bit < 8; ++bit) {
            const uint64_t ones = __ballot(on && ((c >> bit) & 1));
            eq &= ((c >> bit) & 1) ? ones : ~ones;
        }
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        const uint32_t rank = (uint32_t)__popcll(eq & below);
        if (on) s_lf[r] = (uint16_t)(s_cnt[wave][c] + rank);
        wave_lds_barrier();
        // the last copy of each byte value in the group moves its base on
        if (on && (eq >> lane) == 1ull) s_cnt[wave][c] += (uint32_t)__popcll(eq);
        wave_lds_barrier();
    }
    lds_sync();
    // walkers
    const uint32_t S = 1u << every_log2;
    const uint32_t nwalk = (m + S - 1) >> every_log2;
    for (uint32_t wk = tid; wk < nwalk; wk += kBwtThreads) {
        const uint32_t beg = wk << every_log2, end = min(m, beg + S);
        uint32_t r = rows[(lo + (end == m ? 0 : end)) >> every_log2];
        if (r >= m) {
            atomicMin(status, (int32_t)HUFF_E_CORRUPT);
            continue;
        }
        for (uint32_t p = end; p-- > beg;) {
            s_out[p] = s_L[r];
            r = s_lf[r];
        }
    }
    lds_sync();
    for (uint32_t i = tid; i < m; i += kBwtThreads) out[lo + i] = s_out[i];
}

hipError_t launch_bwt(const uint8_t* in, uint64_t n, uint32_t block, uint32_t every_log2, uint8_t* last,
                      uint16_t* rows, hipStream_t s) {
    const uint64_t nblk = (n + block - 1) / block;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwt, dim3((uint32_t)nblk), dim3(kBwtThreads), 0, s, in, n, block, every_log2, last, rows);
    return hipGetLastError();
}

hipError_t launch_unbwt(const uint8_t* last, uint64_t n, uint32_t block, uint32_t every_log2, const uint16_t* rows,
                        uint8_t* out, int32_t* status, hipStream_t s) {
    const uint64_t nblk = (n + block - 1) / block;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unbwt, dim3((uint32_t)nblk), dim3(kBwtThreads), 0, s, last, n, block, every_log2, rows, out,
                       status);
    return hipGetLastError();
}

hipError_t launch_mtf(const uint8_t* in, uint64_t n, uint32_t block, uint8_t* out, bool inverse, hipStream_t s) {
    const uint64_t nblk = (n + block - 1) / block;
    if (nblk == 0) return hipSuccess;
    const dim3 grid((uint32_t)((nblk + 3) / 4)), wg(256);
    if (inverse) hipLaunchKernelGGL(k_mtf<true>, grid, wg, 0, s, in, n, block, out);
    else hipLaunchKernelGGL(k_mtf<false>, grid, wg, 0, s, in, n, block, out);
    return hipGetLastError();
}

}  // namespace huff

// HIP kernels of the Huffman codec for gfx950 (CDNA4, wave64).
//
//   k_hist      byte histogram: LDS-privatised replicated counters, one
//               global atomic per bin per workgroup, self-resetting
//               accumulator finalised by the last workgroup.
//   k_codebook  tie-ruled Huffman code lengths, canonical codes and decode
//               tables for one file per workgroup.
//   k_encode    single-pass chunked encode: code lengths per 16-byte unit,
//               workgroup scan, decoupled look-back across tiles for the
//               tile's first stream bit, LDS-staged bit packing, coalesced
//               word stores, segment index and decode index.
//   k_decode    one lane per indexed sub-block (or chunk): table-driven
//               canonical decode from a 64-bit bit window.
//   k_copy      plain 16-byte copy, the bandwidth probe.
#include "common.h"

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

// ============================================================== histogram
__global__ __launch_bounds__(kHistThreads) void k_hist(HistArgs a) {
    __shared__ uint32_t sh[256 * kHistMaxDepth];
    __shared__ int s_last;
    const uint32_t dl = a.depth_log2, depth = 1u << dl;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < 256u * depth; i += blockDim.x) sh[i] = 0;
    __syncthreads();
    const uint32_t rep = tid & (depth - 1);
    const uint8_t* in = a.in;
    const uint64_t n = a.n;
    const uint64_t head = min<uint64_t>(n, (16u - ((uintptr_t)in & 15u)) & 15u);
    const uint64_t nvec = (n - head) >> 4;
    const uint4* vec = reinterpret_cast<const uint4*>(in + head);
    const uint64_t per = a.per_block >> 4;
    const uint64_t vlo = (uint64_t)blockIdx.x * per;
    const uint64_t vhi = min(nvec, vlo + per);
    auto count = [&](uint32_t b) { atomicAdd(&sh[(b << dl) | rep], 1u); };
    auto count4 = [&](uint32_t w) {
        count(w & 0xffu);
        count((w >> 8) & 0xffu);
        count((w >> 16) & 0xffu);
        count(w >> 24);
    };
    uint64_t i = vlo + tid;
    const uint32_t stride = blockDim.x;
    for (; i + 3 * stride < vhi; i += 4 * stride) {
        uint4 q0 = vec[i], q1 = vec[i + stride], q2 = vec[i + 2 * stride], q3 = vec[i + 3 * stride];
        count4(q0.x); count4(q0.y); count4(q0.z); count4(q0.w);
        count4(q1.x); count4(q1.y); count4(q1.z); count4(q1.w);
        count4(q2.x); count4(q2.y); count4(q2.z); count4(q2.w);
        count4(q3.x); count4(q3.y); count4(q3.z); count4(q3.w);
    }
    for (; i < vhi; i += stride) {
        uint4 q = vec[i];
        count4(q.x); count4(q.y); count4(q.z); count4(q.w);
    }
    if (blockIdx.x == 0) {
        for (uint64_t k = tid; k < head; k += stride) count(in[k]);
        for (uint64_t k = head + (nvec << 4) + tid; k < n; k += stride) count(in[k]);
    }
    __syncthreads();
    for (uint32_t v = tid; v < 256; v += stride) {
        uint32_t s = 0;
        for (uint32_t r = 0; r < depth; ++r) s += sh[(v << dl) | ((r + v) & (depth - 1))];
        if (s) atomicAdd(&a.st->acc[v], (unsigned long long)s);
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&a.st->done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        __threadfence();
        for (uint32_t v = tid; v < 256; v += stride) a.out[v] = atomicExch(&a.st->acc[v], 0ull);
        if (tid == 0) atomicExch(&a.st->done, 0u);
    }
}

hipError_t launch_histogram(const HistArgs& a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_hist, dim3(blocks), dim3(kHistThreads), 0, s, a);
    return hipGetLastError();
}

// =============================================================== codebook
// One workgroup of 256 threads; thread v owns byte value v.
__global__ __launch_bounds__(kCbThreads) void k_codebook(CbArgs a) {
    __shared__ unsigned long long s_h[256];
    __shared__ unsigned long long s_w[512];  // node weights: sorted leaves, then internal nodes
    __shared__ uint16_t s_par[512];
    __shared__ uint16_t s_d[512], s_p[512];
    __shared__ uint8_t s_len[256];
    __shared__ uint8_t s_sorted[256];
    __shared__ uint32_t s_cnt[64], s_fidx[64];
    __shared__ unsigned long long s_first[64];
    __shared__ unsigned long long s_tot, s_n;
    __shared__ uint32_t s_max;
    const uint32_t v = threadIdx.x;
    uint64_t h = 0;
    uint32_t myLen = 0;
    if (v == 0) { s_tot = 0; s_n = 0; s_max = 0; }
    if (v < 64) s_cnt[v] = 0;
    s_sorted[v] = 0;
    if (!a.from_lengths) {
        h = a.hist[v];
        s_h[v] = h;
        __syncthreads();
        const int K = __syncthreads_count(h != 0);
        uint32_t rank = 0;
        if (h) {
            for (uint32_t u = 0; u < 256; ++u) {
                const uint64_t hu = s_h[u];
                rank += (hu != 0) & ((hu < h) | ((hu == h) & (u < v)));
            }
            s_w[rank] = h;
        }
        __syncthreads();
        if (K == 1) {
            myLen = h ? 1u : 0u;
        } else if (K >= 2) {
            if (v == 0) {
                // Two queues: leaves s_w[0..K) ascending, internal nodes
                // s_w[K..K+made) in creation order (never decreasing).  On
                // equal weight the leaf (smaller id) is taken first.
                uint32_t li = 0, qi = 0;
                for (uint32_t m = 0; m < (uint32_t)K - 1; ++m) {
                    uint32_t id[2];
                    uint64_t w[2];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const bool leaf = li < (uint32_t)K && (qi >= m || s_w[li] <= s_w[K + qi]);
                        id[t] = leaf ? li : K + qi;
                        w[t] = s_w[id[t]];
                        li += leaf;
                        qi += !leaf;
                    }
                    s_w[K + m] = w[0] + w[1];
                    s_par[id[0]] = (uint16_t)(K + m);
                    s_par[id[1]] = (uint16_t)(K + m);
                }
            }
            __syncthreads();
            // depths by pointer jumping: d = distance to p, p -> p's ancestor
            const uint32_t nodes = 2 * K - 1, root = nodes - 1;
            for (uint32_t i = v; i < nodes; i += 256) {
                s_d[i] = i == root ? 0 : 1;
                s_p[i] = i == root ? root : s_par[i];
            }
            __syncthreads();
            for (int it = 0; it < 8; ++it) {
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
            if (h) myLen = s_d[rank];
        }
        atomicAdd(&s_tot, (unsigned long long)(h * myLen));
        atomicAdd(&s_n, (unsigned long long)h);
    } else {
        myLen = a.len[v];
    }
    s_len[v] = (uint8_t)myLen;
    __syncthreads();
    int32_t status = HUFF_OK;
    if (myLen) {
        atomicMax(&s_max, myLen);
        if (myLen < 64) atomicAdd(&s_cnt[myLen], 1u);
    }
    __syncthreads();
    const uint32_t maxLen = s_max;
    if (maxLen > HUFF_MAX_CODE_LEN) status = HUFF_E_CODELEN;
    if (v < 64) {
        // first canonical code of length v: sum over j < v of count[j] * 2^(v-j)
        uint32_t fidx = 0;
        uint64_t fc = 0;
        for (uint32_t j = 1; j < v; ++j) {
            fidx += s_cnt[j];
            fc += (uint64_t)s_cnt[j] << (v - j);
        }
        s_fidx[v] = fidx;
        s_first[v] = fc;
    }
    __syncthreads();
    uint64_t code = 0;
    if (myLen && myLen < 64) {
        uint32_t r = 0;
        for (uint32_t u = 0; u < v; ++u) r += s_len[u] == myLen;
        code = s_first[myLen] + r;
        s_sorted[s_fidx[myLen] + r] = (uint8_t)v;
    }
    __syncthreads();
    huff_dcb* d = a.out;
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
    for (uint32_t p = v; p < (1u << HUFF_LUT_BITS); p += 256) {
        uint16_t e = 0;
        if (p < (1u << lutBits)) {
            for (uint32_t l = 1; l <= lutBits; ++l) {
                const uint64_t c = p >> (lutBits - l);
                if (c - s_first[l] < s_cnt[l]) {
                    e = (uint16_t)(s_sorted[s_fidx[l] + (uint32_t)(c - s_first[l])] | (l << 8));
                    break;
                }
            }
        }
        d->lut[p] = e;
    }
    if (v == 0) {
        uint32_t k = 0;
        for (uint32_t l = 1; l < 64; ++l) k += s_cnt[l];
        d->nsym = k;
        d->max_len = maxLen;
        d->lut_bits = lutBits;
        d->status = status;
        d->total_bits = a.from_lengths ? 0 : s_tot;
        d->n = a.from_lengths ? 0 : s_n;
        if (status != HUFF_OK) atomicMin(a.err, status);
    }
}

hipError_t launch_codebook(const CbArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), 0, s, a);
    return hipGetLastError();
}

// ================================================================= encode
constexpr int kBufWords = 3200;  // >= one 4 KiB round at 24 bits/byte, one wave's units at 63 bits/byte

__device__ __forceinline__ uint4 load_unit(const uint8_t* in, uint64_t q, uint64_t n, bool aligned) {
    if (aligned && q + 16 <= n) return *reinterpret_cast<const uint4*>(in + q);
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (q + i < n) w[i >> 2] |= (uint32_t)in[q + i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Append `len` (<= 32) bits of `c`; full 32-bit words go to the LDS buffer.
struct Packer {
    uint64_t acc;
    uint32_t na;  // valid low bits in acc (< 32 between appends)
    uint32_t wi;  // LDS word that receives the next full word
    __device__ __forceinline__ void put(uint64_t c, uint32_t len, uint32_t* buf) {
        acc = (acc << len) | c;
        na += len;
        if (na >= 32) {
            na -= 32;
            atomicOr(&buf[wi++], (uint32_t)(acc >> na));
        }
    }
    __device__ __forceinline__ void finish(uint32_t* buf) {
        if (na) atomicOr(&buf[wi], (uint32_t)(acc << (32 - na)));
    }
};

template <int R, bool kBatch>
__global__ __launch_bounds__(kEncThreads) void k_encode(EncArgs a) {
    __shared__ uint32_t s_enc[256];
    __shared__ unsigned long long s_code[256];
    __shared__ uint8_t s_len[256];
    __shared__ uint8_t s_prev[32];
    __shared__ uint32_t s_buf[kBufWords];
    __shared__ uint32_t s_wsum[4][R];
    __shared__ unsigned long long s_excl;
    __shared__ uint32_t s_ticket, s_carry, s_maxlen;
    __shared__ int s_last, s_wrap;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t epoch = __hip_atomic_load(&a.st->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t tagE = (uint64_t)epoch << 44;
    const huff_dcb* loaded = nullptr;
    constexpr uint64_t kTile = (uint64_t)R * kRoundBytes;

    for (uint32_t i = tid; i < kBufWords; i += kEncThreads) s_buf[i] = 0;

    for (;;) {
        if (tid == 0) s_ticket = atomicAdd(&a.st->ticket, 1u);
        __syncthreads();
        const uint64_t g = s_ticket;
        if (g >= a.ntiles) break;
        FileDesc f;
        if constexpr (kBatch) f = a.files[find_file(a.files, a.nfiles, g)];
        else f = a.one;
        const uint64_t j = g - f.first;
        const uint64_t tstart = j * kTile;
        const uint64_t n = f.n;
        const bool lastTile = tstart + kTile >= n;
        const bool aligned = ((uintptr_t)f.in & 15u) == 0;
        int32_t* err = f.status ? f.status : a.err;

        // issue the tile's loads before the (possibly) serialising table load
        uint4 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = load_unit(f.in, tstart + (uint64_t)(r * kEncThreads + tid) * 16, n, aligned);
        if (tid < 32 && j > 0) s_prev[tid] = f.in[tstart - 32 + tid];

        if (f.cb != loaded) {
            s_enc[tid] = f.cb->enc[tid];
            s_code[tid] = f.cb->code[tid];
            s_len[tid] = f.cb->len[tid];
            if (tid == 0) s_maxlen = f.cb->max_len;
            loaded = f.cb;
        }
        __syncthreads();
        const uint32_t maxLen = s_maxlen;
        const bool generic = maxLen > 24;

        // 1) code bits per 16-byte unit
        uint32_t usum[R];
        bool missing = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t q = tstart + (uint64_t)(r * kEncThreads + tid) * 16;
            const uint32_t nv = q >= n ? 0u : (uint32_t)min<uint64_t>(16, n - q);
            uint32_t s = 0;
            if (nv == 16) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint32_t l = s_len[byte_of(x[r], i)];
                    s += l;
                    missing |= l == 0;
                }
            } else {
                for (uint32_t i = 0; i < nv; ++i) {
                    const uint32_t l = s_len[byte_of(x[r], i)];
                    s += l;
                    missing |= l == 0;
                }
            }
            usum[r] = s;
        }
        if (missing) report(f.status, a.err, HUFF_E_INVAL);

        // 2) workgroup scan of unit totals in unit order (round-major)
        uint32_t incl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) incl[r] = wave_incl_scan(usum[r]);
        if (lane == 63) {
#pragma unroll
            for (int r = 0; r < R; ++r) s_wsum[wave][r] = incl[r];
        }
        __syncthreads();
        uint32_t uexcl[R], rstart[R + 1];
        uint32_t base = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t before = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t ws = s_wsum[w][r];
                tot += ws;
                before += w < wave ? ws : 0u;
            }
            rstart[r] = base;
            uexcl[r] = base + before + incl[r] - usum[r];
            base += tot;
        }
        rstart[R] = base;
        const uint32_t agg = base;

        // 3) decoupled look-back for the tile's first stream bit
        if (j == 0) {
            if (tid == 0) {
                __hip_atomic_store(&a.lb[g], kFlagPre | tagE | (uint64_t)agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_excl = 0;
            }
        } else if (wave == 0) {
            if (lane == 0)
                __hip_atomic_store(&a.lb[g], kFlagAgg | tagE | (uint64_t)agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t excl = 0;
            int64_t pos = (int64_t)j - 1;
            for (;;) {
                const int64_t idx = pos - lane;
                uint64_t st = 0;
                bool valid = true, pre = true;
                if (idx >= 0) {
                    st = __hip_atomic_load(&a.lb[g - j + (uint64_t)idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t fl = (uint32_t)(st >> 62);
                    valid = fl != 0 && (uint32_t)((st >> 44) & kEpochMax) == epoch;
                    pre = valid && fl == 2;
                }
                const uint64_t bp = __ballot(pre);
                const uint64_t bi = __ballot(!valid);
                const int first = bp ? __ffsll((unsigned long long)bp) - 1 : 64;
                const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1);
                if (bi & upto) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += wave_sum_u64((lane <= first && idx >= 0) ? (st & kValueMask) : 0ull);
                if (first < 64) break;
                pos -= 64;
            }
            if (lane == 0) {
                __hip_atomic_store(&a.lb[g], kFlagPre | tagE | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_excl = excl;
            }
        }
        __syncthreads();
        const uint64_t S = s_excl;
        if (tid == 0) {
            // bits of the shared first word that belong to earlier bytes,
            // recomputed from the 32 bytes before the tile
            const uint32_t rb = (uint32_t)(S & 31);
            uint32_t carry = 0;
            if (rb) {
                uint64_t acc = 0;
                uint32_t nb = 0;
                int k = 31;
                while (nb < rb && k >= 0) {
                    const uint32_t b = s_prev[k--];
                    acc |= (uint64_t)s_code[b] << nb;
                    nb += s_len[b];
                }
                carry = (uint32_t)(acc & ((1u << rb) - 1)) << (32 - rb);
            }
            s_carry = carry;
        }
        // 4) segment index and decode index
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t q = tstart + (uint64_t)(r * kEncThreads + tid) * 16;
            if (q < n) {
                const uint64_t bp = S + uexcl[r];
                if ((q & ((1ull << a.chunk_log2) - 1)) == 0) f.chunk_off[q >> a.chunk_log2] = bp;
                if (a.sub_log2 != kNoSub && (q & ((1ull << a.sub_log2) - 1)) == 0) f.sub_lo[q >> a.sub_log2] = (uint32_t)bp;
            }
        }
        if (lastTile && tid == 0) {
            const uint64_t T = S + agg;
            f.chunk_off[(n + (1ull << a.chunk_log2) - 1) >> a.chunk_log2] = T;
            if (a.sub_log2 != kNoSub) f.sub_lo[(n + (1ull << a.sub_log2) - 1) >> a.sub_log2] = (uint32_t)T;
            if (((T + 31) >> 5) > f.nwords) report(f.status, a.err, HUFF_E_CAPACITY);
        }
        __syncthreads();

        // 5) pack into LDS and stream out complete words
        uint32_t carry = s_carry;
        const int wavesPerPass = generic ? 1 : 4;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            for (int wp = 0; wp < 4; wp += wavesPerPass) {
                uint32_t pre = 0, mid = 0;
                for (int w = 0; w < 4; ++w) {
                    const uint32_t ws = s_wsum[w][r];
                    pre += w < wp ? ws : 0u;
                    mid += (w >= wp && w < wp + wavesPerPass) ? ws : 0u;
                }
                const uint64_t A = S + rstart[r] + pre, B = A + mid;
                const uint64_t w0 = A >> 5;
                if (tid == 0 && carry) atomicOr(&s_buf[0], carry);
                if (wave >= wp && wave < wp + wavesPerPass) {
                    const uint64_t q = tstart + (uint64_t)(r * kEncThreads + tid) * 16;
                    const uint32_t nv = q >= n ? 0u : (uint32_t)min<uint64_t>(16, n - q);
                    const uint32_t lbit = (uint32_t)(S + uexcl[r] - (w0 << 5));
                    Packer pk{0, lbit & 31, lbit >> 5};
                    if (!generic && nv == 16) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            const uint32_t e = s_enc[byte_of(x[r], i)];
                            pk.put(e >> 8, e & 0xffu, s_buf);
                        }
                    } else if (!generic) {
                        for (uint32_t i = 0; i < nv; ++i) {
                            const uint32_t e = s_enc[byte_of(x[r], i)];
                            pk.put(e >> 8, e & 0xffu, s_buf);
                        }
                    } else {
                        for (uint32_t i = 0; i < nv; ++i) {
                            const uint32_t b = byte_of(x[r], i);
                            const uint32_t l = s_len[b];
                            const uint64_t c = s_code[b];
                            if (l > 32) {
                                pk.put(c >> 32, l - 32, s_buf);
                                pk.put(c & 0xffffffffull, 32, s_buf);
                            } else {
                                pk.put(c, l, s_buf);
                            }
                        }
                    }
                    pk.finish(s_buf);
                }
                __syncthreads();
                const uint32_t nfull = (uint32_t)((B >> 5) - w0);
                for (uint32_t k = tid; k < nfull; k += kEncThreads)
                    if (w0 + k < f.nwords) f.words[w0 + k] = s_buf[k];
                carry = (B & 31) ? s_buf[nfull] : 0u;
                __syncthreads();
                for (uint32_t k = tid; k <= nfull; k += kEncThreads) s_buf[k] = 0;
                __syncthreads();
            }
        }
        if (lastTile && tid == 0) {
            const uint64_t T = S + agg;
            if ((T & 31) && (T >> 5) < f.nwords) f.words[T >> 5] = carry;
        }
    }

    // the last workgroup out resets the ticket and done counters and
    // advances the epoch (clearing the look-back words when it wraps)
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        s_last = atomicAdd(&a.st->done, 1u) == gridDim.x - 1;
        s_wrap = 0;
        if (s_last) {
            uint32_t e = epoch + 1;
            if (e > kEpochMax) { e = 1; s_wrap = 1; }
            atomicExch(&a.st->ticket, 0u);
            atomicExch(&a.st->done, 0u);
            atomicExch(&a.st->epoch, e);
        }
    }
    __syncthreads();
    if (s_last && s_wrap)
        for (uint64_t i = tid; i < a.lb_cap; i += kEncThreads) a.lb[i] = 0;
}

template <int R>
static hipError_t launch_encode_r(const EncArgs& a, uint32_t grid, hipStream_t s) {
    if (a.files) hipLaunchKernelGGL((k_encode<R, true>), dim3(grid), dim3(kEncThreads), 0, s, a);
    else hipLaunchKernelGGL((k_encode<R, false>), dim3(grid), dim3(kEncThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_encode(const EncArgs& a, uint32_t grid, hipStream_t s) {
    switch (a.rounds) {
        case 1: return launch_encode_r<1>(a, grid, s);
        case 2: return launch_encode_r<2>(a, grid, s);
        case 4: return launch_encode_r<4>(a, grid, s);
        case 8: return launch_encode_r<8>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
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

template <bool kBatch>
__global__ __launch_bounds__(256) void k_decode(DecArgs a) {
    __shared__ uint16_t s_lut[1 << HUFF_LUT_BITS];
    __shared__ unsigned long long s_first[64];
    __shared__ uint32_t s_cnt[64], s_fidx[64];
    __shared__ uint8_t s_sorted[256];

    const uint64_t item = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    FileDesc f;
    if constexpr (kBatch) f = a.files[find_file(a.files, a.nfiles, (uint64_t)blockIdx.x * blockDim.x)];
    else f = a.one;
    const huff_dcb* cb = f.cb;
    const uint32_t lutBits = cb->lut_bits, maxLen = cb->max_len;
    for (uint32_t i = threadIdx.x; i < (1u << lutBits); i += blockDim.x) s_lut[i] = cb->lut[i];
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) {
        s_first[i] = cb->first_code[i];
        s_cnt[i] = cb->count[i];
        s_fidx[i] = cb->first_index[i];
    }
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) s_sorted[i] = cb->sorted_sym[i];
    __syncthreads();

    const uint64_t j = item - f.first;
    const uint64_t n = f.n;
    const uint32_t il = a.item_log2, cl = a.chunk_log2;
    const uint64_t nitems = (n + (1ull << il) - 1) >> il;
    if (j >= nitems) return;
    const uint64_t nchunks = (n + (1ull << cl) - 1) >> cl;
    uint64_t start, end;
    if (a.use_sub) {
        const uint64_t c = (j << il) >> cl;
        const uint64_t base = f.chunk_off[c];
        start = base + (uint32_t)(f.sub_lo[j] - (uint32_t)base);
        if (j + 1 == nitems) {
            end = f.chunk_off[nchunks];
        } else {
            const uint64_t c2 = ((j + 1) << il) >> cl;
            const uint64_t b2 = f.chunk_off[c2];
            end = b2 + (uint32_t)(f.sub_lo[j + 1] - (uint32_t)b2);
        }
    } else {
        start = f.chunk_off[j];
        end = f.chunk_off[j + 1];
    }
    const uint64_t first = j << il;
    const uint64_t nsym = min<uint64_t>(1ull << il, n - first);
    uint8_t* out = f.out + first;
    bool bad = start > end || end > f.nwords * 32ull || maxLen == 0 || maxLen > HUFF_MAX_CODE_LEN;
    uint64_t used = 0;

    if (!bad && maxLen <= 32) {
        BitReader br;
        br.init(f.words, f.nwords, start);
        const uint32_t lutShift = 32 - lutBits;
        auto one = [&]() -> uint32_t {
            br.refill();
            const uint32_t top = (uint32_t)(br.win >> 32);
            const uint32_t e = s_lut[top >> lutShift];
            uint32_t len = e >> 8, sym = e & 0xffu;
            if (len == 0) {
                for (uint32_t l = lutBits + 1; l <= maxLen; ++l) {
                    const uint64_t c = top >> (32 - l);
                    if (c - s_first[l] < s_cnt[l]) {
                        sym = s_sorted[s_fidx[l] + (uint32_t)(c - s_first[l])];
                        len = l;
                        break;
                    }
                }
                if (len == 0) { bad = true; len = 1; }
            }
            br.win <<= len;
            br.avail -= len;
            used += len;
            return sym;
        };
        const uint64_t groups = nsym >> 4;
        const bool vec_ok = (((uintptr_t)out) & 15u) == 0;
        for (uint64_t gi = 0; gi < groups; ++gi) {
            uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 16; ++i) o[i >> 2] |= one() << (8 * (i & 3));
            if (vec_ok) {
                reinterpret_cast<uint4*>(out)[gi] = make_uint4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) out[gi * 16 + i] = (uint8_t)(o[i >> 2] >> (8 * (i & 3)));
            }
        }
        for (uint64_t i = groups << 4; i < nsym; ++i) out[i] = (uint8_t)one();
    } else if (!bad) {
        // codes longer than 32 bits: canonical search on a 64-bit peek
        uint64_t pos = start;
        for (uint64_t i = 0; i < nsym; ++i) {
            const uint64_t top = peek64(f.words, f.nwords, pos);
            uint32_t len = 0, sym = 0;
            for (uint32_t l = 1; l <= maxLen; ++l) {
                const uint64_t c = top >> (64 - l);
                if (c - s_first[l] < s_cnt[l]) {
                    sym = s_sorted[s_fidx[l] + (uint32_t)(c - s_first[l])];
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
    if (bad || start + used != end) report(f.status, a.err, HUFF_E_CORRUPT);
}

hipError_t launch_decode(const DecArgs& a, uint32_t block, hipStream_t s) {
    const uint64_t blocks = (a.nitems + block - 1) / block;
    if (a.files) hipLaunchKernelGGL(k_decode<true>, dim3((uint32_t)blocks), dim3(block), 0, s, a);
    else hipLaunchKernelGGL(k_decode<false>, dim3((uint32_t)blocks), dim3(block), 0, s, a);
    return hipGetLastError();
}

// =================================================================== misc
__global__ __launch_bounds__(256) void k_copy(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, uint64_t bytes) {
    const uint64_t nvec = bytes >> 4;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) d[i] = s[i];
    if (blockIdx.x == 0)
        for (uint64_t i = (nvec << 4) + threadIdx.x; i < bytes; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
    uint64_t blocks = (bytes / 16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint8_t*)src, (uint8_t*)dst, bytes);
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

}  // namespace huff

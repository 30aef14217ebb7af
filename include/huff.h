/*
 * huff.h -- C ABI of the MI355X (gfx950) Huffman codec.
 *
 * The operation is the Huffman coding of Noel, Graham & Liu, "Parallel Data
 * Compression Techniques", Section III.A:
 *   Method 1: count how often each byte value occurs; repeatedly replace the
 *             two lowest-weight nodes by one internal node whose weight is
 *             their sum until the root remains; frequent bytes get short codes.
 *   Method 2: cut the input into segments with ids, code them, and put the
 *             coded segments back together in id order.
 * Points the paper leaves open are fixed as follows (every function below
 * obeys them, bit for bit):
 *   - tie rule: leaves are ranked by (count, byte value), internal nodes get
 *     ids after all leaves in creation order, and each merge takes the two
 *     nodes with the smallest (weight, id); one distinct byte gets a 1-bit code;
 *   - codes are canonical (RFC 1951 section 3.2.2): only the lengths come
 *     from the tree, codes of one length are consecutive in byte order;
 *   - the stream is the concatenation of the codes, most significant bit
 *     first: stream bit b is bit (31 - b%32) of 32-bit word b/32, words are
 *     little-endian in memory, unused trailing bits are zero;
 *   - segments ("chunks" of chunk_size input bytes) are bit-contiguous; the
 *     segment index chunk_off[c] (u64) is the stream bit where chunk c starts,
 *     chunk_off[nchunks] = T, the total bit count.  The words do not depend on
 *     the chunk size.
 *   - an optional finer decode index sub_lo[j] holds the low 32 bits of the
 *     stream bit where input byte j*sub_size starts (sub_lo[nsub] = low bits of
 *     T); the full offset is recovered from the enclosing chunk's chunk_off,
 *     because no chunk spans 2^32 bits.
 *
 * Conventions:
 *   - Every call returns huff_status (0 = HUFF_OK, negative = error) and never
 *     throws or aborts.  Argument errors are reported before anything is
 *     launched.
 *   - Pointers named d_* are device pointers owned by the caller; they must
 *     stay valid until the work queued on `stream` has finished.  Other
 *     pointers are host memory, read before the call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device calls
 *     are asynchronous on it.  Errors found by a kernel (corrupt stream, too
 *     small an output) are written with atomic min into the int32 d_status
 *     word if one is given (the caller zeroes it first), otherwise into the
 *     context's own status word, read by huff_ctx_status().
 *   - A context owns small device workspaces that its kernels update in
 *     place; calls that share one context must be ordered (one stream at a
 *     time).  Use one context per concurrent stream.
 *   - Limits: n < 2^38 bytes per stream or file; chunk_size a power of two in
 *     [1 KiB, 64 MiB]; sub_size 0 (no sub index) or a power of two in
 *     [16, chunk_size].  Every byte present gets a code of at most 63 bits
 *     (longer needs more than 2^38 input bytes).
 */
#ifndef HUFF_H
#define HUFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t huff_status;
enum {
    HUFF_OK = 0,
    HUFF_E_INVAL = -1,    /* bad argument (null pointer, size out of range) */
    HUFF_E_CAPACITY = -2, /* output buffer smaller than the encoded stream */
    HUFF_E_CORRUPT = -3,  /* decode found an invalid code or a wrong chunk end */
    HUFF_E_NOMEM = -4,    /* device allocation failed / over the memory budget */
    HUFF_E_AGAIN = -5,    /* server: request still pending */
    HUFF_E_HIP = -6,      /* a HIP runtime call failed */
    HUFF_E_CODELEN = -7,  /* a code would be longer than 63 bits */
    HUFF_E_NOTFOUND = -8  /* server: unknown ticket or stream handle */
};

#define HUFF_MAX_CODE_LEN 63
#define HUFF_LUT_BITS 10

/* Host-side canonical codebook (plain data). */
typedef struct huff_codebook {
    uint8_t len[256];   /* code length of byte v; 0 = v absent */
    uint64_t code[256]; /* canonical code, right-aligned: code[v] < 2^len[v] */
    uint32_t nsym;      /* K: bytes with a code */
    uint32_t max_len;   /* longest code (0 when K = 0) */
} huff_codebook;

/*
 * Device-resident codebook: everything the encoder and the decoder read.
 * Built on the device by huff_build_codebook_device() or from host lengths by
 * huff_codebook_upload(); fixed size, 256-byte aligned by the caller.
 */
typedef struct huff_dcb {
    uint32_t nsym;                /* K */
    uint32_t max_len;             /* longest code length */
    uint32_t lut_bits;            /* index width of lut[] (min(max_len, HUFF_LUT_BITS)) */
    int32_t status;               /* HUFF_OK or HUFF_E_CODELEN */
    uint64_t total_bits;          /* T = sum h[v]*len[v] (0 if built from lengths) */
    uint64_t n;                   /* sum h[v] (0 if built from lengths) */
    uint8_t len[256];             /* code length per byte value */
    uint8_t sorted_sym[256];      /* present bytes in (length, value) order */
    uint64_t code[256];           /* canonical codes, right-aligned */
    uint64_t first_code[64];      /* first canonical code of each length */
    uint32_t first_index[64];     /* sorted_sym index of that first code */
    uint32_t count[64];           /* number of codes of each length */
    uint32_t enc[256];            /* (code << 8) | len when max_len <= 24, else 0 */
    uint16_t lut[1 << HUFF_LUT_BITS]; /* peek lut_bits bits -> sym | len << 8; 0 = longer code */
} huff_dcb;

/* Launch knobs; 0 selects the built-in or autotuned default. */
typedef struct huff_params {
    uint32_t hist_blocks;     /* histogram workgroups (persistent grid) */
    uint32_t hist_depth;      /* histogram replicas per workgroup (1..32, power of 2) */
    uint32_t dec_block;       /* direct-decode workgroup size (64, 128, 192 or 256) */
    uint32_t enc_blocks_per_cu; /* persistent encode workgroups per compute unit (1..16) */
} huff_params;

typedef struct huff_ctx huff_ctx;

const char* huff_strerror(huff_status s);

/* Context on HIP device `device`; params may be NULL. */
huff_status huff_ctx_create(int device, const huff_params* params, huff_ctx** out);
void huff_ctx_destroy(huff_ctx* ctx);
huff_status huff_ctx_set_params(huff_ctx* ctx, const huff_params* params);
huff_status huff_ctx_get_params(const huff_ctx* ctx, huff_params* out);
/* Waits for the device, returns the context's status word in *out and, if
   reset != 0, clears it. */
huff_status huff_ctx_status(huff_ctx* ctx, int32_t* out, int reset);

/*
 * Byte histogram (Method 1's frequency count): d_hist[v] = number of i < n
 * with d_in[i] == v, as 256 u64.  d_in has any alignment.
 */
huff_status huff_histogram(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint64_t* d_hist, void* stream);

/*
 * Huffman code lengths under the tie rule above, then canonical codes, on
 * the host.  hist and out are host memory.  HUFF_E_CODELEN if a code would
 * exceed 63 bits.
 */
huff_status huff_build_codebook(const uint64_t hist[256], huff_codebook* out);

/* T = sum over v of hist[v] * cb->len[v] (host). */
uint64_t huff_encoded_bits(const uint64_t hist[256], const huff_codebook* cb);

/*
 * Same codebook built on the device from a device histogram (one workgroup,
 * no host round trip): fills d_cb including the decode tables, total_bits
 * and n.  On an over-long code, d_cb->status = HUFF_E_CODELEN and d_status
 * gets it too.
 */
huff_status huff_build_codebook_device(huff_ctx* ctx, const uint64_t* d_hist, huff_dcb* d_cb, int32_t* d_status,
                                       void* stream);

/*
 * Device codebook from the code lengths of a host codebook (cb->len only;
 * codes and tables are derived on the device).  Asynchronous: the lengths
 * travel as kernel arguments.
 */
huff_status huff_codebook_upload(huff_ctx* ctx, const huff_codebook* cb, huff_dcb* d_cb, void* stream);

/*
 * Encode d_in[0..n) with the codebook d_cb (Method 1 coding, Method 2
 * segment index).  Outputs:
 *   d_words[0..ceil(T/32))        the packed stream; cap_words is the size of
 *                                 d_words.  ceil(n/4) words always suffice
 *                                 (a Huffman code never averages more than
 *                                 8 bits per byte).  If T > 32*cap_words
 *                                 nothing beyond cap_words is written and
 *                                 HUFF_E_CAPACITY is reported.
 *   d_chunk_off[0..nchunks]       u64 segment index, nchunks = ceil(n/chunk_size)
 *   d_sub_lo[0..nsub]             optional (sub_size != 0): u32 decode index,
 *                                 nsub = ceil(n/sub_size)
 * A byte with no code in d_cb is reported as HUFF_E_INVAL through d_status.
 */
huff_status huff_encode(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, const huff_dcb* d_cb, uint32_t chunk_size,
                        uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off, uint32_t sub_size,
                        uint32_t* d_sub_lo, int32_t* d_status, void* stream);

/*
 * The whole compress path in one call, with no host round trip: histogram
 * of d_in, codebook built on the device into d_cb (and, if d_hist is not
 * NULL, the histogram copied to d_hist), then huff_encode.  Same arguments
 * and outputs as huff_histogram + huff_build_codebook_device + huff_encode.
 */
huff_status huff_compress(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint32_t chunk_size, huff_dcb* d_cb,
                          uint64_t* d_hist, uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off,
                          uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status, void* stream);

/*
 * Chunk-indexed decode (the inverse of huff_encode): writes n bytes to
 * d_out.  d_words has nwords valid words; every read past them is treated as
 * corrupt.  With d_sub_lo (sub_size != 0) the decoder starts one lane at
 * every sub_size input bytes, otherwise one lane per chunk.  A code that is
 * not in d_cb, or a chunk / sub-block whose last code does not end exactly at
 * the next index entry, is reported as HUFF_E_CORRUPT (the bytes of that
 * sub-block are then unspecified).
 */
huff_status huff_decode(huff_ctx* ctx, const uint32_t* d_words, uint64_t nwords, const uint64_t* d_chunk_off,
                        uint64_t n, uint32_t chunk_size, const uint32_t* d_sub_lo, uint32_t sub_size,
                        const huff_dcb* d_cb, uint8_t* d_out, int32_t* d_status, void* stream);

/*
 * Plain device copy of `bytes` bytes with 16-byte vector loads and stores:
 * the bandwidth probe the kernels are compared against.
 */
huff_status huff_copy(huff_ctx* ctx, const void* d_src, void* d_dst, uint64_t bytes, void* stream);

/* sizeof of the ABI structs, for bindings: 0 huff_dcb, 1 huff_codebook,
   2 huff_params; 0 for any other value. */
uint64_t huff_abi_sizeof(int which);

#ifdef __cplusplus
}
#endif

#endif /* HUFF_H */

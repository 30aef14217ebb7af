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
 *   - The device calls allocate nothing once the context's workspaces are
 *     large enough for the input, so they can be captured into a HIP graph
 *     after one eager call of the same size; a later call on that context
 *     with a larger input grows (reallocates) the workspaces the graph
 *     refers to.  Keep captured work on a context of its own, or use
 *     huff_compress_noalloc.
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
    HUFF_E_NOTFOUND = -8, /* server: unknown ticket or stream handle */
    HUFF_E_MISMATCH = -9  /* server: the result differs from the expected result the request carried */
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
 * huff_codebook_upload(); fixed size.  Its address must be a multiple of 16
 * (the encoder copies its tables with 16-byte transfers); calls given a
 * misaligned d_cb return HUFF_E_INVAL.
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

/* Launch knobs (they change how the work is split, never the output).  A
   field of 0 keeps the library's built-in default for it; the autotuner
   (paper_2306_11070_amd/autotune.py) times candidates on the caller's data
   and passes its choices in through these fields. */
typedef struct huff_params {
    uint32_t hist_blocks;     /* histogram workgroups (persistent grid) */
    uint32_t hist_depth;      /* histogram replicas per workgroup (1..32, power of 2) */
    uint32_t dec_block;       /* direct-decode workgroup size (64, 128, 192 or 256) */
    uint32_t enc_blocks_per_cu; /* encode workgroups per compute unit (1..1024; a grid of at least one
                                   workgroup per 16 KiB tile takes one tile per workgroup) */
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
 * Kernel timing (measurement support, not part of the method).  While timing
 * is on, the single-stream calls (huff_histogram, huff_compress, huff_encode,
 * huff_decode and the device codebook builds) record a HIP event before and
 * after each launch of the kernels below, on the stream the kernel runs on;
 * batch plans and the server record nothing.  huff_ctx_kernel_time waits for
 * the recorded events and returns the summed launch durations (ms) and the
 * launch count of one kernel since the last reset; reset != 0 clears that
 * kernel's record.  Turning timing off drops unread records.  Launches
 * queued on a stream that is being captured into a graph are not recorded.
 */
enum {
    HUFF_K_HIST = 0,      /* k_hist: byte histogram */
    HUFF_K_CODEBOOK = 1,  /* k_codebook: lengths, canonical codes, decode tables */
    HUFF_K_SCAN = 2,      /* k_tile_bits + k_tile_scan: tile offsets */
    HUFF_K_ENCODE = 3,    /* k_encode: packing, segment and decode index */
    HUFF_K_DECODE = 4,    /* k_decode_lds (all its launches) or k_decode */
    HUFF_K_COUNT = 5
};
huff_status huff_ctx_set_timing(huff_ctx* ctx, int enable);
huff_status huff_ctx_kernel_time(huff_ctx* ctx, int kernel, double* total_ms, uint64_t* launches, int reset);

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
 * huff_compress for callers that cannot allocate device memory: code under
 * HIP graph capture, serving loops and harnesses that forbid hipMalloc.  Same
 * arguments, outputs and results as huff_compress, but every workspace comes
 * from one fixed device array that the library holds on each device until the
 * process ends (about 8.5 MB), so the call itself allocates nothing.  n must
 * be at most HUFF_NOALLOC_MAX_N; a larger n returns HUFF_E_INVAL before
 * anything is queued.  All calls on one device share that array: calls that
 * overlap on one device (different streams, or different host threads) race
 * and must be ordered by the caller.  HUFF_E_HIP if the array's address could
 * not be found when ctx was created.
 */
#define HUFF_NOALLOC_MAX_N (256ull << 20)
huff_status huff_compress_noalloc(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint32_t chunk_size, huff_dcb* d_cb,
                                  uint64_t* d_hist, uint32_t* d_words, uint64_t cap_words, uint64_t* d_chunk_off,
                                  uint32_t sub_size, uint32_t* d_sub_lo, int32_t* d_status, void* stream);

/*
 * Chunk-indexed decode (the inverse of huff_encode): writes n bytes to
 * d_out.  d_words has nwords valid words; every read past them is treated as
 * corrupt.  With d_sub_lo (sub_size != 0) the decoder starts one lane at
 * every sub_size input bytes, otherwise one lane per chunk.  A code that is
 * not in d_cb, or a chunk / sub-block whose last code does not end exactly at
 * the next index entry, is reported as HUFF_E_CORRUPT (the bytes of that
 * sub-block are then unspecified).  d_out has any alignment; 16-byte aligned
 * is the fast path.
 */
huff_status huff_decode(huff_ctx* ctx, const uint32_t* d_words, uint64_t nwords, const uint64_t* d_chunk_off,
                        uint64_t n, uint32_t chunk_size, const uint32_t* d_sub_lo, uint32_t sub_size,
                        const huff_dcb* d_cb, uint8_t* d_out, int32_t* d_status, void* stream);

/*
 * Plain device copy of `bytes` bytes (the bandwidth probe the kernels are
 * compared against): one workgroup per contiguous 16 KiB, each thread
 * issuing four 16-byte non-temporal loads before it stores them.  d_src and
 * d_dst must be 16-byte aligned.
 */
huff_status huff_copy(huff_ctx* ctx, const void* d_src, void* d_dst, uint64_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Method 3 (Section III.A): a block transform before the Huffman code.  The
 * input is cut into blocks; each block's cyclic rotations are sorted and
 * their last column kept (the Burrows-Wheeler transform), which gathers
 * equal bytes into runs; the last column is then move-to-front coded (each
 * byte becomes its position in a list of the 256 byte values, reset to value
 * order at every block, and moves to the front), because a byte Huffman code
 * of the last column alone costs exactly the bits of the input (it is a
 * permutation of each block).  The coded positions are then compressed with
 * huff_compress (Methods 1 and 2).  Blocks are independent, so both
 * directions run block-parallel.
 *
 * Readings: rotations compare as byte strings, equal rotations (a periodic
 * block) in start order; the inverse needs the sorted row of one rotation per
 * block, and these calls record the row of every rotation that starts at a
 * multiple of `every` (a decode index, like sub_lo: the inverse rebuilds each
 * `every`-byte piece independently).
 * ------------------------------------------------------------------------ */
#define HUFF_BWT_MAX_BLOCK 16384u

/*
 * Forward transform of d_in[0..n) in blocks of `block` bytes (a power of two
 * in [1024, HUFF_BWT_MAX_BLOCK]; the last block shorter).  d_last[0..n): each
 * block's last column; d_rows[j] (j < ceil(n/every)): the sorted row (< 2^14)
 * of the rotation that starts at byte j*every, within its block; `every` a
 * power of two in [16, block].  d_rows[j] for j = b*block/every is block b's
 * classic primary index.
 */
huff_status huff_bwt(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint32_t block, uint32_t every, uint8_t* d_last,
                     uint16_t* d_rows, void* stream);
/*
 * Inverse of huff_bwt: d_out[0..n) from d_last and d_rows (same block and
 * every).  A row index past its block is reported as HUFF_E_CORRUPT through
 * d_status (or the context's status word); the bytes of that piece are then
 * unspecified.
 */
huff_status huff_unbwt(huff_ctx* ctx, const uint8_t* d_last, uint64_t n, uint32_t block, uint32_t every,
                       const uint16_t* d_rows, uint8_t* d_out, int32_t* d_status, void* stream);
/*
 * Move-to-front coding of d_in[0..n), the list reset every `block` bytes
 * (a power of two in [64, 2^24]): d_out[i] = position of d_in[i] in the list.
 */
huff_status huff_mtf(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint32_t block, uint8_t* d_out, void* stream);
/* Inverse of huff_mtf (same block). */
huff_status huff_unmtf(huff_ctx* ctx, const uint8_t* d_in, uint64_t n, uint32_t block, uint8_t* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many independent files, each with its own histogram, codebook and
 * stream (Method 1 applied per file, as Method 2 applies it per segment).
 * A batch plan is built once on the host; its calls then launch a fixed
 * sequence of persistent kernels over all files at once (no per-file
 * launches, no host synchronisation, no allocation), which is what makes
 * them capturable in a HIP graph (huff_batch_run with use_graph).
 * ------------------------------------------------------------------------ */
typedef struct huff_file {
    const uint8_t* in;   /* device: the file's bytes (compress / encode input) */
    uint64_t n;          /* file length in bytes (< 2^38) */
    huff_dcb* cb;        /* device: its codebook (compress writes it; encode and decode read it); 16-byte aligned */
    uint32_t* words;     /* device: its encoded words (16-byte aligned); compress / encode write, decode reads */
    uint64_t cap_words;  /* capacity of words (encode) / words valid (decode) */
    uint64_t* chunk_off; /* device: nchunks + 1 segment offsets */
    uint32_t* sub_lo;    /* device: nsub + 1 decode-index entries, or NULL when the batch has no sub index */
    uint8_t* out;        /* device: decode output (n bytes, 16-byte aligned), or NULL if the batch is never decoded */
    uint64_t* hist;      /* device: 256-entry histogram written by compress, or NULL */
    int32_t* status;     /* device: the file's status word, or NULL for the context's */
} huff_file;

typedef struct huff_batch huff_batch;

enum { HUFF_OP_COMPRESS = 0, HUFF_OP_ENCODE = 1, HUFF_OP_DECODE = 2 };

/*
 * Plan a batch of nfiles files (host array, copied) with one chunk_size and
 * sub_size for all.  Allocates the plan's device tables (tile -> file map,
 * per-tile histograms and offsets), sized for these files.  The plan belongs
 * to ctx's device and is freed by huff_batch_destroy.  Returns HUFF_E_INVAL
 * for a bad file (null pointer with n > 0, misaligned cb or words, n too
 * large) and HUFF_E_NOMEM if the tables do not fit.
 */
huff_status huff_batch_create(huff_ctx* ctx, const huff_file* files, uint32_t nfiles, uint32_t chunk_size,
                              uint32_t sub_size, huff_batch** out);
void huff_batch_destroy(huff_batch* batch);

/*
 * Runs one operation over every file of the batch on `stream`:
 *   HUFF_OP_COMPRESS: per-file histogram and codebook (into files[i].cb),
 *                     then encode;
 *   HUFF_OP_ENCODE:   encode with the codebooks already in files[i].cb;
 *   HUFF_OP_DECODE:   decode every file into files[i].out.
 * Results are bit-identical to the single-file calls on each file.  With
 * use_graph != 0 the launch sequence of this operation is captured into a
 * HIP graph on first use and replayed afterwards (the files' buffers must
 * then stay the same).  Errors found on the device go to files[i].status.
 * HUFF_OP_DECODE on a plan where a non-empty file has no `out` returns
 * HUFF_E_INVAL.
 */
huff_status huff_batch_run(huff_batch* batch, int op, int use_graph, void* stream);

/* The three operations by name (no graph). */
huff_status huff_compress_batch(huff_batch* batch, void* stream);
huff_status huff_encode_batch(huff_batch* batch, void* stream);
huff_status huff_decode_batch(huff_batch* batch, void* stream);

/* ------------------------------------------------------------------------
 * Request server: a request loop that admits compress and decompress
 * requests of mixed sizes against a device-memory budget, keeps compressed
 * streams (codebook, words, indexes) resident on the device, and batches the
 * requests that are waiting whenever a launch slot is free (continuous
 * batching: requests arriving while others are on the GPU join the next
 * batch, which runs concurrently on another stream).  Each request's result
 * is bit-identical to the single-stream calls on the same data.
 * A server thread owns the scheduling; the calls below are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct huff_server huff_server;

typedef struct huff_server_cfg {
    uint64_t mem_budget_bytes; /* device memory for resident streams, outputs and batch tables (0: 1 GiB) */
    uint32_t nslots;           /* batches in flight at once, one stream each (0: 2) */
    uint32_t max_batch;        /* requests per batch (0: 512) */
    uint32_t chunk_size;       /* segment size of compressed streams (0: 256 KiB) */
    uint32_t sub_size;         /* decode index granularity, 0 for none (default 0) */
} huff_server_cfg;

enum { HUFF_REQ_DISCARD = 1 }; /* request flag: free the result's device memory as soon as it is done */

typedef struct huff_request {
    int32_t op;             /* HUFF_OP_COMPRESS or HUFF_OP_DECODE */
    uint32_t flags;         /* HUFF_REQ_* */
    const uint8_t* d_in;    /* compress: device input of n bytes, caller-owned until the request is done */
    uint64_t n;             /* compress: input length */
    uint64_t stream_handle; /* decode: a resident stream (result of a finished compress) */
    /* Optional check of the result on the device (NULL: none).  Once the
       request has run, its result is compared with d_expect: for a compress,
       the stream must be expect_bits long and its ceil(expect_bits/32) words
       must equal those at d_expect; for a decode, the n decoded bytes must
       equal those at d_expect.  A difference sets the result's status to
       HUFF_E_MISMATCH.  d_expect is caller-owned until the request is done. */
    const void* d_expect;
    uint64_t expect_bits;   /* compress with d_expect: the expected total bits T */
} huff_request;

typedef struct huff_result {
    int32_t status;         /* HUFF_OK or the request's error */
    uint64_t handle;        /* compress: the resident stream; decode: the output buffer (release both);
                               0 with HUFF_REQ_DISCARD */
    uint64_t in_bytes;      /* bytes the request consumed (compress: n; decode: encoded bytes) */
    uint64_t out_bytes;     /* compress: encoded bytes (ceil(T/8)); decode: n */
    double t_submit, t_start, t_done; /* seconds on a steady clock: submitted, launched, seen complete */
} huff_result;

typedef struct huff_stream_info {
    uint64_t n;             /* original length */
    uint64_t total_bits;    /* T (compress results) */
    const huff_dcb* cb;     /* device pointers valid until the handle is released */
    const uint32_t* words;
    const uint64_t* chunk_off;
    const uint32_t* sub_lo; /* NULL without a sub index */
    const uint8_t* out;     /* decode results: the decoded bytes */
} huff_stream_info;

/* Creates a server on ctx's device (it takes over ctx: use another context
   for other calls).  Reserves the memory budget up front. */
huff_status huff_server_create(huff_ctx* ctx, const huff_server_cfg* cfg, huff_server** out);
/* Queues a request; never blocks on the GPU.  HUFF_E_NOMEM if it can never
   fit the budget, HUFF_E_NOTFOUND for an unknown stream handle. */
huff_status huff_server_submit(huff_server* s, const huff_request* req, uint64_t* ticket);
/* HUFF_E_AGAIN while pending; HUFF_OK once done (result filled, ticket
   retired); HUFF_E_NOTFOUND for an unknown ticket. */
huff_status huff_server_poll(huff_server* s, uint64_t ticket, huff_result* out);
/* Blocks until the request is done, then as huff_server_poll. */
huff_status huff_server_wait(huff_server* s, uint64_t ticket, huff_result* out);
/* Device pointers of a resident stream or decode output. */
huff_status huff_server_stream(huff_server* s, uint64_t handle, huff_stream_info* out);
/* Frees a resident stream or decode output (deferred while a queued decode
   still reads it). */
huff_status huff_server_release(huff_server* s, uint64_t handle);
/* Open-loop load generator: submits reqs[i] at arrival_s[i] seconds after
   the call (spinning between arrivals), waits for all, fills results[i].
   results[i].t_submit is the scheduled arrival time, so latency includes
   any delay in submitting. */
huff_status huff_server_replay(huff_server* s, const huff_request* reqs, const double* arrival_s, uint32_t count,
                               huff_result* results);
/* Counters: [0] batches launched, [1] requests done, [2] bytes in use of the
   budget, [3] peak bytes in use, [4] requests waiting, [5] batches in flight. */
huff_status huff_server_stats(huff_server* s, uint64_t out[6]);
/* Drains the requests in flight, then frees everything. */
void huff_server_destroy(huff_server* s);

/* sizeof of the ABI structs, for bindings: 0 huff_dcb, 1 huff_codebook,
   2 huff_params, 3 huff_file, 4 huff_server_cfg, 5 huff_request,
   6 huff_result, 7 huff_stream_info; 0 for any other value. */
uint64_t huff_abi_sizeof(int which);

#ifdef __cplusplus
}
#endif

#endif /* HUFF_H */

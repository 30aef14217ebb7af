/*
 * Seeded synthetic inputs for the Huffman codec: the byte streams that both
 * the CPU oracle and the GPU library consume.  Nothing here encodes or
 * decodes; it only draws bytes.
 *
 * The paper measures on a 45 MB English book corpus (Section III.A) that is
 * not available, so these generators stand in for it with text-shaped data:
 *   - i.i.d. Zipf(s) bytes over an alphabet given in rank order;
 *   - an order-2 byte Markov chain over the 96 printable symbols (newline and
 *     0x20..0x7E), each transition row a Zipf(s) distribution over its own
 *     seeded permutation of the alphabet, with a newline forced after a line
 *     length drawn from a rounded normal distribution;
 *   - word-level text: words drawn i.i.d. Zipf(s) from a seeded vocabulary of
 *     lowercase words, separated by spaces, lines broken as above.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, "Scrambled linear
 * pseudorandom number generators", 2018) seeded through SplitMix64
 * (Steele, Lea & Flood, OOPSLA 2014).  A stream is cut into independent
 * generation blocks of GEN_BLOCK bytes; block b draws from its own generator,
 * so any block range can be produced on its own thread and the bytes do not
 * depend on how the work was split.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GEN_BLOCK (1u << 20) /* bytes per independent generation block */

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* Generator for (seed, stream id): the four state words come from SplitMix64. */
static void rng_seed(rng_t* r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull);
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* Standard normal by the Box-Muller transform. */
static double rng_normal(rng_t* r) {
    double u1 = rng_unit(r), u2 = rng_unit(r);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Cumulative Zipf(s) over ranks 1..k, normalised so that cdf[k-1] == 1. */
static void zipf_cdf(double s, uint32_t k, double* cdf) {
    double acc = 0.0;
    for (uint32_t i = 0; i < k; ++i) {
        acc += pow((double)(i + 1), -s);
        cdf[i] = acc;
    }
    for (uint32_t i = 0; i < k; ++i) cdf[i] /= acc;
    cdf[k - 1] = 1.0;
}

/* Smallest rank index i with u < cdf[i]. */
static inline uint32_t cdf_pick(const double* cdf, uint32_t k, double u) {
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

uint32_t gen_block_bytes(void) { return GEN_BLOCK; }

/* Fisher-Yates shuffle of symbols[0..k) into out, driven by (seed, stream). */
void gen_permutation(const uint8_t* symbols, uint32_t k, uint64_t seed, uint64_t stream, uint8_t* out) {
    rng_t r;
    rng_seed(&r, seed, stream);
    memcpy(out, symbols, k);
    for (uint32_t i = k; i > 1; --i) {
        uint32_t j = (uint32_t)(rng_next(&r) % i);
        uint8_t t = out[i - 1];
        out[i - 1] = out[j];
        out[j] = t;
    }
}

/*
 * i.i.d. Zipf(s) bytes: rank i (0-based) maps to alphabet[i].  Fills the
 * generation blocks [blk_lo, blk_hi) of an n-byte stream.  Returns 0, or -1 on
 * bad arguments.
 */
int gen_zipf_iid(uint8_t* out, uint64_t n, uint64_t seed, double s, const uint8_t* alphabet, uint32_t k,
                 uint64_t blk_lo, uint64_t blk_hi) {
    if (k == 0 || k > 256 || (n && !out)) return -1;
    double cdf[256];
    zipf_cdf(s, k, cdf);
    for (uint64_t b = blk_lo; b < blk_hi; ++b) {
        uint64_t lo = b * (uint64_t)GEN_BLOCK;
        if (lo >= n) break;
        uint64_t hi = lo + GEN_BLOCK < n ? lo + GEN_BLOCK : n;
        rng_t r;
        rng_seed(&r, seed, 0x100000000ull + b);
        for (uint64_t i = lo; i < hi; ++i) out[i] = alphabet[cdf_pick(cdf, k, rng_unit(&r))];
    }
    return 0;
}

/* The 96 printable symbols: newline, then 0x20..0x7E. */
static void a96(uint8_t* sym) {
    sym[0] = 0x0A;
    for (int i = 0; i < 95; ++i) sym[1 + i] = (uint8_t)(0x20 + i);
}

uint32_t gen_markov_table_bytes(void) { return 96u * 96u * 96u; }

/*
 * Transition table of the order-2 chain: row (a, b) (indices into the 96
 * printable symbols) holds its own seeded permutation of the alphabet; entry
 * [row*96 + rank] is the symbol of that Zipf rank.
 */
void gen_markov_table(uint64_t seed, uint8_t* table) {
    uint8_t sym[96];
    a96(sym);
    for (uint32_t row = 0; row < 96u * 96u; ++row) gen_permutation(sym, 96, seed, 0x200000000ull + row, table + (uint64_t)row * 96);
}

static inline uint32_t a96_index(uint8_t c) { return c == 0x0A ? 0u : (uint32_t)(c - 0x20 + 1); }

static inline uint32_t draw_line_len(rng_t* r, double mu, double sigma) {
    double v = floor(mu + sigma * rng_normal(r) + 0.5);
    return v < 1.0 ? 1u : (uint32_t)v;
}

/*
 * Order-2 Markov text.  Every generation block starts from the state
 * (newline, newline) with a fresh line length; after `len` non-newline bytes
 * a newline is forced, and any newline (forced or drawn) starts a new line.
 */
int gen_markov(uint8_t* out, uint64_t n, uint64_t seed, double s, double line_mu, double line_sigma,
               const uint8_t* table, uint64_t blk_lo, uint64_t blk_hi) {
    if (n && (!out || !table)) return -1;
    double cdf[96];
    zipf_cdf(s, 96, cdf);
    for (uint64_t b = blk_lo; b < blk_hi; ++b) {
        uint64_t lo = b * (uint64_t)GEN_BLOCK;
        if (lo >= n) break;
        uint64_t hi = lo + GEN_BLOCK < n ? lo + GEN_BLOCK : n;
        rng_t r;
        rng_seed(&r, seed, 0x300000000ull + b);
        uint32_t p2 = 0, p1 = 0; /* both newline */
        uint32_t run = 0, line = draw_line_len(&r, line_mu, line_sigma);
        for (uint64_t i = lo; i < hi; ++i) {
            uint8_t c;
            if (run >= line) {
                c = 0x0A;
            } else {
                const uint8_t* row = table + (uint64_t)(p2 * 96u + p1) * 96u;
                c = row[cdf_pick(cdf, 96, rng_unit(&r))];
            }
            if (c == 0x0A) {
                run = 0;
                line = draw_line_len(&r, line_mu, line_sigma);
            } else {
                ++run;
            }
            out[i] = c;
            p2 = p1;
            p1 = a96_index(c);
        }
    }
    return 0;
}

/*
 * Per-file parameters of the batched workload: size log-uniform in
 * [size_lo, size_hi], Zipf exponent uniform in [s_lo, s_hi], alphabet size
 * uniform in {k_lo..k_hi}.  File i draws from stream (seed, i).
 */
void gen_file_params(uint64_t seed, uint32_t i, uint64_t size_lo, uint64_t size_hi, double s_lo, double s_hi,
                     uint32_t k_lo, uint32_t k_hi, uint64_t* size, double* s, uint32_t* k) {
    rng_t r;
    rng_seed(&r, seed, 0x400000000ull + i);
    double a = log((double)size_lo), bnd = log((double)size_hi);
    double v = floor(exp(a + (bnd - a) * rng_unit(&r)));
    if (v < (double)size_lo) v = (double)size_lo;
    if (v > (double)size_hi) v = (double)size_hi;
    *size = (uint64_t)v;
    *s = s_lo + (s_hi - s_lo) * rng_unit(&r);
    *k = k_lo + (uint32_t)(rng_next(&r) % (uint64_t)(k_hi - k_lo + 1));
}

/*
 * Word-level text.  The vocabulary (seed, its own stream) holds `vocab`
 * words of 1..`max_word` lowercase letters: lengths uniform, letters Zipf(1.0)
 * over a seeded permutation of 'a'..'z'.  Text: word ranks drawn Zipf(s)
 * (rank 1 = vocabulary word 0), one space between words, and a newline in
 * place of the space once the line has reached a length drawn as in
 * gen_markov.  Every generation block starts a new line with a fresh word.
 * `scratch` holds vocab * (max_word + 1) bytes plus 8 * vocab bytes (the
 * cumulative word distribution) and may be shared by the threads that fill
 * different blocks only if every thread filled it the same way first.
 */
uint64_t gen_words_scratch_bytes(uint32_t vocab, uint32_t max_word) {
    return (uint64_t)vocab * (max_word + 1) + 8ull * vocab;
}

int gen_words_vocab(uint64_t seed, uint32_t vocab, uint32_t max_word, uint8_t* scratch) {
    if (vocab == 0 || max_word == 0 || max_word > 64 || !scratch) return -1;
    uint8_t letters[26], perm[26];
    for (int i = 0; i < 26; ++i) letters[i] = (uint8_t)('a' + i);
    gen_permutation(letters, 26, seed, 0x500000000ull, perm);
    double lcdf[26];
    zipf_cdf(1.0, 26, lcdf);
    rng_t r;
    rng_seed(&r, seed, 0x600000000ull);
    uint8_t* words = scratch;  /* word w: length byte, then its letters */
    for (uint32_t w = 0; w < vocab; ++w) {
        uint8_t* p = words + (uint64_t)w * (max_word + 1);
        const uint32_t len = 1 + (uint32_t)(rng_next(&r) % max_word);
        p[0] = (uint8_t)len;
        for (uint32_t k = 0; k < len; ++k) p[1 + k] = perm[cdf_pick(lcdf, 26, rng_unit(&r))];
    }
    return 0;
}

int gen_words(uint8_t* out, uint64_t n, uint64_t seed, double s, uint32_t vocab, uint32_t max_word, double line_mu,
              double line_sigma, const uint8_t* scratch, uint64_t blk_lo, uint64_t blk_hi) {
    if (vocab == 0 || max_word == 0 || max_word > 64 || (n && (!out || !scratch))) return -1;
    const uint8_t* words = scratch;
    double* cdf = (double*)malloc(sizeof(double) * vocab);
    if (!cdf) return -1;
    zipf_cdf(s, vocab, cdf);
    for (uint64_t b = blk_lo; b < blk_hi; ++b) {
        uint64_t lo = b * (uint64_t)GEN_BLOCK;
        if (lo >= n) break;
        uint64_t hi = lo + GEN_BLOCK < n ? lo + GEN_BLOCK : n;
        rng_t r;
        rng_seed(&r, seed, 0x700000000ull + b);
        uint32_t line = draw_line_len(&r, line_mu, line_sigma), run = 0;
        uint64_t i = lo;
        while (i < hi) {
            const uint8_t* w = words + (uint64_t)cdf_pick(cdf, vocab, rng_unit(&r)) * (max_word + 1);
            for (uint32_t k = 0; k < w[0] && i < hi; ++k, ++run) out[i++] = w[1 + k];
            if (i >= hi) break;
            if (run >= line) {
                out[i++] = 0x0A;
                run = 0;
                line = draw_line_len(&r, line_mu, line_sigma);
            } else {
                out[i++] = 0x20;
                ++run;
            }
        }
    }
    free(cdf);
    return 0;
}

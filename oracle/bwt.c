/*
 * CPU oracle for the block transform before Huffman coding -- TEST
 * INFRASTRUCTURE ONLY (loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline legs; never by the product path).  Plain, slow,
 * serial C that shares no code with the GPU library.
 *
 * What it follows (Noel, Graham & Liu, "Parallel Data Compression
 * Techniques", Section III.A, Method 3): the data is cut into blocks, each
 * block is transformed with the Burrows-Wheeler transform (the block's cyclic
 * rotations sorted, the last column kept), which gathers equal characters
 * into runs, and the result is Huffman coded in parallel.  Readings of what
 * the paper leaves open:
 *   - blocks of `block` bytes, the last one shorter; each block is
 *     transformed on its own (so blocks decode in parallel);
 *   - rotations compare as byte strings; equal rotations (a periodic block)
 *     are ordered by their start position;
 *   - the transformed block is the last column L of the sorted rotations;
 *     the inverse needs the row of one rotation, and this oracle records the
 *     row of every rotation that starts at a multiple of `every` (row of the
 *     rotation starting at 0 first: that is the classic primary index);
 *   - a byte-level Huffman code of L alone costs exactly as many bits as one
 *     of the block (L is a permutation of it), so, as in the usual use of the
 *     transform, L is move-to-front coded before the Huffman code: each byte
 *     becomes its position in a list of the 256 byte values (initially in
 *     value order, reset at every block), and then moves to the list's front.
 * Return codes: 0 ok, -1 invalid argument, -3 corrupt input.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_INVAL (-1)
#define O_CORRUPT (-3)

typedef struct {
    const uint8_t* s;
    uint32_t m;
} rot_ctx;

/* Rotation a against rotation b of the block: byte by byte, then start position. */
static int rot_cmp(const void* pa, const void* pb, void* arg) {
    const rot_ctx* c = (const rot_ctx*)arg;
    uint32_t a = *(const uint32_t*)pa, b = *(const uint32_t*)pb;
    for (uint32_t k = 0; k < c->m; ++k) {
        uint8_t x = c->s[(a + k) % c->m], y = c->s[(b + k) % c->m];
        if (x != y) return x < y ? -1 : 1;
    }
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int block_args(uint64_t n, uint32_t block, uint32_t every) {
    return block > 0 && every > 0 && block % every == 0 && (n == 0 || block <= (1u << 30));
}

/*
 * Forward transform of in[0..n): last[0..n) receives each block's last
 * column; rows receives, for block b, ceil(m_b / every) entries at
 * rows[b * (block / every) + k] = sorted row of the rotation starting at k*every.
 */
int oracle_bwt(const uint8_t* in, uint64_t n, uint32_t block, uint32_t every, uint8_t* last, uint32_t* rows) {
    if (!block_args(n, block, every) || (n && (!in || !last || !rows))) return O_INVAL;
    uint32_t* sa = (uint32_t*)malloc((size_t)block * sizeof(uint32_t));
    if (!sa) return O_INVAL;
    const uint64_t per = block / every;
    for (uint64_t lo = 0, b = 0; lo < n; lo += block, ++b) {
        const uint32_t m = (uint32_t)(n - lo < block ? n - lo : block);
        rot_ctx c = {in + lo, m};
        for (uint32_t i = 0; i < m; ++i) sa[i] = i;
        qsort_r(sa, m, sizeof(uint32_t), rot_cmp, &c);
        for (uint32_t r = 0; r < m; ++r) {
            last[lo + r] = c.s[(sa[r] + m - 1) % m];
            if (sa[r] % every == 0) rows[b * per + sa[r] / every] = r;
        }
    }
    free(sa);
    return O_OK;
}

/*
 * Inverse transform: out[0..n) from the last columns and the row of the
 * rotation starting at 0 of every block (rows[b * (block / every)]).  A row
 * of the sorted rotations with last character c is followed, one position
 * back in the block, by the row that starts with that same occurrence of c:
 * the j-th c of the last column is the j-th c of the first column.
 */
int oracle_unbwt(const uint8_t* last, uint64_t n, uint32_t block, uint32_t every, const uint32_t* rows, uint8_t* out) {
    if (!block_args(n, block, every) || (n && (!last || !rows || !out))) return O_INVAL;
    uint32_t* lf = (uint32_t*)malloc((size_t)block * sizeof(uint32_t));
    if (!lf) return O_INVAL;
    const uint64_t per = block / every;
    int rc = O_OK;
    for (uint64_t lo = 0, b = 0; lo < n && rc == O_OK; lo += block, ++b) {
        const uint32_t m = (uint32_t)(n - lo < block ? n - lo : block);
        const uint8_t* L = last + lo;
        uint64_t count[256] = {0}, first[256], seen[256] = {0};
        for (uint32_t r = 0; r < m; ++r) count[L[r]]++;
        uint64_t acc = 0;
        for (int c = 0; c < 256; ++c) { first[c] = acc; acc += count[c]; }
        for (uint32_t r = 0; r < m; ++r) lf[r] = (uint32_t)(first[L[r]] + seen[L[r]]++);
        uint32_t r = rows[b * per];
        if (r >= m) { rc = O_CORRUPT; break; }
        for (uint32_t k = m; k-- > 0;) {  /* the block backwards from its end */
            out[lo + k] = L[r];
            r = lf[r];
        }
    }
    free(lf);
    return rc;
}

/* Move-to-front coding of in[0..n), the list reset at every block. */
int oracle_mtf(const uint8_t* in, uint64_t n, uint32_t block, uint8_t* out) {
    if (block == 0 || (n && (!in || !out))) return O_INVAL;
    uint8_t list[256];
    for (uint64_t i = 0; i < n; ++i) {
        if (i % block == 0)
            for (int v = 0; v < 256; ++v) list[v] = (uint8_t)v;
        const uint8_t c = in[i];
        int p = 0;
        while (list[p] != c) ++p;
        out[i] = (uint8_t)p;
        for (; p > 0; --p) list[p] = list[p - 1];
        list[0] = c;
    }
    return O_OK;
}

/* Inverse of oracle_mtf. */
int oracle_unmtf(const uint8_t* in, uint64_t n, uint32_t block, uint8_t* out) {
    if (block == 0 || (n && (!in || !out))) return O_INVAL;
    uint8_t list[256];
    for (uint64_t i = 0; i < n; ++i) {
        if (i % block == 0)
            for (int v = 0; v < 256; ++v) list[v] = (uint8_t)v;
        int p = in[i];
        const uint8_t c = list[p];
        out[i] = c;
        for (; p > 0; --p) list[p] = list[p - 1];
        list[0] = c;
    }
    return O_OK;
}

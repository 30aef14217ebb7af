/*
 * CPU oracle for the Huffman codec -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, serial C that states what the GPU path must produce, bit for
 * bit.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never does.  It shares no code, header or
 * table with the GPU library.
 *
 * What it follows (Noel, Graham & Liu, "Parallel Data Compression
 * Techniques", Section III.A):
 *   - Method 1: count how often each symbol of the fixed alphabet occurs, then
 *     build an extended weighted binary tree by repeatedly replacing the two
 *     lowest-weight nodes with one internal node whose weight is their sum,
 *     until one root remains; frequent symbols get short codes.
 *   - Method 2: the input is cut into segments with ids and the coded segments
 *     are put back together in id order.
 * The paper leaves silent: how ties between equal weights are broken, which
 * child gets 0 or 1, the bit order, and the segment layout.  The readings used
 * here are:
 *   - ties: leaves are ranked by (count, byte value); internal nodes get ids
 *     after all leaves, in creation order; each step removes the two nodes with
 *     the smallest (weight, id).  A single distinct symbol gets a 1-bit code.
 *   - codes are canonical (RFC 1951 section 3.2.2): only the code lengths are
 *     taken from the tree, codes of equal length are consecutive in symbol
 *     order.  This makes the 0/1 labelling irrelevant.
 *   - the coded stream is the concatenation of all codes, most significant
 *     bit first; stream bit b lives in 32-bit word b/32 at bit 31 - b%32;
 *     unused trailing bits are zero.
 *   - segments (chunks of C input bytes) are bit-contiguous: no padding, so
 *     the words do not depend on C; chunk_off[c] is the stream bit at which
 *     chunk c starts and chunk_off[nchunks] is the total bit count.
 * Return codes: 0 ok, -1 invalid argument, -2 output capacity too small,
 * -3 corrupt stream, -7 a code would exceed 63 bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_INVAL (-1)
#define O_CAPACITY (-2)
#define O_CORRUPT (-3)
#define O_CODELEN (-7)
#define O_MAXLEN 63

/* O1: h[v] = number of positions i with in[i] == v. */
int oracle_histogram(const uint8_t* in, uint64_t n, uint64_t* hist) {
    if (!hist || (n && !in)) return O_INVAL;
    for (int v = 0; v < 256; ++v) hist[v] = 0;
    for (uint64_t i = 0; i < n; ++i) hist[in[i]] += 1;
    return O_OK;
}

/* Present symbols ordered by (count, value), ascending; returns K. */
static int sorted_leaves(const uint64_t* hist, int* sym) {
    int k = 0;
    for (int v = 0; v < 256; ++v)
        if (hist[v]) sym[k++] = v;
    /* insertion sort: K <= 256 */
    for (int i = 1; i < k; ++i) {
        int s = sym[i], j = i - 1;
        while (j >= 0 && (hist[sym[j]] > hist[s] || (hist[sym[j]] == hist[s] && sym[j] > s))) {
            sym[j + 1] = sym[j];
            --j;
        }
        sym[j + 1] = s;
    }
    return k;
}

/* Leaf depths from parent links; node ids grow from children to parents. */
static int depths_to_lengths(int k, const int* parent, const int* sym, uint8_t* len) {
    int depth[511];
    int root = 2 * k - 2;
    depth[root] = 0;
    for (int id = root - 1; id >= 0; --id) depth[id] = depth[parent[id]] + 1;
    for (int i = 0; i < k; ++i) {
        if (depth[i] > O_MAXLEN) return O_CODELEN;
        len[sym[i]] = (uint8_t)depth[i];
    }
    return O_OK;
}

/* ---- O2, first implementation: a binary min-heap keyed by (weight, id). ---- */
typedef struct { uint64_t w; int id; } node_t;

static int node_less(node_t a, node_t b) { return a.w < b.w || (a.w == b.w && a.id < b.id); }

static void heap_push(node_t* h, int* n, node_t x) {
    int i = (*n)++;
    h[i] = x;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!node_less(h[i], h[p])) break;
        node_t t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static node_t heap_pop(node_t* h, int* n) {
    node_t top = h[0];
    h[0] = h[--(*n)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && node_less(h[l], h[m])) m = l;
        if (r < *n && node_less(h[r], h[m])) m = r;
        if (m == i) break;
        node_t t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

/* O2: Huffman code lengths, len[v] = depth of leaf v (0 if v is absent). */
int oracle_code_lengths(const uint64_t* hist, uint8_t* len) {
    if (!hist || !len) return O_INVAL;
    memset(len, 0, 256);
    int sym[256];
    int k = sorted_leaves(hist, sym);
    if (k == 0) return O_OK;
    if (k == 1) { len[sym[0]] = 1; return O_OK; }
    node_t heap[512];
    int hn = 0, parent[511];
    for (int i = 0; i < k; ++i) heap_push(heap, &hn, (node_t){hist[sym[i]], i});
    for (int next = k; next < 2 * k - 1; ++next) {
        node_t a = heap_pop(heap, &hn);
        node_t b = heap_pop(heap, &hn);
        parent[a.id] = next;
        parent[b.id] = next;
        heap_push(heap, &hn, (node_t){a.w + b.w, next});
    }
    return depths_to_lengths(k, parent, sym, len);
}

/*
 * O2, second and independent implementation: the two-queue method.  Leaves
 * wait in (count, value) order, internal nodes in creation order (their
 * weights never decrease); on equal weight the leaf is taken first, which is
 * the same (weight, id) rule as above.
 */
int oracle_code_lengths_twoqueue(const uint64_t* hist, uint8_t* len) {
    if (!hist || !len) return O_INVAL;
    memset(len, 0, 256);
    int sym[256];
    int k = sorted_leaves(hist, sym);
    if (k == 0) return O_OK;
    if (k == 1) { len[sym[0]] = 1; return O_OK; }
    uint64_t iw[256];
    int parent[511];
    int li = 0, qi = 0, made = 0;
    for (int step = 0; step < k - 1; ++step) {
        int pick[2];
        uint64_t w[2];
        for (int t = 0; t < 2; ++t) {
            int take_leaf = li < k && (qi >= made || hist[sym[li]] <= iw[qi]);
            if (take_leaf) { pick[t] = li; w[t] = hist[sym[li]]; ++li; }
            else { pick[t] = k + qi; w[t] = iw[qi]; ++qi; }
        }
        iw[made] = w[0] + w[1];
        parent[pick[0]] = k + made;
        parent[pick[1]] = k + made;
        ++made;
    }
    return depths_to_lengths(k, parent, sym, len);
}

/* O3: canonical codes from lengths, as in RFC 1951 section 3.2.2. */
int oracle_canonical_codes(const uint8_t* len, uint64_t* code) {
    if (!len || !code) return O_INVAL;
    uint64_t bl_count[O_MAXLEN + 2] = {0}, next_code[O_MAXLEN + 2] = {0};
    for (int v = 0; v < 256; ++v) {
        if (len[v] > O_MAXLEN) return O_CODELEN;
        if (len[v]) bl_count[len[v]] += 1;
    }
    uint64_t c = 0;
    for (int bits = 1; bits <= O_MAXLEN; ++bits) {
        c = (c + bl_count[bits - 1]) << 1;
        next_code[bits] = c;
    }
    for (int v = 0; v < 256; ++v) {
        code[v] = 0;
        if (len[v]) code[v] = next_code[len[v]]++;
    }
    return O_OK;
}

/* T = sum over v of h[v] * len[v]. */
uint64_t oracle_total_bits(const uint64_t* hist, const uint8_t* len) {
    uint64_t t = 0;
    for (int v = 0; v < 256; ++v) t += hist[v] * len[v];
    return t;
}

/*
 * O4/O5: bit-by-bit encode of in[0..n) with chunk size `chunk` (>= 1).
 * words must hold cap_words entries; chunk_off must hold ceil(n/chunk)+1.
 */
int oracle_encode(const uint8_t* in, uint64_t n, const uint8_t* len, const uint64_t* code, uint64_t chunk,
                  uint32_t* words, uint64_t cap_words, uint64_t* chunk_off) {
    if (!len || !code || chunk == 0 || !chunk_off || (n && (!in || !words))) return O_INVAL;
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (len[in[i]] == 0) return O_INVAL; /* symbol without a code */
        total += len[in[i]];
    }
    uint64_t nw = (total + 31) / 32;
    if (nw > cap_words) return O_CAPACITY;
    for (uint64_t w = 0; w < nw; ++w) words[w] = 0;
    uint64_t b = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (i % chunk == 0) chunk_off[i / chunk] = b;
        uint8_t l = len[in[i]];
        uint64_t c = code[in[i]];
        for (int j = l - 1; j >= 0; --j) {
            if ((c >> j) & 1u) words[b / 32] |= 1u << (31 - (b % 32));
            ++b;
        }
    }
    chunk_off[(n + chunk - 1) / chunk] = b;
    return O_OK;
}

/* O6: canonical decode, one bit at a time, chunk by chunk from chunk_off. */
int oracle_decode(const uint32_t* words, uint64_t nwords, const uint64_t* chunk_off, uint64_t n, uint64_t chunk,
                  const uint8_t* len, uint8_t* out) {
    if (!len || chunk == 0 || !chunk_off || (n && (!out || !words))) return O_INVAL;
    int max_len = 0;
    uint64_t count[O_MAXLEN + 2] = {0};
    for (int v = 0; v < 256; ++v) {
        if (len[v] > O_MAXLEN) return O_CODELEN;
        if (len[v]) count[len[v]] += 1;
        if (len[v] > max_len) max_len = len[v];
    }
    /* first canonical code of each length and the symbols in (length, value) order */
    uint64_t first[O_MAXLEN + 2] = {0};
    int start[O_MAXLEN + 2] = {0};
    uint8_t sorted[256];
    uint64_t c = 0;
    int pos = 0;
    for (int l = 1; l <= max_len; ++l) {
        c = (c + count[l - 1]) << 1;
        first[l] = c;
        start[l] = pos;
        for (int v = 0; v < 256; ++v)
            if (len[v] == l) sorted[pos++] = (uint8_t)v;
    }
    uint64_t nbits = nwords * 32;
    uint64_t nchunks = (n + chunk - 1) / chunk;
    for (uint64_t ch = 0; ch < nchunks; ++ch) {
        uint64_t b = chunk_off[ch];
        uint64_t lo = ch * chunk, hi = lo + chunk < n ? lo + chunk : n;
        for (uint64_t i = lo; i < hi; ++i) {
            uint64_t code_acc = 0;
            int found = 0;
            for (int l = 1; l <= max_len; ++l) {
                if (b >= nbits) return O_CORRUPT;
                code_acc = (code_acc << 1) | ((words[b / 32] >> (31 - (b % 32))) & 1u);
                ++b;
                if (count[l] && code_acc >= first[l] && code_acc - first[l] < count[l]) {
                    out[i] = sorted[start[l] + (int)(code_acc - first[l])];
                    found = 1;
                    break;
                }
            }
            if (!found) return O_CORRUPT;
        }
        if (b != chunk_off[ch + 1]) return O_CORRUPT;
    }
    return O_OK;
}

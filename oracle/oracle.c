/*
 * Plain, slow CPU oracle for the compressed key sort
 * (Kwon et al., "Compressed Key Sort and Fast Index Reconstruction").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header, table or helper with the HIP library; both sides only see the same
 * seeded input bytes.  Every routine favours being checkable by eye against the
 * paper over being fast.
 *
 * Conventions (Sec. 3.1): a key is a string of bits; position 0 is the most
 * significant bit of byte 0, position p lives in byte p/8 under mask
 * 0x80 >> (p%8).  Variable-length keys are logically padded with zero bytes up
 * to the key width L (Sec. 4.1, multi-column keys; varchar keys carry a NUL
 * terminator which the zero padding supplies).  Record IDs are the row indices
 * 0..n-1 (Sec. 5, step 2), so ties between equal keys go by row index.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

static double pow_u(double b, uint32_t e)
{
    double r = 1;
    while (e--) r *= b;
    return r;
}

/* ------------------------------------------------------------------------- */
/* Key access                                                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    const uint8_t  *bytes;
    const uint64_t *offsets; /* NULL: fixed width, key i at bytes + i*stride */
    uint64_t n;
    uint32_t L;
    uint32_t stride;
} keyset;

/* Pointer to key i and its stored length (<= L for variable-length keys). */
static const uint8_t *key_ptr(const keyset *k, uint64_t i, uint32_t *len)
{
    if (k->offsets) {
        *len = (uint32_t)(k->offsets[i + 1] - k->offsets[i]);
        return k->bytes + k->offsets[i];
    }
    *len = k->L;
    return k->bytes + i * (uint64_t)k->stride;
}

/* Byte j of key i, zero past the stored length (Sec. 4.1 zero padding). */
static uint8_t key_byte(const keyset *k, uint64_t i, uint32_t j)
{
    uint32_t len;
    const uint8_t *p = key_ptr(k, i, &len);
    return j < len ? p[j] : 0;
}

/* Bit at position p (MSB-first) of key i. */
static int key_bit(const keyset *k, uint64_t i, uint32_t p)
{
    return (key_byte(k, i, p >> 3) >> (7 - (p & 7))) & 1;
}

/* Lexicographic comparison of the zero-padded L-byte strings. */
static int key_cmp(const keyset *k, uint64_t a, uint64_t b)
{
    for (uint32_t j = 0; j < k->L; ++j) {
        uint8_t x = key_byte(k, a, j), y = key_byte(k, b, j);
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

/* D-bit(a, b): the most significant position where keys a and b differ
 * (Sec. 3.1), or -1 when they are equal. */
static int64_t key_dbit(const keyset *k, uint64_t a, uint64_t b)
{
    for (uint32_t j = 0; j < k->L; ++j) {
        uint8_t x = key_byte(k, a, j) ^ key_byte(k, b, j);
        if (x) {
            int hb = 7;
            while (!((x >> hb) & 1)) --hb;
            return (int64_t)j * 8 + (7 - hb);
        }
    }
    return -1;
}

static void set_bit(uint8_t *bitmap, uint32_t p) { bitmap[p >> 3] |= (uint8_t)(0x80u >> (p & 7)); }
static int get_bit(const uint8_t *bitmap, uint32_t p) { return (bitmap[p >> 3] >> (7 - (p & 7))) & 1; }

/* ------------------------------------------------------------------------- */
/* Full-key sort: the order that compressed key sort must reproduce.          */
/* ------------------------------------------------------------------------- */

static int cmp_full(const void *pa, const void *pb, void *ctx)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    int c = key_cmp((const keyset *)ctx, a, b);
    if (c) return c;
    return a < b ? -1 : (a > b); /* record ID tie-break (Sec. 5, step 2) */
}

/* perm[r] = row of the r-th smallest (key, row) pair. */
int oracle_full_sort(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                     uint32_t L, uint32_t stride, uint32_t *perm)
{
    keyset k = {bytes, offsets, n, L, stride};
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    qsort_r(perm, n, sizeof(uint32_t), cmp_full, &k);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Distinction bits (Sec. 3.1, Theorem 1): union over adjacent sorted pairs.  */
/* ------------------------------------------------------------------------- */

/* bitmap (L bytes) receives D = { D-bit(key[perm[i-1]], key[perm[i]]) }.
 * Equal adjacent keys contribute nothing.  Returns 1 if some adjacent pair
 * is in descending order (the earlier key has a 1 at the D position), else 0. */
int oracle_dbits(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                 uint32_t L, uint32_t stride, const uint32_t *perm, uint8_t *bitmap)
{
    keyset k = {bytes, offsets, n, L, stride};
    int descending = 0;
    memset(bitmap, 0, L);
    for (uint64_t i = 1; i < n; ++i) {
        uint64_t a = perm ? perm[i - 1] : i - 1, b = perm ? perm[i] : i;
        int64_t p = key_dbit(&k, a, b);
        if (p < 0) continue;
        if (key_bit(&k, a, (uint32_t)p)) descending = 1;
        set_bit(bitmap, (uint32_t)p);
    }
    return descending;
}

/* D-bit of an arbitrary pair of rows; -1 if equal.  Used by the Lemma 1 pin. */
int64_t oracle_dbit_pair(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                         uint32_t L, uint32_t stride, uint64_t a, uint64_t b)
{
    keyset k = {bytes, offsets, n, L, stride};
    return key_dbit(&k, a, b);
}

/* ------------------------------------------------------------------------- */
/* D-offset (Sec. 5.3): D-offset[c] = position of the (c+1)-st 1 in the map.  */
/* ------------------------------------------------------------------------- */

uint32_t oracle_doffset(const uint8_t *bitmap, uint32_t L, uint32_t *doff)
{
    uint32_t c = 0;
    for (uint32_t p = 0; p < 8 * L; ++p)
        if (get_bit(bitmap, p)) {
            if (doff) doff[c] = p;
            ++c;
        }
    return c;
}

/* ------------------------------------------------------------------------- */
/* Compress (Sec. 3.2): the key's bits at the bitmap's 1-positions, in        */
/* ascending position order.  The string is stored left-aligned, MSB first,  */
/* in w = ceil(|D|/64) 64-bit words, word-major: ckeys[k*n + i] is word k of */
/* row i; bits past |D| are zero.                                             */
/* ------------------------------------------------------------------------- */

/* Bit-by-bit definition. */
int oracle_compress(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                    uint32_t L, uint32_t stride, const uint8_t *bitmap,
                    uint32_t w, uint64_t *ckeys)
{
    keyset k = {bytes, offsets, n, L, stride};
    memset(ckeys, 0, sizeof(uint64_t) * (size_t)w * n);
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = 0;
        for (uint32_t p = 0; p < 8 * L; ++p) {
            if (!get_bit(bitmap, p)) continue;
            if ((c >> 6) >= w) return -1;
            if (key_bit(&k, i, p))
                ckeys[(uint64_t)(c >> 6) * n + i] |= 1ull << (63 - (c & 63));
            ++c;
        }
    }
    return 0;
}

/* The extraction procedure of Sec. 5.1: cut the bitmap into 8-byte masks,
 * each starting at the byte holding the next 1 not yet covered; pull each
 * key's bits under a mask into the low-order end of a word (the effect of a
 * PEXT, here done one bit at a time); join the pieces by shift and OR. */
uint32_t oracle_windows(const uint8_t *bitmap, uint32_t L, uint32_t *start, uint64_t *mask)
{
    uint32_t nw = 0, j = 0;
    while (j < L) {
        if (!bitmap[j]) { ++j; continue; }
        uint64_t m = 0;
        for (uint32_t t = 0; t < 8; ++t) m = (m << 8) | (j + t < L ? bitmap[j + t] : 0);
        if (start) start[nw] = j;
        if (mask) mask[nw] = m;
        ++nw;
        j += 8;
    }
    return nw;
}

static uint64_t soft_pext(uint64_t v, uint64_t m, uint32_t *cnt)
{
    uint64_t r = 0;
    uint32_t c = 0;
    for (int b = 63; b >= 0; --b)
        if ((m >> b) & 1) { r = (r << 1) | ((v >> b) & 1); ++c; }
    *cnt = c;
    return r;
}

int oracle_compress_windows(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                            uint32_t L, uint32_t stride, const uint8_t *bitmap,
                            uint32_t w, uint64_t *ckeys)
{
    keyset k = {bytes, offsets, n, L, stride};
    uint32_t nwin = oracle_windows(bitmap, L, NULL, NULL);
    uint32_t *st = (uint32_t *)malloc(sizeof(uint32_t) * (nwin + 1));
    uint64_t *mk = (uint64_t *)malloc(sizeof(uint64_t) * (nwin + 1));
    oracle_windows(bitmap, L, st, mk);
    memset(ckeys, 0, sizeof(uint64_t) * (size_t)w * n);
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = 0; /* bits emitted so far */
        for (uint32_t q = 0; q < nwin; ++q) {
            uint64_t v = 0;
            for (uint32_t t = 0; t < 8; ++t) v = (v << 8) | key_byte(&k, i, st[q] + t);
            uint32_t cnt;
            uint64_t piece = soft_pext(v, mk[q], &cnt);
            /* shift-and-OR the cnt-bit piece onto the running string */
            for (int b = (int)cnt - 1; b >= 0; --b, ++c) {
                if ((c >> 6) >= w) { free(st); free(mk); return -1; }
                if ((piece >> b) & 1) ckeys[(uint64_t)(c >> 6) * n + i] |= 1ull << (63 - (c & 63));
            }
        }
    }
    free(st);
    free(mk);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sort of compressed keys (Sec. 3.2): order by the compressed strings, then  */
/* by record ID.                                                              */
/* ------------------------------------------------------------------------- */

typedef struct { const uint64_t *ck; uint32_t w; uint64_t n; } ckset;

static int cmp_comp(const void *pa, const void *pb, void *ctx)
{
    const ckset *s = (const ckset *)ctx;
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    for (uint32_t k = 0; k < s->w; ++k) {
        uint64_t x = s->ck[(uint64_t)k * s->n + a], y = s->ck[(uint64_t)k * s->n + b];
        if (x != y) return x < y ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}

int oracle_csort(const uint64_t *ckeys, uint32_t w, uint64_t n, uint32_t *perm)
{
    ckset s = {ckeys, w, n};
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    qsort_r(perm, n, sizeof(uint32_t), cmp_comp, &s);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* DS-metadata refresh at rebuild (Sec. 4.3): distinction positions of the    */
/* adjacent sorted compressed keys, mapped back to full-key positions via     */
/* D-offset (Sec. 5.3).                                                       */
/* ------------------------------------------------------------------------- */

/* ckeys: word-major, in row order; perm: the sorted order.  bitmap_out (L
 * bytes) receives the new D-bitmap; pair_pos[i-1] (optional) the full-key
 * D position of sorted pair (i-1, i), 0xFFFFFFFF when the compressed keys are
 * equal.  Returns -1 if a D index falls outside the bitmap's 1-positions. */
int oracle_refine(const uint64_t *ckeys, uint32_t w, uint64_t n, const uint32_t *perm,
                  const uint8_t *bitmap_in, uint32_t L, uint8_t *bitmap_out, uint32_t *pair_pos)
{
    uint32_t nd = oracle_doffset(bitmap_in, L, NULL);
    uint32_t *doff = (uint32_t *)malloc(sizeof(uint32_t) * (nd + 1));
    oracle_doffset(bitmap_in, L, doff);
    memset(bitmap_out, 0, L);
    for (uint64_t i = 1; i < n; ++i) {
        uint64_t a = perm[i - 1], b = perm[i];
        int64_t c = -1;
        for (uint32_t k = 0; k < w && c < 0; ++k) {
            uint64_t x = ckeys[(uint64_t)k * n + a] ^ ckeys[(uint64_t)k * n + b];
            if (x) {
                int lead = 0;
                while (!((x >> (63 - lead)) & 1)) ++lead;
                c = (int64_t)k * 64 + lead;
            }
        }
        if (c < 0) {
            if (pair_pos) pair_pos[i - 1] = 0xFFFFFFFFu;
            continue;
        }
        if ((uint64_t)c >= nd) { free(doff); return -1; }
        set_bit(bitmap_out, doff[c]);
        if (pair_pos) pair_pos[i - 1] = doff[c];
    }
    free(doff);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Variant bitmap and reference key (Sec. 4.2-4.3).                           */
/* ------------------------------------------------------------------------- */

/* variant (L bytes) = OR over all keys of (key XOR reference), with the
 * reference key taken as row ref_row. */
int oracle_variant(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                   uint32_t L, uint32_t stride, uint64_t ref_row, uint8_t *variant)
{
    keyset k = {bytes, offsets, n, L, stride};
    memset(variant, 0, L);
    for (uint64_t i = 0; i < n; ++i)
        for (uint32_t j = 0; j < L; ++j) variant[j] |= key_byte(&k, i, j) ^ key_byte(&k, ref_row, j);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* DS-metadata maintenance (Sec. 4.3).                                        */
/* ------------------------------------------------------------------------- */

/* Inserts, one after another, as Sec. 4.3 describes them.  Rows order[0..ns)
 * of the key set form the current index in key order; rows ins[0..m) are
 * inserted in that sequence.  For each inserted key K: find its place between
 * A and B (the last key <= K and the first key > K), then set
 * max(D-bit(A, K), D-bit(K, B)) in the D-bitmap -- by Lemma 1 the smaller of
 * the two is D-bit(A, B), which is set already -- and OR (K xor reference key)
 * into the variant bitmap.  A missing neighbour (K first or last) or an equal
 * one (D-bit -1) contributes nothing.  dbitmap (and variant, if not NULL) are
 * L-byte bitmaps updated in place; ref_row is the reference key's row.
 * Deletes (Sec. 4.3) leave both bitmaps unchanged, so they have no routine. */
int oracle_insert(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                  uint32_t L, uint32_t stride, const uint32_t *order, uint64_t ns,
                  const uint32_t *ins, uint64_t m, uint64_t ref_row,
                  uint8_t *dbitmap, uint8_t *variant)
{
    keyset k = {bytes, offsets, n, L, stride};
    uint32_t *cur = (uint32_t *)malloc((ns + m + 1) * sizeof(uint32_t));
    if (!cur) return -1;
    if (ns) memcpy(cur, order, ns * sizeof(uint32_t));
    uint64_t c = ns;
    for (uint64_t t = 0; t < m; ++t) {
        uint32_t K = ins[t];
        uint64_t lo = 0, hi = c; /* place: first index whose key is greater than K */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (key_cmp(&k, cur[mid], K) <= 0) lo = mid + 1; else hi = mid;
        }
        int64_t da = lo > 0 ? key_dbit(&k, cur[lo - 1], K) : -1;
        int64_t db = lo < c ? key_dbit(&k, K, cur[lo]) : -1;
        int64_t mx = da > db ? da : db;
        if (mx >= 0) set_bit(dbitmap, (uint32_t)mx);
        memmove(cur + lo + 1, cur + lo, (c - lo) * sizeof(uint32_t));
        cur[lo] = K;
        ++c;
        if (variant)
            for (uint32_t j = 0; j < L; ++j) variant[j] |= key_byte(&k, K, j) ^ key_byte(&k, ref_row, j);
    }
    free(cur);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Index tree bulk load (Sec. 5.3, index construction).                       */
/*                                                                            */
/* Sorted keys fill 256-byte nodes bottom-up: leaves of at most 14 entries of */
/* 16 bytes (24-byte header plus an 8-byte next pointer: (256-32)/16 = 14),   */
/* inner nodes of at most 9 entries of 24 bytes; each node is filled with     */
/* floor(fanout * fill) entries, the last node of a level with the rest.      */
/* Node layout (little-endian; unused bytes zero):                            */
/*   header: high rid u64 @0, count u16 @8, level u16 @10 (0 = leaf),         */
/*           zero u32 @12, sorted position of the node's first key u64 @16    */
/*   leaf:   next leaf's node index u64 @24 (all ones for the last leaf),     */
/*           entries @32: partial key u32, D position u16, key length u16,    */
/*           record ID u64                                                    */
/*   inner:  entries @24: partial key u32, D position u16, key length u16,    */
/*           child node index u64, child's highest key's record ID u64        */
/* Levels are stored leaves first, each level's nodes in key order; the      */
/* children of an inner node are consecutive nodes of the level below.        */
/* An entry's D position is that of its key against the previous entry's key  */
/* at the same level (0xFFFF: first entry of the level; 0xFFFE: equal keys).  */
/* Its partial key is the pk bits after that position (Sec. 4.2), MSB-first   */
/* and left-aligned in 32 bits; the first entry takes the key's first pk      */
/* bits, an entry equal to its predecessor all zeros.                         */
/* ------------------------------------------------------------------------- */

#define TREE_NODE 256
#define TREE_LEAF_FANOUT 14
#define TREE_INNER_FANOUT 9
#define TREE_MAX_LEVELS 32

static void put16(uint8_t *p, uint16_t v) { for (int b = 0; b < 2; ++b) p[b] = (uint8_t)(v >> (8 * b)); }
static void put32(uint8_t *p, uint32_t v) { for (int b = 0; b < 4; ++b) p[b] = (uint8_t)(v >> (8 * b)); }
static void put64(uint8_t *p, uint64_t v) { for (int b = 0; b < 8; ++b) p[b] = (uint8_t)(v >> (8 * b)); }

/* Entries per node for a fill factor in (0, 1]. */
void oracle_tree_fill(double fill, uint32_t *leaf_per, uint32_t *inner_per)
{
    uint32_t a = (uint32_t)floor(TREE_LEAF_FANOUT * fill), b = (uint32_t)floor(TREE_INNER_FANOUT * fill);
    *leaf_per = a < 1 ? 1 : a;
    *inner_per = b < 2 ? 2 : b;
}

/* Nodes per level (leaves first); returns the height (0 for n == 0). */
uint32_t oracle_tree_shape(uint64_t n, double fill, uint64_t *level_nodes)
{
    uint32_t lp, ip, h = 0;
    oracle_tree_fill(fill, &lp, &ip);
    if (n == 0) return 0;
    uint64_t nodes = (n + lp - 1) / lp;
    level_nodes[h++] = nodes;
    while (nodes > 1) {
        nodes = (nodes + ip - 1) / ip;
        level_nodes[h++] = nodes;
    }
    return h;
}

static uint16_t entry_dpos(const keyset *k, int first, uint64_t prev_row, uint64_t row)
{
    if (first) return 0xFFFF;
    int64_t d = key_dbit(k, prev_row, row);
    return d < 0 ? 0xFFFE : (uint16_t)d;
}

static uint32_t partial_key(const keyset *k, uint64_t row, uint16_t dpos, uint32_t pk)
{
    if (dpos == 0xFFFE) return 0;
    uint32_t start = dpos == 0xFFFF ? 0 : (uint32_t)dpos + 1, v = 0;
    for (uint32_t t = 0; t < pk; ++t) {
        uint32_t p = start + t;
        if (p < 8 * k->L && key_bit(k, row, p)) v |= 1u << (31 - t);
    }
    return v;
}

static uint16_t key_length(const keyset *k, uint64_t row)
{
    uint32_t len;
    key_ptr(k, row, &len);
    return (uint16_t)(len < k->L ? len : k->L);
}

/* nodes: (sum of level_nodes) * 256 bytes, written completely. */
int oracle_bulk_load(const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                     uint32_t L, uint32_t stride, const uint32_t *perm, uint32_t pk,
                     double fill, uint8_t *nodes)
{
    keyset k = {bytes, offsets, n, L, stride};
    uint64_t level_nodes[TREE_MAX_LEVELS], first[TREE_MAX_LEVELS], span[TREE_MAX_LEVELS];
    uint32_t lp, ip, h = oracle_tree_shape(n, fill, level_nodes);
    oracle_tree_fill(fill, &lp, &ip);
    uint64_t total = 0;
    for (uint32_t l = 0; l < h; ++l) {
        first[l] = total;
        total += level_nodes[l];
        span[l] = l == 0 ? lp : span[l - 1] * ip; /* keys under a full node of level l */
    }
    memset(nodes, 0, total * TREE_NODE);
    for (uint32_t l = 0; l < h; ++l) {
        for (uint64_t j = 0; j < level_nodes[l]; ++j) {
            uint8_t *nd = nodes + (first[l] + j) * TREE_NODE;
            uint64_t lo = j * span[l], hi = (j + 1) * span[l] < n ? (j + 1) * span[l] : n;
            uint64_t per = l == 0 ? lp : ip;
            uint64_t below = l == 0 ? n : level_nodes[l - 1];       /* entries of this level */
            uint64_t e0 = j * per, e1 = e0 + per < below ? e0 + per : below;
            put64(nd + 0, perm[hi - 1]);
            put16(nd + 8, (uint16_t)(e1 - e0));
            put16(nd + 10, (uint16_t)l);
            put64(nd + 16, lo);
            if (l == 0) put64(nd + 24, j + 1 < level_nodes[0] ? j + 1 : ~0ull);
            for (uint64_t e = e0; e < e1; ++e) {
                /* the entry's key: sorted position e (leaf) or the highest key of child e */
                uint64_t pos = l == 0 ? e : ((e + 1) * span[l - 1] < n ? (e + 1) * span[l - 1] : n) - 1;
                uint64_t ppos = 0;
                if (e > 0) ppos = l == 0 ? e - 1 : e * span[l - 1] - 1;
                uint64_t row = perm[pos];
                uint16_t dp = entry_dpos(&k, e == 0, e > 0 ? perm[ppos] : 0, row);
                uint8_t *en = l == 0 ? nd + 32 + (e - e0) * 16 : nd + 24 + (e - e0) * 24;
                put32(en + 0, partial_key(&k, row, dp, pk));
                put16(en + 4, dp);
                put16(en + 6, key_length(&k, row));
                if (l == 0) {
                    put64(en + 8, row);
                } else {
                    put64(en + 8, first[l - 1] + e);
                    put64(en + 16, row);
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* CDF model for learned bucketing (not in the paper; the model of the       */
/* learned bucketing extension).  fp64 reference of a 4 -> H -> 1 ReLU MLP.  */
/* Parameter vector p (length 6H + 1):                                        */
/*   W1[k][j] = p[4k + j] (k < H, j < 4), b1[k] = p[4H + k], w2[k] = p[5H + k],*/
/*   b2 = p[6H].                                                              */
/* Features of a 64-bit key prefix x: f_j = ((x >> (48 - 16 j)) & 0xFFFF)/65536. */
/* ------------------------------------------------------------------------- */

#define MLP_H 64
#define MLP_P (6 * MLP_H + 1)

static double mlp_forward_one(const double *p, const double *x, double *h)
{
    double y = p[6 * MLP_H];
    for (int k = 0; k < MLP_H; ++k) {
        double a = p[4 * MLP_H + k];
        for (int j = 0; j < 4; ++j) a += p[4 * k + j] * x[j];
        h[k] = a > 0 ? a : 0;
        y += p[5 * MLP_H + k] * h[k];
    }
    return y;
}

/* y[i] = MLP(X[i]) for M rows of 4 features. */
void oracle_mlp_forward(const double *p, const double *X, uint64_t M, double *y)
{
    double h[MLP_H];
    for (uint64_t i = 0; i < M; ++i) y[i] = mlp_forward_one(p, X + 4 * i, h);
}

/* Mean squared error over M rows and its gradient with respect to p. */
double oracle_mlp_loss_grad(const double *p, const double *X, const double *t, uint64_t M,
                            double *grad)
{
    double h[MLP_H], loss = 0;
    memset(grad, 0, sizeof(double) * MLP_P);
    for (uint64_t i = 0; i < M; ++i) {
        const double *x = X + 4 * i;
        double e = mlp_forward_one(p, x, h) - t[i];
        loss += e * e;
        double dy = 2.0 * e / (double)M;        /* d(mean e^2)/dy */
        grad[6 * MLP_H] += dy;                  /* b2 */
        for (int k = 0; k < MLP_H; ++k) {
            grad[5 * MLP_H + k] += dy * h[k];   /* w2 */
            if (h[k] > 0) {
                double g = dy * p[5 * MLP_H + k];
                grad[4 * MLP_H + k] += g;       /* b1 */
                for (int j = 0; j < 4; ++j) grad[4 * k + j] += g * x[j];
            }
        }
    }
    return loss / (double)M;
}

/* One Adam step (Kingma & Ba) on n parameters at step t (1-based). */
void oracle_adam(double *p, const double *g, double *m, double *v, uint32_t n, double lr,
                 double b1, double b2, double eps, uint32_t t)
{
    for (uint32_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1 - b1) * g[i];
        v[i] = b2 * v[i] + (1 - b2) * g[i] * g[i];
        double mh = m[i] / (1 - pow_u(b1, t));
        double vh = v[i] / (1 - pow_u(b2, t));
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Threshold table of the learned bucketing (the extension's definition of a
 * bucket): B thresholds cut a sorted training set of m first compressed words
 * into B rank ranges of (nearly) equal size.  T[0] = 0 so every 64-bit value
 * has a bucket; for b >= 1, T[b] = sorted[floor(b*m/B)], the word of rank
 * floor(b*m/B).  T is non-decreasing because sorted is. */
void oracle_thresholds(const uint64_t *sorted, uint64_t m, uint32_t B, uint64_t *T)
{
    for (uint32_t b = 0; b < B; ++b) {
        if (b == 0) { T[b] = 0; continue; }
        /* b*m < 2^16 * 2^32 here, so the product cannot overflow */
        uint64_t rank = ((uint64_t)b * m) / B;
        T[b] = sorted[rank];
    }
}

/* bucket[i] = the b with T[b] <= x[i] < T[b+1] (T[B] taken as +infinity),
 * for a non-decreasing threshold table T of B entries with T[0] = 0. */
void oracle_bucket(const uint64_t *x, uint64_t n, const uint64_t *T, uint32_t B, uint32_t *bucket)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t lo = 0, hi = B; /* invariant: T[lo] <= x < T[hi] */
        while (hi - lo > 1) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (T[mid] <= x[i]) lo = mid; else hi = mid;
        }
        bucket[i] = lo;
    }
}

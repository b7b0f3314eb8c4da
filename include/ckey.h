/*
 * ckey.h -- C ABI of libckey.so: compressed key sort on AMD MI355X (gfx950).
 *
 * Method: Kwon, Ryu, Cha, Lee, Park, Moon, "Compressed Key Sort and Fast Index
 * Reconstruction" (arXiv 2009.11543).
 *
 * Bit conventions (Sec. 3.1): a key is a string of key_bytes bytes read as a
 * bit string; position 0 is the most significant bit of byte 0, position p is
 * bit (7 - p%8) of byte p/8.  Variable-length keys are zero-padded to
 * key_bytes (Sec. 4.1: the varchar terminator and multi-column padding).
 * A D-bitmap is key_bytes bytes in the same bit order: bit p set means
 * "position p is (possibly) a distinction bit position" (Sec. 4.2).
 *
 * Compressed keys (Sec. 3.2): the key's bits at the bitmap's 1-positions in
 * ascending position order, packed most significant bit first into
 * w = ceil(nbits/64) 64-bit words (word 0 most significant; bits past nbits
 * are zero), stored word-major: ckeys[k*n + i] is word k of row i.
 *
 * Memory: every pointer marked "device" is device memory owned by the caller;
 * "host" pointers are read during the call only.  The library never allocates
 * or frees memory: calls that need scratch space take a caller workspace
 * (device, 256-byte aligned) sized by a query call with workspace == NULL,
 * which only writes *workspace_bytes and returns CKEY_OK.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Every call
 * validates its arguments on the host, returns a status synchronously and
 * enqueues its kernels asynchronously on `stream`; results are ready when the
 * stream is.  Conditions only the device can see are OR-ed into an optional
 * device uint32 `flags` word (CKEY_FLAG_*), which the caller clears.
 * Calls are reentrant; two calls that share a workspace must be ordered.
 */
#ifndef CKEY_H
#define CKEY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CKEY_OK = 0,
    CKEY_ERR_INVALID = 1,     /* null pointer, size out of range, bad bitmap   */
    CKEY_ERR_UNSUPPORTED = 2, /* valid request beyond this library's limits    */
    CKEY_ERR_WORKSPACE = 3,   /* *workspace_bytes smaller than required        */
    CKEY_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed    */
} ckey_status;

/* Device-side conditions, OR-ed into the caller's flags word. */
#define CKEY_FLAG_DESCENDING   0x1u /* ckey_distinction_bits: an adjacent pair descends     */
#define CKEY_FLAG_KEY_TOO_LONG 0x2u /* a variable-length key is longer than key_bytes       */
#define CKEY_FLAG_SPIN_LIMIT   0x4u /* a sort pass gave up waiting on a predecessor tile    */
#define CKEY_FLAG_BUCKET_OVERFLOW 0x8u /* bucketing sort: a bucket was finished by the radix sort */

/* Limits of this build. */
#define CKEY_MAX_KEY_BYTES 2048u          /* key_bytes                       */
#define CKEY_MAX_ROWS (1ull << 30)        /* n                               */
/* Limits of the one-launch table rebuild (ckey_sort_opts.fused_table). */
#define CKEY_TABLE_MAX_INDEXES 8u         /* indexes per call                 */
#define CKEY_TABLE_MAX_KEY_BYTES 64u      /* key_bytes of each index          */
#define CKEY_TABLE_MAX_PASSES 64u         /* radix passes of each index       */

/* A set of n keys in device memory.
 *   offsets == NULL: fixed width; key i occupies bytes[i*stride, i*stride+key_bytes).
 *   offsets != NULL: variable length; offsets is device uint64[n+1], key i is
 *                    bytes[offsets[i], offsets[i+1]) and must be <= key_bytes long
 *                    (longer keys set CKEY_FLAG_KEY_TOO_LONG); stride is ignored.
 * Row i's record ID is i (Sec. 5, step 2). */
typedef struct {
    const uint8_t *bytes;
    const uint64_t *offsets;
    uint64_t n;
    uint32_t key_bytes;
    uint32_t stride;
} ckey_keys;

/* Host-only planning of the extraction (Sec. 5.1 and Sec. 5.3).
 * bitmap: host, key_bytes bytes.  Writes nbits = |D| (popcount), words =
 * max(1, ceil(nbits/64)) and the number of Sec. 5.1 8-byte masks (each starts
 * at the byte holding the next 1 not covered by the previous mask).  If
 * window_start/window_mask are non-NULL, up to max_windows (start byte,
 * big-endian 64-bit mask) pairs are written.  Touches no GPU. */
ckey_status ckey_plan_query(const uint8_t *bitmap, uint32_t key_bytes, uint32_t *nbits,
                            uint32_t *words, uint32_t *windows, uint32_t *window_start,
                            uint64_t *window_mask, uint32_t max_windows);

/* Distinction bits of keys taken in sorted order (Sec. 3.1, Theorem 1):
 * bitmap (device, key_bytes bytes, overwritten) = union over adjacent pairs of
 * the most significant differing position.  order: device uint32[n] giving
 * the sorted order (row order[r] has rank r), or NULL when the rows are
 * already sorted.  Equal adjacent keys contribute nothing; a descending pair
 * sets CKEY_FLAG_DESCENDING.  n <= 1 gives an empty bitmap.  Needs a workspace. */
ckey_status ckey_distinction_bits(const ckey_keys *keys, const uint32_t *order, uint8_t *bitmap,
                                  uint32_t *flags, void *workspace, size_t *workspace_bytes,
                                  void *stream);

/* Compress every key with a D-bitmap (Sec. 3.2, Sec. 5.1).  bitmap: host,
 * key_bytes bytes, any superset of the keys' true distinction positions
 * (Theorem 2 covers supersets).  ckeys: device uint64[words*n], words >=
 * the plan's w (extra words are written as zero).  rowids: device uint32[n]
 * receiving 0..n-1, or NULL.  No workspace. */
ckey_status ckey_compress(const ckey_keys *keys, const uint8_t *bitmap, uint64_t *ckeys,
                          uint32_t words, uint32_t *rowids, uint32_t *flags, void *stream);

typedef enum {
    CKEY_SORT_RADIX = 0,   /* stable LSD radix sort over the top nbits                  */
    CKEY_SORT_LEARNED = 1, /* CDF-model bucketing + in-LDS bucket sorts (needs a model) */
    CKEY_SORT_SPLITTER = 2 /* the same bucketing with a binary search of the thresholds */
} ckey_sort_method;

typedef struct {
    uint32_t method;      /* ckey_sort_method                                          */
    uint32_t digit_bits;  /* radix digit width, 1..8; 0 = 8                           */
    uint32_t bucket_log2; /* learned/splitter: log2 of the model's bucket count, 8..16 */
    uint32_t skip_trivial; /* radix, ckey_sort / ckey_compress_sort only: 1 = read the
                            * digit histograms back (one stream synchronization) and
                            * skip every pass whose digit is equal for all rows; the
                            * index-rebuild entry points ignore it                   */
    const void *model;    /* learned/splitter: device model memory (ckey_cdf_*)        */
    uint32_t *flags;      /* device flags word or NULL                                 */
    uint32_t fused_table; /* ckey_rebuild_index / ckey_graph_create only (the call's
                           * opts): 1 = every index rebuilt by one persistent kernel
                           * launch (radix method; see ckey_rebuild_index)          */
    uint32_t tile;        /* rows a workgroup takes at once (an autotuning choice);
                           * 0 = chosen from the shape.  Radix, keys of 1..8 words:
                           * 1 = the full pass tile (1024 threads x 12, 10, 8, 6, 6,
                           * 5, 4, 4 rows for 1..8 words), 2 = half of it (512
                           * threads); wider keys have one tile.  Bucketing: the
                           * in-LDS capacity of a bucket, 1 = 2560 rows (512
                           * threads), 2 = 5120, 3 = 10240 (1024 threads); 0 picks
                           * by the mean bucket size (<= 1600, <= 4400, more)      */
} ckey_sort_opts;

/* Sort (compressed key, row id) pairs (Sec. 3.2 compressed key sort; Sec. 5,
 * step 3) in place: afterwards ckeys (device, word-major, words x n) are in
 * ascending order of their top nbits and rowids (device uint32[n]) moved with
 * them.  Ties go to the smaller row id, as in the paper's sort key (row id
 * inside the sort key): the radix method is stable (so this holds when the
 * row ids arrive ascending, as ckey_compress writes them); the bucketing
 * methods compare row ids explicitly.  opts may be NULL (radix, 8-bit
 * digits).  The bucketing methods synchronize `stream` once to learn whether
 * a bucket overflowed the in-LDS sort (5120 rows; 2560 when the mean bucket
 * holds at most 1600): such buckets are sorted again in LDS with a 10240-row
 * capacity (a second synchronization), and those still left (larger, or with
 * a run of more than 32 equal first words) are finished by the radix sort and
 * raise CKEY_FLAG_BUCKET_OVERFLOW; so does a widespread overflow (more than
 * 64 buckets or an eighth of the rows), which radix-sorts everything.  While
 * `stream` is being captured into a graph the same decisions are taken on the
 * device instead (see ckey_graph_create), with no synchronization.  Needs a
 * workspace. */
ckey_status ckey_sort(uint64_t *ckeys, uint32_t words, uint32_t nbits, uint32_t *rowids,
                      uint64_t n, const ckey_sort_opts *opts, void *workspace,
                      size_t *workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ckey_sort
 * with the radix method, its scratch space taken from one static device array
 * of CKEY_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of a caller workspace.  Arguments, results
 * and flags as for ckey_sort.  The call allocates no memory (no hipMalloc, no
 * host heap) and never synchronizes the stream; the scratch array's address
 * is looked up once per device, on the first call with that device current.
 * Returns CKEY_ERR_UNSUPPORTED for a bucketing method, skip_trivial, more
 * than 512 radix passes, or a sort whose workspace (ckey_sort's query with
 * the same arguments) exceeds CKEY_NOALLOC_SCRATCH_BYTES -- e.g. about
 * 5.5 million rows of one-word keys, 2.3 million of three words.  All calls on
 * one GPU share its array: calls that overlap on one GPU (different streams
 * without ordering) race and give wrong results. */
#define CKEY_NOALLOC_SCRATCH_BYTES (64u << 20)
ckey_status ckey_sort_noalloc(uint64_t *ckeys, uint32_t words, uint32_t nbits, uint32_t *rowids,
                              uint64_t n, const ckey_sort_opts *opts, void *stream);

/* Compress and sort in one call (Sec. 5 steps 2-3: extract the compressed
 * keys, sort the (compressed key, row id) pairs): ckeys (device, words x n)
 * and rowids (device uint32[n]) receive the sorted compressed keys and the row
 * ids in full-key order.  Arguments as for ckey_compress and ckey_sort.  With
 * a bucketing method the record IDs are generated by the first grouping pass
 * instead of being written and read back; with fixed-width keys each key's
 * bucket is found while the key is compressed for the learned method, and for
 * the splitter beyond 2^14 buckets.
 * Needs a workspace (the size ckey_sort needs). */
ckey_status ckey_compress_sort(const ckey_keys *keys, const uint8_t *bitmap, uint64_t *ckeys,
                               uint32_t words, uint32_t *rowids, const ckey_sort_opts *opts,
                               void *workspace, size_t *workspace_bytes, void *stream);

/* One index to rebuild (Sec. 5 steps 2-3 and the DS-metadata refresh of Sec. 4.3). */
typedef struct {
    ckey_keys keys;
    const uint8_t *bitmap_in; /* host, key_bytes bytes: current D-bitmap (any superset
                                 of the true D); NULL = first build over full keys     */
    uint32_t *perm;           /* device uint32[n] out: row ids in full-key order        */
    uint8_t *bitmap_out;      /* device key_bytes bytes out: the refreshed D-bitmap, or NULL */
    uint32_t *pair_pos;       /* device uint32[n-1] out or NULL: full-key D position of
                                 each adjacent sorted pair (Sec. 5.3 D-offset lookup),
                                 0xFFFFFFFF where the keys are equal                   */
    uint64_t *ckeys;          /* device uint64[w*n] out or NULL: the sorted compressed keys */
    uint32_t *flags;          /* device flags word or NULL                              */
    const ckey_sort_opts *opts; /* sort options of this index, or NULL for the call's  */
} ckey_index_desc;

/* Rebuild `count` indexes of a table: compress each with its bitmap, sort, and
 * refresh its D-bitmap from adjacent sorted compressed keys (Sec. 4.3, Sec. 5).
 * opts as for ckey_sort (NULL = radix), per index overridable.  With count > 1
 * each index gets its own part of the workspace and its own stream forked from
 * `stream` (and joined back), so the indexes' kernels overlap.  Needs a
 * workspace.
 *
 * opts->fused_table = 1: the whole table in one persistent kernel launch (after
 * one fill kernel that clears its counters), whose workgroups take work items
 * from a queue -- per index: compress tiles, a histogram scan, the tiles of each
 * radix pass, refresh tiles -- each waiting on the items it depends on.  Every
 * index must use the radix method (per-index digit_bits allowed); at most
 * CKEY_TABLE_MAX_INDEXES indexes of at most CKEY_TABLE_MAX_KEY_BYTES key bytes,
 * n < 2^30 and at most CKEY_TABLE_MAX_PASSES passes each, else
 * CKEY_ERR_UNSUPPORTED.  The workspace layout differs from the forked form
 * (query with the same opts).  A wait that exceeds its spin bound raises
 * CKEY_FLAG_SPIN_LIMIT in that index's flags word (the results are then not
 * valid).  In this build the one-launch form is switched off: workspace
 * queries and argument checks work, a real call (and ckey_graph_create)
 * returns CKEY_ERR_UNSUPPORTED. */
ckey_status ckey_rebuild_index(const ckey_index_desc *idx, uint32_t count,
                               const ckey_sort_opts *opts, void *workspace,
                               size_t *workspace_bytes, void *stream);

/* A table rebuild captured once into a HIP graph and replayed with one launch.
 * ckey_graph_create records what ckey_rebuild_index(idx, count, opts, ...)
 * enqueues (the descriptors' pointers, bitmaps, sizes and models are fixed at
 * creation; the workspace must stay valid while the graph exists) and
 * instantiates it.  Every sort method can be captured: a captured bucketing
 * sort never asks the host about overflowing buckets -- one kernel walks the
 * overflow list on the device (more than 64 overflowing buckets skip it), and
 * a radix sort of the whole index, whose kernels are always in the graph and
 * return at once unless a device word opens them, finishes any bucket still
 * unsorted (raising CKEY_FLAG_BUCKET_OVERFLOW).  With opts->fused_table the
 * graph holds the fill kernel and the one persistent launch.
 * ckey_graph_launch replays it on `stream`. */
typedef struct ckey_graph ckey_graph;
ckey_status ckey_graph_create(const ckey_index_desc *idx, uint32_t count, const ckey_sort_opts *opts,
                              void *workspace, size_t workspace_bytes, ckey_graph **graph);
ckey_status ckey_graph_launch(ckey_graph *graph, void *stream);
ckey_status ckey_graph_destroy(ckey_graph *graph);

/* Autotuning: rebuild index `idx` once per candidate option set (after one
 * warm-up each) timing it with HIP events on `stream`; *best receives the
 * index of the fastest candidate and times_ms (host float[ncand], or NULL)
 * each candidate's time.  Synchronizes `stream`.  The workspace must fit every
 * candidate (ckey_rebuild_index's query with each). */
ckey_status ckey_tune_index(const ckey_index_desc *idx, const ckey_sort_opts *candidates,
                            uint32_t ncand, void *workspace, size_t workspace_bytes,
                            void *stream, uint32_t *best, float *times_ms);

/* ---- DS-metadata maintenance (Sec. 4.3) --------------------------------------
 * The DS-metadata of an index: the D-bitmap, the variant bitmap (1 where the
 * keys may differ) and a reference key (any key of the index).  */

/* Variant bitmap (Sec. 4.3, rebuild step 3): variant (device, key_bytes bytes,
 * overwritten) = OR over all keys K of (K xor reference), keys zero-padded to
 * key_bytes.  ref: device, key_bytes bytes, or NULL to take key 0 as the
 * reference (an arbitrary index key, as the paper allows); ref_out (device,
 * key_bytes bytes, or NULL) receives the reference used.  Every D position is
 * a variant position, so the result is a superset of D that needs no sort: it
 * can stand in for the all-ones bitmap of a first build.  n == 0 gives an
 * all-zero bitmap.  Workspace: ceil(key_bytes/4) words (query with
 * workspace == NULL). */
ckey_status ckey_variant_bitmap(const ckey_keys *keys, const uint8_t *ref, uint8_t *variant,
                                uint8_t *ref_out, uint32_t *flags, void *workspace,
                                size_t *workspace_bytes, void *stream);

/* Batched insert (Sec. 4.3, insert): the DS-metadata update for inserting
 * every key of `batch` into the index `index`.  index_order (device
 * uint32[index->n]) lists the index rows in key order (as ckey_rebuild_index's
 * perm does); NULL: the rows are stored in key order.  batch_order likewise
 * for the batch; NULL: the library sorts the batch itself (full-key radix sort
 * in the workspace, which then grows with the batch and its key width).
 * Both key sets must have the same key_bytes.  For each inserted key K that
 * lands between A and B the paper sets max(D-bit(A,K), D-bit(K,B)) (the
 * smaller is D-bit(A,B), already set, Lemma 1); for the whole batch this is
 * every D-bit of an adjacent pair of the merged order that holds a batch key,
 * OR-ed into dbitmap (device, key_bytes bytes, updated in place).  The result
 * equals inserting the keys one by one, in any sequence, provided dbitmap
 * covered the index's D before the call (always true of DS-metadata).  If
 * variant (device, key_bytes bytes) is not NULL, (K xor ref) is OR-ed into it
 * for every batch key; ref (device, key_bytes bytes) is then required.
 * Deletes leave the DS-metadata unchanged (Sec. 4.3), so there is no delete
 * call: the kept bitmaps stay valid supersets, and the next rebuild
 * (ckey_rebuild_index) drops the stale bits. */
ckey_status ckey_insert_keys(const ckey_keys *index, const uint32_t *index_order,
                             const ckey_keys *batch, const uint32_t *batch_order,
                             uint8_t *dbitmap, uint8_t *variant, const uint8_t *ref,
                             uint32_t *flags, void *workspace, size_t *workspace_bytes,
                             void *stream);

/* ---- Index tree bulk load (Sec. 5.3, index construction) ---------------------
 * The sorted output of a rebuild filled bottom-up into the paper's index tree:
 * 256-byte nodes with a 24-byte header; leaves hold up to 14 entries of 16
 * bytes (after an 8-byte next pointer), inner nodes up to 9 entries of 24
 * bytes.  A full node holds floor(fanout * fill) entries (at least 1 in a
 * leaf, 2 in an inner node); the last node of a level holds the rest.  Levels
 * are stored leaves first, each in key order, so node indexes are positions
 * in the caller's node array.  Layout (little-endian, unused bytes zero):
 *   header: record ID of the node's highest key u64 @0, entry count u16 @8,
 *           level u16 @10 (0 = leaf), zero u32 @12, sorted position of the
 *           node's first key u64 @16
 *   leaf:   next leaf's node index u64 @24 (all ones for the last leaf),
 *           entries @32: partial key u32, D position u16, key length u16,
 *           record ID u64
 *   inner:  entries @24: partial key u32, D position u16, key length u16,
 *           child node index u64, record ID of the child's highest key u64
 * An entry's D position is that of its key against the previous entry's key
 * on the same level (CKEY_DPOS_FIRST for a level's first entry,
 * CKEY_DPOS_EQUAL for a key equal to the previous one); its partial key
 * (Sec. 4.2) is the pk bits after that position, MSB-first, left-aligned in
 * 32 bits (the first entry: the key's first pk bits; an equal key: 0). */
#define CKEY_TREE_NODE_BYTES 256u
#define CKEY_TREE_LEAF_FANOUT 14u
#define CKEY_TREE_INNER_FANOUT 9u
#define CKEY_TREE_MAX_LEVELS 32u
#define CKEY_DPOS_FIRST 0xFFFFu
#define CKEY_DPOS_EQUAL 0xFFFEu

typedef struct {
    uint32_t height;          /* levels, leaves included (0 for n == 0)        */
    uint32_t leaf_entries;    /* entries of a full leaf                        */
    uint32_t inner_entries;   /* entries of a full inner node                  */
    uint32_t reserved;
    uint64_t level_nodes[CKEY_TREE_MAX_LEVELS]; /* nodes per level, leaves first */
    uint64_t level_first[CKEY_TREE_MAX_LEVELS]; /* index of each level's first node */
    uint64_t total_nodes;     /* the node array holds total_nodes * 256 bytes  */
} ckey_tree_shape;

/* Host only: the tree's shape for n keys and a fill factor in (0, 1]. */
ckey_status ckey_tree_plan(uint64_t n, float fill, ckey_tree_shape *shape);

typedef struct {
    ckey_keys keys;           /* the index's keys (lengths; bits read by record ID) */
    const uint32_t *perm;     /* device uint32[n]: rows in key order               */
    const uint64_t *ckeys;    /* device uint64[words*n]: the sorted compressed keys */
    uint32_t words;
    const uint8_t *cbitmap;   /* host, key_bytes: the bitmap ckeys were made with   */
    const uint32_t *pair_pos; /* device uint32[n-1]: the rebuild's per-pair D positions */
    const uint8_t *variant;   /* host, key_bytes, or NULL                           */
    const uint8_t *ref;       /* device, key_bytes: reference key (with variant)    */
} ckey_tree_input;

/* Build the tree into `nodes` (device, shape.total_nodes * 256 bytes) from a
 * rebuild's outputs: perm, the sorted compressed keys and pair_pos of
 * ckey_rebuild_index (made with cbitmap).  Each partial-key bit is taken as
 * Sec. 5.3 lists: from the compressed key when cbitmap has its position, from
 * the reference key when the variant bitmap has 0 there, else from the key
 * itself by record ID (option b).  Without a variant bitmap every position
 * outside cbitmap is read from the key.  deref (device uint64, or NULL) is
 * increased by the number of entries that read their key.  pk_bits: 1..32.
 * Leaf D positions come from pair_pos; inner ones from the level below
 * (Lemma 1).  Workspace: 4 * key_bytes (query with workspace == NULL). */
ckey_status ckey_bulk_load(const ckey_tree_input *in, uint32_t pk_bits, float fill, void *nodes,
                           uint64_t *deref, void *workspace, size_t *workspace_bytes, void *stream);

/* ---- CDF model for learned bucketing (an extension; not in the paper) -------
 * Model memory is device memory owned by the caller, ckey_cdf_model_bytes()
 * long, 256-byte aligned: a 4 -> 64 -> 1 ReLU MLP (385 fp32 parameters, plus
 * Adam moments) and a table T of 2^bucket_log2 sorted 64-bit thresholds.
 * Layout: the parameters as float[385] at byte 0 (ckey_cdf_grad's order),
 * Adam's first and second moments as float[385] at bytes 2048 and 4096, T as
 * uint64[2^bucket_log2] at byte 8192; a caller may write the parameters
 * (zeroing the moments) in place of ckey_cdf_model_init.
 * bucket(x) = the b with T[b] <= x < T[b+1] for the key's first compressed
 * word x; it is non-decreasing in key order.  The network predicts b from x's
 * four 16-bit chunks (each / 65536); a search of T from the prediction makes
 * it exact, so results never depend on the network: the sort searches the
 * 2^10 buckets around the guess at a fixed depth (all of T when the key lies
 * outside them), ckey_cdf_bucket with statistics searches exponentially
 * outward from the guess, then by bisection. */
size_t ckey_cdf_model_bytes(uint32_t bucket_log2);

/* Initialise the parameters deterministically from `seed`, zero the moments. */
ckey_status ckey_cdf_model_init(void *model, uint32_t bucket_log2, uint64_t seed, void *stream);

typedef struct {
    uint32_t steps;   /* Adam steps                                  */
    uint32_t batch;   /* samples per step, 1..2^20                   */
    float lr, beta1, beta2, eps;
    uint64_t seed;    /* minibatch sampling: sample j of step s is row
                         SplitMix64(seed + phi*((s << 32) + j + 1)) mod m */
} ckey_cdf_train_opts;

/* Fit a model to the sorted first compressed words of a training set
 * (device uint64[m], ascending): T[b] = sorted_prefix[b*m / 2^bucket_log2]
 * (T[0] = 0), then `steps` Adam steps on the mean squared error between the
 * network output and the normalised rank (r + 0.5)/m of sampled rows.
 * loss_trace: device float[steps] (or NULL) receives each step's loss.
 * Needs a workspace. */
ckey_status ckey_cdf_fit(void *model, uint32_t bucket_log2, const uint64_t *sorted_prefix,
                         uint64_t m, const ckey_cdf_train_opts *opts, float *loss_trace,
                         void *workspace, size_t *workspace_bytes, void *stream);

/* Loss and gradient of the network on an explicit batch: prefix (device
 * uint64[m]) and target (device float[m]); grad: device float[385] in the
 * parameter order W1[k][j] (k<64, j<4), b1[k], w2[k], b2; loss: device
 * float.  Reductions run in a fixed order (deterministic).  Needs a workspace. */
ckey_status ckey_cdf_grad(const void *model, const uint64_t *prefix, const float *target,
                          uint64_t m, float *grad, float *loss, void *workspace,
                          size_t *workspace_bytes, void *stream);

/* Exact bucket of n prefixes (device uint64[n]) into bucket (device
 * uint32[n]) with method CKEY_SORT_LEARNED or CKEY_SORT_SPLITTER; predicted
 * (device uint32[n] or NULL, learned only) gets the network's raw guess;
 * stats (device uint64[2] or NULL, accumulated) gets the number of threshold
 * probes after the first guess (learned: the exact search from the network's
 * guess, in LDS up to 2^14 buckets, else in global memory; splitter: the
 * global search below its LDS sample, none up to 2^14 buckets, where every
 * threshold is in LDS) and the summed |bucket - guess|. */
ckey_status ckey_cdf_bucket(const void *model, uint32_t bucket_log2, uint32_t method,
                            const uint64_t *prefix, uint64_t n, uint32_t *bucket,
                            uint32_t *predicted, uint64_t *stats, void *stream);

/* ---- Benchmark support (not part of the method) ---------------------------
 * Per-kernel timing: while enabled, every launch of the library's main kernels
 * ("compress", "hist", "onesweep", "refine", "dbits", "stream_copy") is
 * bracketed by HIP events on its stream.  ckey_profile_read waits for the
 * recorded events and returns the summed duration and launch count of the
 * kernels named `name` (NULL: all); ckey_profile_reset drops the records. */
ckey_status ckey_profile_enable(int on);
ckey_status ckey_profile_read(const char *name, double *total_ms, uint64_t *launches);
ckey_status ckey_profile_reset(void);

/* A plain device-to-device copy kernel ("stream_copy") of `bytes` bytes
 * (multiple of 16, 16-byte aligned device pointers): measures achievable HBM
 * bandwidth and calibrates hardware byte counters. */
ckey_status ckey_bench_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Human-readable status name. */
const char *ckey_status_string(ckey_status s);

#ifdef __cplusplus
}
#endif

#endif /* CKEY_H */

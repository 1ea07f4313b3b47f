/*
 * pfac.h -- C ABI of the MI355X (gfx950) PFAC DNA matcher.
 *
 * PFAC (Parallel Failure-less Aho-Corasick, paper Sec. IV): every start
 * position of a DNA text runs its own walk through the goto trie of the
 * patterns, with no failure links, stops at the first missing transition,
 * and reports the longest pattern it passed (only the longest: sub-patterns
 * of a longer match at the same start are not reported, Sec. IV).  The
 * transition table has four columns, one per base (Sec. V.A, Table I), and
 * is built on the host by inserting the patterns one at a time (Sec. V.A);
 * matching runs on the GPU (Sec. V.B).
 *
 * Conventions shared by every entry point
 *   - Bases are the upper-case ASCII bytes 'A','C','G','T'.  Any other text
 *     byte has no transition, so a walk that reaches it stops there.
 *   - Pattern IDs are 1 + the pattern's index in the input array (Table I
 *     numbers its three patterns 1, 2, 3 in input order); 0 means "no match".
 *     When several identical patterns are given, the smallest ID is reported
 *     and every copy is counted in the occurrence totals.
 *   - Text encodings: PFAC_TEXT_ASCII, one byte per base; PFAC_TEXT_2BIT,
 *     A=0 C=1 G=2 T=3, base 4k+j in bits 2j..2j+1 of byte k (every value is
 *     a valid base).
 *   - Every function returns a pfac_status (0 on success) and never throws
 *     or aborts.  Device pointers are hipMalloc'ed memory of the device that
 *     is current on the calling thread; the caller owns them.  `stream` is a
 *     hipStream_t (NULL = the legacy default stream).  Match calls are
 *     asynchronous with respect to the host: they only enqueue work on
 *     `stream`; results are valid once the stream reaches that point.
 *   - Argument errors are reported synchronously before anything is
 *     enqueued; on error no output buffer is written.
 */
#ifndef PFAC_H
#define PFAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFAC_OK = 0,
  PFAC_E_ARG = -1,        /* null/invalid argument, size out of range, wrong device */
  PFAC_E_PATTERN = -2,    /* empty pattern or pattern byte outside A,C,G,T */
  PFAC_E_TOO_LARGE = -3,  /* trie would need 2^31 or more states */
  PFAC_E_NOMEM = -4,      /* host or device allocation failed */
  PFAC_E_HIP = -5,        /* a HIP runtime call failed */
  PFAC_E_NODEV = -6,      /* no usable gfx950 device */
  PFAC_E_SCRATCH = -7     /* the input needs more scratch than a fixed-size scratch
                             area holds */
} pfac_status;

enum { PFAC_TEXT_ASCII = 0, PFAC_TEXT_2BIT = 1 };

/* Opaque trie.  Immutable after pfac_build_table; it owns its device memory
 * and may be used concurrently from several streams and host threads. */
typedef struct pfac_table pfac_table;

/* One reported start position: pos = start index in the text, pid = the
 * longest pattern starting there (never 0). */
typedef struct {
  uint32_t pos;
  int32_t pid;
} pfac_hit;

/* One reported start position of a batched call (text = index in the
 * descriptor array). */
typedef struct {
  uint32_t text;
  uint32_t pos;
  int32_t pid;
} pfac_batch_hit;

typedef struct {
  uint64_t num_states;     /* trie states including the root */
  uint32_t num_patterns;
  uint32_t max_len;        /* longest pattern */
  uint32_t min_len;        /* shortest pattern */
  uint32_t max_depth_full; /* deepest level d at which all 4^d prefixes are trie states */
  uint64_t device_bytes;   /* device memory owned by the table */
  uint64_t states_to_depth[9]; /* states of depth <= d, d = 0..8 (BFS prefix sizes) */
  uint32_t prefix_k;       /* K2 of the prefix filter, 0 when the table has none */
  uint32_t reserved;
  uint64_t prefix_keys;    /* distinct K2-base pattern prefixes */
} pfac_table_stats;

/* Launch shape of a match call.  Any field left 0 is chosen by the library.
 * Results never depend on the plan: every plan computes the same walks. */
typedef struct {
  uint32_t block;       /* threads per workgroup: 256, 512, 768 or 1024 */
  uint32_t depth;       /* filter depth D, 6..10: every position first looks up its
                           D-base window in an LDS bitmap of 4^D bits; only windows
                           whose walk continues past depth D (or passes a final state
                           within D bases) go on to the global-memory trie */
  uint32_t grid;        /* persistent workgroups (0 = fill the device; at most 2048) */
  uint32_t variant;     /* PFAC_VARIANT_TILED (LDS text tile + filter bitmap) or one
                           of the global-memory variants below (every walk from the
                           root, text and table read straight from global memory) */
  uint32_t levels;      /* when every pattern is longer than D: trie levels from
                           depth D down kept in LDS, found by rank from the filter
                           bit (0 = as many as fit, possibly none); the walk goes on
                           in the global next-state table below them.
                           PFAC_LEVELS_NONE = filter bitmap only: surviving windows
                           read the global depth-D jump table (always the case when
                           some pattern has D bases or fewer) */
  uint32_t hash_bits;   /* second filter for the positions that pass the first one,
                           used when every pattern has more than D bases: their first
                           K = min(shortest pattern, 16) bases hashed twice into an
                           LDS bitmap of 2^hash_bits bits (12..20); only windows whose
                           two bits are set walk on (for K <= 12 and sets that let
                           more than 30 % of windows through the depth-D filter:
                           hashed once, see pfac_build_host_hash1).  0 = library
                           choice, PFAC_HASH_NONE = no second filter */
  uint32_t walks;       /* where the walks that pass the filters run:
                           PFAC_WALKS_INLINE = by the wave that found them, with the
                           tile; PFAC_WALKS_DEFERRED = the wave keeps each one (start
                           position + its next 64 bases; room for a number per tile
                           the library sizes from the filters' pass rates, more walk
                           inline) and walks them all after its last tile, so the
                           streaming scan does not wait on their table reads.
                           0 = library choice (deferred when a second or prefix
                           filter is on and no pattern is longer than 64 bases). */
  uint32_t tile;        /* start positions per wave tile: 1024 or 2048 (one-text and
                           batched calls), 256 (batched calls only).  0 = library
                           choice: 2048 for one text; in a batch 256 for texts of at
                           most 512 bases and 2048 for longer ones, except that
                           fewer than 4096 short texts of a table that also has
                           longer ones get 2048 with them (an explicit value
                           applies to every text of the batch) */
  uint32_t prefix;      /* prefix filter, used when every pattern is longer than D:
                           windows that pass the LDS filters are looked up in an exact
                           bitmap of the patterns' first K2 bases held in global
                           memory (4^K2 bits; K2 = min(shortest pattern, 12) > D), and
                           only those whose K2-base prefix starts some pattern walk on.
                           0 = library choice (on when the hashed second filter is
                           off and K2 > D), PFAC_PREFIX_NONE = off, 1 = on */
  uint32_t pair;        /* the depth-D filter as a pair table (D <= 9, no LDS trie
                           levels): one byte per string m of D-1 bases holds the filter
                           bits of the windows that start one base before m and at m,
                           so one LDS read tests two neighbouring positions; it takes
                           twice the LDS of the bitmap.  0 = library choice (on when it
                           fits), 1 = on, PFAC_PAIR_NONE = off */
} pfac_plan;

enum { PFAC_WALKS_INLINE = 1, PFAC_WALKS_DEFERRED = 2 };
#define PFAC_PREFIX_NONE 0xFFFFFFFFu
#define PFAC_PAIR_NONE 0xFFFFFFFFu

/* Variants.  TILED: text tile in LDS, filters, deep walks (the library's).
 * GLOBAL: the paper's kernel (Sec. V.B): every position walks from the root,
 * text and table read from global memory; the table as edge words with a
 * final bit and per-state pattern IDs.  The two other global-memory variants
 * use the paper's own table layouts (Sec. VII): GLOBAL_TWO_ARRAYS reads the
 * next state and the matched pattern ID of each cell from two S x 4 arrays,
 * GLOBAL_MERGED from one array of {next state, pattern ID} cells; their
 * arrays are built on the device from the table the first time a call asks
 * for them (one-text calls only). */
enum {
  PFAC_VARIANT_TILED = 0,
  PFAC_VARIANT_GLOBAL = 1,
  PFAC_VARIANT_GLOBAL_TWO_ARRAYS = 2,
  PFAC_VARIANT_GLOBAL_MERGED = 3
};
#define PFAC_LEVELS_NONE 0xFFFFFFFFu
#define PFAC_HASH_NONE 0xFFFFFFFFu

/* Per-text descriptor of a batched call (all offsets are from the bases the
 * call passes).  A text of ASCII encoding starting at a 16-byte aligned
 * address is read with 16-byte loads; any other start is read byte-wise. */
typedef struct {
  uint64_t text_offset;   /* byte offset of the text in d_text_base */
  uint64_t n;             /* bases (< 2^32) */
  uint64_t match_offset;  /* element offset of its match array in d_match_base */
  uint32_t table;         /* index into the tables[] array of the call */
  uint32_t enc;           /* PFAC_TEXT_ASCII or PFAC_TEXT_2BIT */
} pfac_text_desc;

/*
 * Build the failure-less goto trie of `num` patterns (Sec. V.A: patterns
 * inserted one at a time, a new state per new character; Sec. V.B: the
 * table is then copied to the device).  States are renumbered in
 * breadth-first order (the state order of Nishimura et al., Sec. II) so that
 * shallow, frequently visited states form a contiguous prefix.
 *   patterns[k]  pointer to lengths[k] bytes (not NUL-terminated), host memory
 *   num          >= 1
 *   out          receives the table; free it with pfac_free_table
 *   bad_index    optional; receives the index of the first invalid pattern on
 *                PFAC_E_PATTERN, -1 otherwise
 * Synchronous.  The table lives on the device current at the call.
 */
int pfac_build_table(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     pfac_table** out, int64_t* bad_index);

/*
 * Build a table over the byte alphabet: every byte value 0..255 is a symbol
 * and patterns are any non-empty byte strings (case, IUPAC codes, N, or
 * non-DNA data) -- the general-purpose setting of the original PFAC library
 * (Sec. I, II).  Same insertion and numbering as pfac_build_table; the
 * transition table is hash-compressed (the hash method Sec. II names): the
 * root's 256 edges form a dense row, every other edge is an entry of one
 * open-addressing hash table keyed by (state, byte), load at most 1/2.
 * Such a table works with pfac_match only (texts PFAC_TEXT_ASCII, read as
 * raw bytes; no byte stops a walk except where no edge exists; plans may set
 * the grid only, and block 1024); the other match calls return PFAC_E_ARG.
 * At most 2^24 - 1 states (PFAC_E_TOO_LARGE beyond); PFAC_E_PATTERN for an
 * empty pattern.
 */
int pfac_build_table_bytes(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                           pfac_table** out, int64_t* bad_index);

/*
 * The same table as pfac_build_table, built on the device (the host only
 * checks and packs the patterns; the trie, its breadth-first numbering and
 * every derived array are computed by kernels): with the patterns sorted as
 * strings, the states of depth d are their distinct d-base prefixes in
 * breadth-first order, so a scan per depth numbers them.  `ids` (or NULL for
 * 1..num) gives each pattern's ID (> 0; the smallest ID among equal patterns
 * is reported).  Patterns of at most 64 bases (PFAC_E_ARG beyond, with
 * *bad_index set).  Synchronous; uses temporary device memory.
 */
int pfac_build_table_device(const char* const* patterns, const uint32_t* lengths,
                            const int32_t* ids, uint32_t num, pfac_table** out,
                            int64_t* bad_index);

/*
 * A new table: the patterns of `base` (each keeps its ID) except those whose
 * ID is in remove_ids, plus `add` (new IDs from one above the largest ID of
 * base, in order; *first_new_id receives the first, may be NULL), built on
 * the device as pfac_build_table_device.  `base` is unchanged and stays
 * usable (a server swaps tables when the new one is ready).  IDs are not
 * renumbered, so removed IDs leave gaps.  Tables from pfac_build_table and
 * pfac_build_table_device keep their pattern sets for this; byte tables are
 * not updated (PFAC_E_ARG).
 */
int pfac_table_update(const pfac_table* base, const char* const* add, const uint32_t* add_lens,
                      uint32_t num_add, const int32_t* remove_ids, uint32_t num_remove,
                      pfac_table** out, int32_t* first_new_id);

/* Copy the table's whole device allocation (every array, at the offsets
 * both builds share; gaps are zero) to host memory: *bytes receives its
 * size, `host` (cap bytes) is written when large enough.  For tests. */
int pfac_table_blob(const pfac_table* table, void* host, uint64_t cap, uint64_t* bytes);

int pfac_table_info(const pfac_table* table, pfac_table_stats* out);

/* Frees host and device memory (synchronises the device first).  NULL is a no-op. */
void pfac_free_table(pfac_table* table);

/*
 * Match one text (Sec. IV semantics; one walk per start position, Sec. V.B).
 *   d_text      device text of n bases in encoding `enc` (n < 2^32; n = 0 is allowed)
 *   d_match     device int32[n] or NULL: longest pattern ID per start position, 0 = none
 *   d_hits      device pfac_hit[hit_cap] or NULL: the positions with match != 0, in
 *               ascending position order; only the first hit_cap are written
 *   d_counters  device uint64[2] (required): [0] = number of positions with a match
 *               (may exceed hit_cap: the caller can retry with a larger buffer),
 *               [1] = total (pattern, position) occurrences, every pattern ID counted
 *   plan        NULL for the library's choice
 * Scratch memory (per-tile hit counts, occurrence counts and hit slots, the
 * finish kernel's look-back words, the buffer of deferred walks) is owned by
 * the library, one area per (device, stream); calls on one stream reuse it in
 * order, calls on different streams may overlap.  A call on a larger text
 * than any before on its stream grows the area (hipMalloc, synchronous), so
 * pfac_match is not meant for graph capture; prepared batches are.
 */
int pfac_match(const pfac_table* table, const void* d_text, uint64_t n, int enc,
               int32_t* d_match, pfac_hit* d_hits, uint64_t hit_cap, uint64_t* d_counters,
               const pfac_plan* plan, void* stream);

/*
 * pfac_match for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it).  Same arguments, kernels and results as pfac_match; the
 * scratch (per-tile counts and hit slots, look-back words, deferred walks)
 * lives in a fixed device array inside the library, pfac_noalloc_scratch_bytes()
 * bytes (64 MiB) per GPU, held from the library's load until the process
 * ends.  The call allocates nothing, copies nothing from the host and issues
 * no memset: it enqueues a small fill kernel that clears the array's
 * look-back words, then the scan and finish kernels.
 *   Returns PFAC_E_SCRATCH, before anything is enqueued, when the text needs
 *   more scratch than the array holds: 268 bytes per tile of 2048 positions
 *   plus 32 bytes per deferred-walk entry plus 2 MiB, so between about 100 Mbase (plans
 *   that defer many walks) and 500 Mbase (walks at once); pfac_match has no
 *   such limit.  PFAC_E_ARG for
 *   byte-alphabet tables and for the paper's two-array and merged-cell
 *   layouts before pfac_match has built them.
 * Every call on one GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (two streams, two host threads) race and give wrong
 * results; the caller serialises them.
 */
int pfac_match_noalloc(const pfac_table* table, const void* d_text, uint64_t n, int enc,
                       int32_t* d_match, pfac_hit* d_hits, uint64_t hit_cap,
                       uint64_t* d_counters, const pfac_plan* plan, void* stream);

/* Size in bytes of the fixed scratch array of pfac_match_noalloc. */
uint64_t pfac_noalloc_scratch_bytes(void);

/*
 * Every occurrence of every pattern in one text: all pairs (start position,
 * pattern ID) with the pattern starting there, including the shorter
 * patterns PFAC's own report leaves out at a position where a longer one
 * matches (the limitation Sec. IV names), and every ID of duplicate
 * patterns.  Computed as a count pass (the scan of pfac_match, which sums
 * the occurrences of each tile), a scan of the per-tile counts, and a write
 * pass that walks again at the positions with a match.
 *   d_occ       device pfac_hit[occ_cap] or NULL: the pairs in ascending
 *               position, then ascending pattern length, then ascending ID;
 *               only the first occ_cap are written
 *   d_counters  device uint64[2] (required): [0] = positions with a match,
 *               [1] = total occurrences (the full list length, may exceed
 *               occ_cap: the caller can retry with a larger buffer)
 *   plan        NULL for the library's choice (as pfac_match)
 * Asynchronous on `stream`; scratch as in pfac_match, plus 32 bytes per tile.
 */
int pfac_match_all(const pfac_table* table, const void* d_text, uint64_t n, int enc,
                   pfac_hit* d_occ, uint64_t occ_cap, uint64_t* d_counters,
                   const pfac_plan* plan, void* stream);

/*
 * Match many texts in one persistent launch per (table, tile size): the
 * waves of each workgroup take (text, tile) work items one at a time from a
 * counter in LDS, in text-then-position order; texts of at most 512 bases get
 * 256-position tiles (unless the plan fixes the tile size, or fewer than 4096
 * of them share their table with longer texts: those go with the longer ones).
 *   tables/num_tables  host array of tables (all on the current device)
 *   descs/num_texts    host array of descriptors (copied by the call)
 *   d_text_base        device base of all texts
 *   d_match_base       device int32 base or NULL (then no dense output)
 *   d_hits             device pfac_batch_hit[hit_cap] or NULL; hits ordered by
 *                      (text index, position)
 *   d_counters         device uint64[2 + 2*num_texts]: [0] hits, [1] occurrences over
 *                      the batch, then per text t: [2+2t] hits, [3+2t] occurrences.
 *                      Text t's hits start at the sum of [2+2u] over u < t.
 */
int pfac_match_batch(const pfac_table* const* tables, uint32_t num_tables,
                     const pfac_text_desc* descs, uint32_t num_texts, const void* d_text_base,
                     int32_t* d_match_base, pfac_batch_hit* d_hits, uint64_t hit_cap,
                     uint64_t* d_counters, const pfac_plan* plan, void* stream);

/*
 * A prepared batch: pfac_batch_create does every host step of
 * pfac_match_batch once (argument checks, plans, tile numbering, descriptor
 * upload, scratch allocation; synchronous), and pfac_batch_launch then only
 * enqueues kernels on `stream` -- no allocation, host copy or memset -- so
 * it may be captured into a hipGraph and replayed.  The texts' sizes,
 * offsets, tables and encodings are fixed at creation; the contents of the
 * buffers passed to each launch may change.  Outputs and their meaning are
 * those of pfac_match_batch.  A batch owns its scratch: launches of one batch
 * must be ordered (one stream, or synchronised); different batches are
 * independent.  pfac_batch_free synchronises the device first.
 */
typedef struct pfac_batch pfac_batch;

int pfac_batch_create(const pfac_table* const* tables, uint32_t num_tables,
                      const pfac_text_desc* descs, uint32_t num_texts, const pfac_plan* plan,
                      pfac_batch** out);

int pfac_batch_launch(pfac_batch* batch, const void* d_text_base, int32_t* d_match_base,
                      pfac_batch_hit* d_hits, uint64_t hit_cap, uint64_t* d_counters,
                      void* stream);

/* The extents a prepared batch reads and writes: *text_extent = bytes of
 * d_text_base its texts reach (offset + encoded length, over the texts with
 * n > 0), *match_extent = int32 elements of d_match_base their dense outputs
 * reach, *tiles = tiles of the call.  Any pointer may be NULL.  Host only. */
int pfac_batch_info(const pfac_batch* batch, uint64_t* text_extent, uint64_t* match_extent,
                    uint64_t* tiles);

void pfac_batch_free(pfac_batch* batch);

/* The plan the library would use for `table` and a text of n bases (fields
 * filled in, none left 0). */
int pfac_default_plan(const pfac_table* table, uint64_t n, int enc, pfac_plan* out);

/*
 * Host-only build of the same table pfac_build_table uploads (no device
 * needed), for inspection and tests.  Buffers are caller-owned host memory:
 *   next     uint32[4*cap]: row s, column a (A=0,C=1,G=2,T=3) = child state in
 *            bits 0..30 (0 = no transition; the root, state 0, is never a
 *            child), bit 31 set when the child is a final state
 *   pid      int32[cap]: smallest pattern ID ending at the state, 0 = none
 *   mult     uint32[cap]: number of pattern IDs ending at the state
 *   jump     uint32[4^D] or NULL, D = depth (6..10): for every D-base window
 *            (key = sum of base_k * 4^(D-1-k), first base most significant;
 *            A=0 C=1 G=2 T=3) the state reached after D steps of
 *            the walk (0 if it stopped earlier), bit 31 set if a final state was
 *            passed; jump_pid/jump_cnt (or NULL) receive the longest pattern
 *            passed and the occurrences passed within the D steps
 * States are numbered breadth-first.  *num_states always receives the state
 * count; the state arrays are written only when it is <= cap.
 */
int pfac_build_host(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                    uint32_t* next, int32_t* pid, uint32_t* mult, uint64_t cap,
                    uint32_t depth, uint32_t* jump, int32_t* jump_pid, uint32_t* jump_cnt,
                    uint64_t* num_states, int64_t* bad_index);

/*
 * Host-only: the LDS image the scan kernel uses for filter depth D (6..10),
 * for inspection and tests.  Layout of `words` (uint32): the 4^D-bit filter
 * bitmap (bit x of word x/32 set iff the D-base window with key x leads to a
 * trie node or passes a final state), then one word per 128 bitmap bits with
 * the number of set bits before it, then for each trie level d = D, D+1, ...
 * (`levels` of them) the node bytes of the level in breadth-first order (4
 * per word, first node in the low byte; bits 0..3 = child A,C,G,T exists,
 * bit 4 = final), padded to 16 nodes, followed by one word per 16 nodes with
 * the number of child bits of the level before that group.
 * meta[0] = levels, meta[1 + 3k .. 3 + 3k] = word offset of level D+k's node
 * bytes, of its count words, and the image size in words up to that level.
 * *num_words always receives the image size; words/meta are written only
 * when it is <= cap (meta needs 1 + 3*8 entries).
 */
int pfac_build_host_image(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                          uint32_t depth, uint32_t* words, uint64_t cap, uint32_t* meta,
                          uint64_t* num_words, int64_t* bad_index);

/*
 * Host-only: the second-filter bitmap of 2^bits bits (bits = 12..20) the
 * scan kernel uses, for inspection and tests.  K = min(shortest pattern, 16);
 * the key of a K-base window is sum of base_k * 4^(15-k) for k < K (first
 * base most significant, left-aligned in 32 bits, lower bits 0); its bits
 * are h1 = (key * 0x9E3779B1 mod 2^32) >> (32 - bits) and
 * h2 = (key * 0x85EBCA77 mod 2^32) >> (32 - bits), and both (bit h of word
 * h/32) are set for the first K bases of every pattern; a window passes the
 * filter when both of its bits are set.  *k receives K; `words`
 * (uint32[2^bits / 32], caller-owned) is written when non-NULL.
 */
int pfac_build_host_hash(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                         uint32_t bits, uint32_t* words, uint32_t* k, int64_t* bad_index);

/*
 * Host-only: the one-hash form of the second filter (2^bits bits, bits =
 * 12..20), which the scan uses instead of the two-hash one for pattern sets
 * with K <= 12 that most windows pass at the filter depth (they also have
 * the exact prefix filter behind it).  The key of a K-base window is
 * sum of base_k * 4^(K-1-k) for k < K (first base most significant,
 * right-aligned); its bit is h = (key * 0xC6A4A7 mod 2^32) >> (32 - bits),
 * set for the first K bases of every pattern; a window passes when its bit
 * is set.  *k receives K and `words` (uint32[2^bits / 32], caller-owned)
 * the bitmap when non-NULL.  PFAC_E_ARG when K > 12 (no such bitmap; words
 * are zeroed).
 */
int pfac_build_host_hash1(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                          uint32_t bits, uint32_t* words, uint32_t* k, int64_t* bad_index);

/*
 * Host-only: the path-compression records the walk uses, for inspection and
 * tests.  chain[2s] = the bases of the run of single-child steps below state
 * s (base k of the run in bits 31-2k..30-2k, A=0 C=1 G=2 T=3) with the run
 * length in bits 0..3, chain[2s+1] = the state the run ends at, bit 31 set
 * when that state is final.  Every state strictly inside a run has exactly
 * one child and is not final; runs are at most 14 bases; a length below 2
 * means no run.  States are numbered as in pfac_build_host.  *num_states
 * always receives the state count; chain (uint32[2*cap]) is written only
 * when it is <= cap.
 */
int pfac_build_host_chain(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                          uint32_t* chain, uint64_t cap, uint64_t* num_states,
                          int64_t* bad_index);

/*
 * Host-only: the prefix-filter bitmap the scan kernel reads, for inspection
 * and tests.  K2 = min(shortest pattern, 12), 0 (no bitmap) when the
 * shortest pattern has fewer than 7 bases; bit x (bit x%32 of word x/32) is
 * set iff some pattern's first K2 bases have the key x = sum of base_k *
 * 4^(K2-1-k) (first base most significant, A=0 C=1 G=2 T=3).  *k receives
 * K2, *num_keys the number of set bits; `words` (uint32[4^K2 / 32]) is
 * written when non-NULL and cap_words holds it.
 */
int pfac_build_host_prefix(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                           uint32_t* words, uint64_t cap_words, uint32_t* k, uint64_t* num_keys,
                           int64_t* bad_index);

/* Human-readable text of a status code (static storage). */
const char* pfac_strerror(int status);

/* Library version string. */
const char* pfac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PFAC_H */

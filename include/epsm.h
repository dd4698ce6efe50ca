/*
 * epsm.h - C ABI of the MI355X (gfx950) exact packed string matching library.
 *
 * The operation is the exact string matching problem as the paper states it
 * (Faro and Kulekci, "Fast Packed String Matching for Short Patterns",
 * Introduction and Section 2): given a text t of length n and a pattern p of
 * length m > 0 over bytes, report ALL positions s, 0 <= s <= n-m, with
 * t[s+j] = p[j] for 0 <= j < m.  Overlapping occurrences are all reported;
 * positions are 0-based starts written as int64 in strictly ascending order.
 * Byte value 0 is an ordinary symbol; texts are length-counted.
 *
 * Method (Section 3): patterns with m < 16 are found by comparing each text
 * position's packed window against the packed pattern prefix, then checking
 * the rest exactly (the role of EPSMa/EPSMb, Sections 3.2-3.3).  Patterns
 * with m >= 16 go through a fingerprint filter over aligned 8-byte text
 * blocks, whose hash selects the pattern offsets j for which position
 * (block - j) is a candidate, followed by an exact check (EPSMc, Section 3.4).
 * Both variants report exactly the set above; the hash only changes speed.
 *
 * Conventions
 *  - "d_" arguments are device pointers (HIP device memory of the device the
 *    plan was created on); other pointers are host pointers.
 *  - stream: a hipStream_t cast to void* (NULL = the default stream).  Every
 *    search call is asynchronous and stream ordered; results are valid after
 *    the stream is synchronised.  No search call (epsm_search, epsm_count,
 *    their DNA forms, epsm_search_batch) waits for the device or allocates
 *    with a device-synchronising call: workspace growth is stream ordered
 *    (hipFreeAsync / hipMallocAsync on the stream), and batch descriptors
 *    reach the device by a stream-ordered copy from pinned staging memory.
 *    Calls that synchronise say so.
 *  - Graph capture: every search call may be captured.  While its stream is
 *    being captured a call allocates nothing; it returns EPSM_EUNSUPPORTED if
 *    the stream's workspace is too small or the stream has no fault word yet,
 *    so call epsm_reserve on the stream before capturing.
 *  - Errors are returned as epsm_status; a thread-local message is available
 *    from epsm_last_error().  Synchronous returns report argument and launch
 *    errors only.
 *  - The caller owns every buffer it passes; the library never frees caller
 *    memory.  A plan owns its own copy of the pattern and its device tables.
 *  - Text and output pointers may have any alignment.
 */
#ifndef EPSM_H
#define EPSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPSM_OK = 0,
    EPSM_EINVAL = 1,       /* invalid argument (m == 0, NULL pointer, bad flags) */
    EPSM_ENOMEM = 2,       /* host or device allocation failed */
    EPSM_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed */
    EPSM_EUNSUPPORTED = 4  /* valid request outside what this build supports */
} epsm_status;

/* Opaque, immutable after creation.  Safe to use concurrently from several
 * host threads and on several streams. */
typedef struct epsm_plan_s *epsm_plan_t;

/* ---- plan flags -------------------------------------------------------- */
/* Build host-side tables only (no device allocation); such a plan can be
 * inspected with epsm_plan_get_info but is rejected by search calls. */
#define EPSM_PLAN_HOST_ONLY 0x1u
/* Force the direct-compare variant (any m). */
#define EPSM_PLAN_FORCE_DIRECT 0x2u
/* Force the fingerprint variant (requires m >= 15, see Section 3.4). */
#define EPSM_PLAN_FORCE_FINGERPRINT 0x4u
/* Test mode: the fingerprint hash is the constant 0, so every aligned block
 * hits the same bucket and every offset is verified; output is unchanged. */
#define EPSM_PLAN_COLLIDE 0x8u
/* Fingerprint width k (bucket count 2^k), Section 3.4 uses k = 11.
 * Encoded in bits 8..11 of flags as EPSM_PLAN_HASH_BITS(k), 8 <= k <= 14;
 * 0 selects the default (11). */
#define EPSM_PLAN_HASH_BITS(k) (((uint32_t)(k) & 0xFu) << 8)
/* The pattern is a string of DNA codes 0..3 (one per byte, e.g. A,C,G,T ->
 * 0,1,2,3; the mapping is the caller's) to be searched in packed 2-bit texts
 * with epsm_search_dna / epsm_count_dna.  Excludes the variant and
 * fingerprint flags. */
#define EPSM_PLAN_DNA 0x10u
/* Never use the strided filter (see EPSM_VARIANT_STRIDE); long patterns then
 * use the per-block fingerprint filter.  Output is the same. */
#define EPSM_PLAN_NO_STRIDE 0x20u
/* Direct variant: filter on a 4-byte prefix even for m >= 5 (the default
 * there compares the first min(m, 8) bytes as one 64-bit word, Section 3.2's
 * packed compare at twice the width).  Output is the same. */
#define EPSM_PLAN_PREFIX4 0x40u
/* Direct variant with m > 16: compare the first 16 bytes from a register run
 * of two 16-byte blocks per lane and check the rest of each surviving
 * candidate from memory (the default run for a direct m > 16 is three
 * blocks, holding 32 pattern bytes).  Output is the same. */
#define EPSM_PLAN_SHORT_RUN 0x80u
/* Alphabet-size hint: the effective number of distinct byte values of the
 * texts the plan will search (1..256; see epsm_estimate_alphabet), in bits
 * 16..24 of flags; 0, the default, means unknown.  Only the variant table
 * (epsm_set_variant_table) reads it; output never depends on it. */
#define EPSM_PLAN_SIGMA(s) (((uint32_t)(s) & 0x1FFu) << 16)

/* Variants */
#define EPSM_VARIANT_DIRECT 1u
#define EPSM_VARIANT_FINGERPRINT 2u
#define EPSM_VARIANT_DNA 3u
/* Long patterns (m >= 263): the fingerprint filter with a stride, as EPSMc
 * (Section 3.4) is defined: only the aligned 8-byte blocks at multiples of S
 * are read (S the largest power of two <= min(m - 7, 2048); a variant-table
 * row may ask for it from m = 39, S >= 32), so the text lines in between are
 * not fetched.  Every occurrence contains exactly one
 * such block, at pattern offset j in [0, S); the plan's table lists the
 * offsets per hash value, and every candidate is checked exactly.  Chosen by
 * default unless a FORCE or COLLIDE flag or EPSM_PLAN_NO_STRIDE is given;
 * inside batches such a plan filters per block like EPSM_VARIANT_FINGERPRINT. */
#define EPSM_VARIANT_STRIDE 4u

/* Kernel classes of single-text searches (the key of the tune table). */
#define EPSM_CLASS_BYTES 0u        /* direct variant, m <= 3: byte compares */
#define EPSM_CLASS_WORDS 1u        /* direct variant, m >= 4: packed-word compares */
#define EPSM_CLASS_FINGERPRINT 2u  /* fingerprint variant (Section 3.4) */
#define EPSM_CLASS_DNA 3u          /* packed 2-bit DNA texts */
#define EPSM_N_CLASSES 4u

/* Longest pattern this build accepts. */
#define EPSM_MAX_M 4096u

/*
 * epsm_plan: preprocess pattern[0..m-1] (host memory, copied) for searches on
 * the current HIP device.  Chooses the variant by m (direct for m < 16,
 * fingerprint for m >= 16) unless forced by flags, packs the pattern into
 * 32-bit words, and for the fingerprint variant builds the table of Section
 * 3.4: entry v holds the set of offsets j in [0,7] with h(p[j..j+7]) = v.
 * Returns EPSM_EINVAL for m == 0, a NULL pattern or out, or bad flags;
 * EPSM_EUNSUPPORTED for m > EPSM_MAX_M; EPSM_ENOMEM / EPSM_EDEVICE if the
 * device copy fails.  On success *out receives the plan.
 */
epsm_status epsm_plan(const uint8_t *pattern, uint64_t m, uint32_t flags, epsm_plan_t *out);

/* Release a plan.  The caller guarantees no search using it is in flight. */
void epsm_plan_destroy(epsm_plan_t plan);

typedef struct {
    uint64_t m;              /* pattern length */
    uint32_t variant;        /* EPSM_VARIANT_* */
    uint32_t flags;          /* flags the plan was built with */
    uint32_t hash_bits;      /* k of the fingerprint variant, or of the block
                                filter of DNA plans with m >= 8 (else 0) */
    uint32_t prefix_words;   /* 32-bit pattern words compared in the filter */
    uint32_t words[8];       /* pattern bytes 4i..4i+3, little endian, 0 past m */
    uint32_t masks[8];       /* 0xFF in each byte lane that lies below m */
    const uint16_t *table;   /* host copy of the fingerprint table, 2^k entries:
                                bit (8-j) of entry v is set iff offset j is in
                                bucket v; for DNA plans with m >= 16, bit j of
                                entry v is set iff the 8-symbol block j..j+7
                                (symbol t at bits 2t) hashes to v
                                (epsm_fingerprint(block, 0, k, 0)); with
                                8 <= m < 16 (k = 8), iff the 4-symbol block
                                j..j+3 equals v; NULL otherwise.  Owned by the
                                plan. */
    int32_t device;          /* HIP device of the device tables, -1 if host only */
    uint32_t kernel_class;   /* EPSM_CLASS_* of the plan's scan kernel */
    uint32_t stride;         /* EPSM_VARIANT_STRIDE: bytes between inspected blocks, else 0 */
    uint32_t prefix_bytes;   /* EPSM_VARIANT_DIRECT: bytes of the prefix compare
                                (min(m, 8); 4 for m > 4 with EPSM_PLAN_PREFIX4
                                or m > 16 on a three-block run), else 0 */
    uint32_t run_blocks;     /* 16-byte blocks of a lane's register run (2 or 3;
                                1 for DNA plans) */
    uint32_t table_row;      /* 1 + the index of the variant-table row that chose
                                the variant, or 0 (built-in choice or forced) */
} epsm_plan_info;

/* Copy the plan's description to *info (host memory). */
epsm_status epsm_plan_get_info(epsm_plan_t plan, epsm_plan_info *info);

/* The fingerprint hash of an 8-byte block whose little-endian 32-bit halves
 * are lo and hi, reduced to k bits (the role of wscrc & mask, Section 3.1 and
 * 3.4).  Exposed so tests can check the table; the device uses the same
 * function.  collide != 0 gives the constant-0 test hash. */
uint32_t epsm_fingerprint(uint32_t lo, uint32_t hi, uint32_t k, int collide);

/*
 * epsm_search: write the occurrence positions of plan's pattern in
 * d_text[0..n-1] to d_out.  d_out receives the first min(count,
 * out_capacity) positions, ascending (a prefix of the full answer);
 * *d_n_hits (device, uint64) receives the full count.  d_out may be NULL if
 * out_capacity == 0.  n == 0 or m > n gives count 0.  Uses a library-owned
 * workspace tied to the stream (grown on demand, in stream order; see
 * epsm_reserve for graph capture).  Long texts with a small out_capacity are
 * searched in two phases (see EPSM_WRITE_AUTO), whose workspace is about n/8
 * bytes; others in a single pass, whose tiles wait (with a bound) on their
 * predecessors' counts: if such a wait ever gave up, the stream's fault word
 * is set and epsm_stream_check reports it.
 */
epsm_status epsm_search(epsm_plan_t plan, const uint8_t *d_text, uint64_t n,
                        int64_t *d_out, uint64_t out_capacity,
                        uint64_t *d_n_hits, void *stream);

/* epsm_count: the occurrence count only, to *d_n_hits (device, uint64). */
epsm_status epsm_count(epsm_plan_t plan, const uint8_t *d_text, uint64_t n,
                       uint64_t *d_n_hits, void *stream);

/*
 * epsm_search_noalloc: epsm_search for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, output, ordering and truncation as
 * epsm_search (out_capacity == 0 gives the count only); it never allocates,
 * frees or waits: its scratch (tile counts, look-back status words,
 * two-phase slots, the fault word of its bounded waits) is one static device
 * array of EPSM_NOALLOC_SCRATCH_BYTES, one copy per device, which every GPU
 * the library runs on holds from the library's load until the process ends.
 * A search whose scratch would not fit takes the single pass (8 bytes per
 * tile: texts up to about 127 GiB at the default 128 KiB tile) instead of the
 * two-phase write (about n/8 bytes); a longer text returns EPSM_EUNSUPPORTED
 * before anything is launched.  Packed DNA plans are rejected (EPSM_EINVAL).
 * Every call on a device shares that device's array and leaves its contents
 * behind (what must start at zero is cleared by each call, in stream
 * order): calls that overlap in time on one device (on different streams or
 * from different threads) race and give wrong output, so serialise them (one
 * stream does).  A give-up of one of its bounded waits is reported by the
 * next epsm_stream_check on any stream of the device.
 */
#define EPSM_NOALLOC_SCRATCH_BYTES (8u << 20)
epsm_status epsm_search_noalloc(epsm_plan_t plan, const uint8_t *d_text, uint64_t n,
                                int64_t *d_out, uint64_t out_capacity, uint64_t *d_n_hits,
                                void *stream);

/* ---- packed DNA texts ------------------------------------------------------ */

/*
 * A text over four symbols stored at two bits per symbol: symbol i occupies
 * bits 2*(i%4) and 2*(i%4)+1 of byte i/4, so n symbols take ceil(n/4) bytes
 * and a little-endian 32-bit word holds 16 consecutive symbols.  The search
 * is the same problem (all s, 0 <= s <= n-m, with t[s+j] = p[j] for j < m;
 * positions and n count symbols) on a quarter of the bytes.  The paper leaves
 * such texts out (it states the byte-alphabet setting in Section 2); this is
 * the packed-text extension of its direct compare.
 */

/* Pack n symbol codes (device bytes; only their low two bits are used) into
 * d_packed (device, ceil(n/4) bytes; no byte past that is written).  Bits of
 * the last byte past n are zero. */
epsm_status epsm_pack_dna(const uint8_t *d_codes, uint64_t n, uint8_t *d_packed, void *stream);

/* epsm_search / epsm_count over a packed text of n symbols at d_packed (any
 * byte alignment).  The plan must be made with EPSM_PLAN_DNA, and such a plan
 * is rejected by the byte searches and by batches (EPSM_EINVAL).  Positions
 * are symbol indices. */
epsm_status epsm_search_dna(epsm_plan_t plan, const uint8_t *d_packed, uint64_t n,
                            int64_t *d_out, uint64_t out_capacity, uint64_t *d_n_hits,
                            void *stream);
epsm_status epsm_count_dna(epsm_plan_t plan, const uint8_t *d_packed, uint64_t n,
                           uint64_t *d_n_hits, void *stream);

/* ---- batched search ------------------------------------------------------ */

typedef struct {
    const uint8_t *d_text;   /* device pointer */
    uint64_t n;              /* length in bytes */
} epsm_text_ref;

typedef struct {
    uint32_t text;           /* index into texts[] */
    epsm_plan_t plan;        /* pattern to search in that text */
} epsm_pair_ref;

#define EPSM_BATCH_COUNT_ONLY 0x1u
/* Filter every pair on its own in the count pass.  By default a text with at
 * least 4 patterns of m >= 4 counts them in groups of up to 32 through one
 * shared filter (a bucket table of their first four bytes, then an exact
 * check); the output is the same either way. */
#define EPSM_BATCH_NO_GROUPS 0x2u

typedef struct {
    const epsm_text_ref *texts;  /* host array [n_texts] */
    uint32_t n_texts;
    const epsm_pair_ref *pairs;  /* host array [n_pairs] */
    uint32_t n_pairs;
    int64_t *d_out;              /* concatenated positions, pair order */
    uint64_t out_capacity;       /* entries available in d_out */
    uint64_t *d_counts;          /* device [n_pairs]: full count of each pair */
    uint64_t *d_offsets;         /* device [n_pairs]: exclusive prefix of counts */
    uint64_t *d_total;           /* device, optional (may be NULL): sum of counts */
    uint32_t flags;              /* EPSM_BATCH_* */
} epsm_batch;

/*
 * epsm_search_batch: every (text, pattern) pair of the batch in one
 * stream-ordered submission.  Pair k's positions (relative to its text) are
 * d_out[d_offsets[k] .. d_offsets[k] + d_counts[k]) in ascending order;
 * entries at or beyond out_capacity are not written (counts and offsets are
 * always complete).  With EPSM_BATCH_COUNT_ONLY only counts, offsets and
 * total are produced.  Output is identical to calling epsm_search per pair.
 * Device plans must live on the current device.  The host arrays are read
 * before the call returns: the work descriptors built from them are copied
 * into pinned staging memory owned by the library and reach the stream's
 * workspace by a stream-ordered copy, so the call does not wait for the
 * device.  A staging block is reused once its copy has completed; a block
 * copied under graph capture is read by every replay and is kept until
 * epsm_release.  Plans may be host-only (EPSM_PLAN_HOST_ONLY): the batch then
 * carries their tables to the device itself, which avoids one device
 * allocation and copy per plan.  Plans must outlive the copy (and, under
 * capture, the graph).
 */
epsm_status epsm_search_batch(const epsm_batch *batch, void *stream);

/* Bytes of stream workspace that epsm_search_batch needs for this batch
 * (the descriptors, the per-(pair, tile) counts and offsets, 8 bytes per
 * pair for the shift from its entries' offsets to its output offset, and
 * 260 bytes per text tile for the count pass's parked hits), for
 * epsm_reserve before a graph capture.  Validates the batch as
 * epsm_search_batch does, without its output pointers. */
epsm_status epsm_batch_workspace(const epsm_batch *batch, uint64_t *bytes);

/* ---- tuning ------------------------------------------------------------- */

/* Select the workgroup tile used by later single-text searches: `waves`
 * wavefronts of 64 lanes per workgroup, each scanning `pieces` KiB per tile
 * (tile = waves * pieces KiB).  Built configurations: 8x16 (default), 8x8,
 * 4x16, 4x32, 16x8, 16x16; others return EPSM_EUNSUPPORTED.  Process-wide; not thread safe
 * against concurrent searches.  Output never depends on the choice. */
epsm_status epsm_set_tile_config(uint32_t waves, uint32_t pieces);

/* The tile configurations built into the library, default first: writes up
 * to `capacity` of them to waves[i] / pieces[i] (either may be NULL) and
 * returns how many are built. */
uint32_t epsm_tile_configs(uint32_t *waves, uint32_t *pieces, uint32_t capacity);

/* Write strategies of epsm_search (the order of the output is the same).
 * SINGLE_PASS: each tile learns its output offset from a decoupled look-back
 * over the counts of the tiles before it and writes its own positions; a tile
 * may wait for its predecessors.  TWO_PHASE: each tile parks its hits in a
 * slot of the workspace (a list of offsets, or its hit masks when the list
 * would be longer) without waiting; a one-workgroup scan of the tile counts
 * then gives each tile its offset, and an expand kernel writes the positions;
 * fastest for sparse output.  AUTO: two-phase for texts of at least 32 tiles
 * with out_capacity <= n / 128 (the capacity bounds the positions written),
 * else single pass. */
#define EPSM_WRITE_AUTO 0u
#define EPSM_WRITE_SINGLE_PASS 1u
#define EPSM_WRITE_TWO_PHASE 2u

/* One row of the tune table: searches of plans of class `kernel_class`, in
 * mode `count_only` (0: epsm_search, 1: epsm_count), over texts of n <=
 * n_max bytes use the tile waves x pieces and write strategy `strategy`
 * (ignored by counts). */
typedef struct {
    uint32_t kernel_class;   /* EPSM_CLASS_* */
    uint32_t count_only;     /* 0 or 1 */
    uint64_t n_max;          /* bytes */
    uint32_t waves;          /* a built tile, see epsm_tile_configs */
    uint32_t pieces;
    uint32_t strategy;       /* EPSM_WRITE_* */
} epsm_tune_entry;

/* Install the tune table (copied; at most 256 rows): a single-text search
 * uses the first row, in array order, that matches its class, mode and
 * length, and the tile of epsm_set_tile_config with EPSM_WRITE_AUTO when
 * none does.  count == 0 clears the table.  EPSM_EINVAL for an unknown
 * class, mode or strategy,
 * EPSM_EUNSUPPORTED for a tile that is not built; the old table is kept on
 * error.  Process-wide; output never depends on the table. */
epsm_status epsm_set_tune_table(const epsm_tune_entry *entries, uint32_t count);

/* Fingerprint width k (Section 3.4) for plans made later without
 * EPSM_PLAN_HASH_BITS; 8 <= k <= 14, 0 restores the default 11.
 * Process-wide; output never depends on k. */
epsm_status epsm_set_default_hash_bits(uint32_t k);

/*
 * Variant table: which variant (and run, prefix width, fingerprint width) a
 * plan made later uses, by pattern length and alphabet hint.  The paper
 * fixes the choice by m alone (Section 3: EPSMa/b below 16 bytes, EPSMc
 * above); which filter is fastest on this device also depends on how often
 * its candidates survive, i.e. on the alphabet, so the autotuner measures
 * the variants per (m, sigma) bucket and installs its choices here.  A plan
 * made without EPSM_PLAN_FORCE_* / EPSM_PLAN_COLLIDE / EPSM_PLAN_DNA takes
 * the first row, in array order, with m_min <= m <= m_max and sigma_min <=
 * sigma <= sigma_max, where sigma is its EPSM_PLAN_SIGMA hint (0 when it has
 * none); with no matching row, the built-in choice (direct below 16, the
 * fingerprint filter from 16, strided from 263).  The row's flags (any of
 * EPSM_PLAN_SHORT_RUN, EPSM_PLAN_PREFIX4, EPSM_PLAN_HASH_BITS(k)) are added
 * to the plan's own; a k of the plan's own wins.  Output never depends on
 * the table.
 */
typedef struct {
    uint32_t m_min, m_max;          /* pattern lengths, inclusive */
    uint32_t sigma_min, sigma_max;  /* alphabet hints, inclusive, 0..256 */
    uint32_t variant;               /* EPSM_VARIANT_DIRECT, _FINGERPRINT (m_min >= 15)
                                       or _STRIDE (m_min >= 39: the strided filter
                                       with S the largest power of two <= min(m - 7,
                                       2048), S >= 32) */
    uint32_t flags;                 /* EPSM_PLAN_SHORT_RUN | EPSM_PLAN_PREFIX4 |
                                       EPSM_PLAN_HASH_BITS(k), or 0 */
} epsm_variant_entry;

/* Install the variant table (copied; at most 256 rows; count == 0 clears it).
 * EPSM_EINVAL for a bad row (empty range, sigma above 256, unknown variant or
 * flags, a fingerprint row below m = 15, a strided row below m = 39, k
 * outside 8..14); the old table is kept on error.  Process-wide; affects
 * plans made later. */
epsm_status epsm_set_variant_table(const epsm_variant_entry *entries, uint32_t count);

/* Effective alphabet size of a text, from its first min(n, 65536) bytes:
 * round(L^2 / sum_c count_c^2), the inverse of the probability that two
 * sampled bytes are equal (sigma for a uniform text over sigma symbols),
 * clamped to 1..256; 0 for n == 0.  Runs one kernel on `stream` and
 * synchronises the stream (the value is returned to the host).  For
 * EPSM_PLAN_SIGMA. */
epsm_status epsm_estimate_alphabet(const uint8_t *d_text, uint64_t n, uint32_t *sigma, void *stream);

/*
 * Prepared batches, for callers that run the same batch structure many times
 * (a serving loop, graph replays).  epsm_batch_prepare validates the batch,
 * builds the work descriptors and copies them to device memory owned by the
 * returned handle (synchronous; the host arrays may be freed afterwards).
 * The output pointers of *batch are recorded and reused by every launch.
 * epsm_batch_launch submits the batch on `stream`: on a non-null stream the
 * kernel sequence is captured into a HIP graph on first use and replayed
 * after that (no host round trip, no allocation); on the null stream the
 * kernels are launched directly.  Launches on one handle must not overlap.
 * Plans referenced by the batch must outlive the handle.
 */
typedef struct epsm_batch_plan_s *epsm_batch_plan_t;
epsm_status epsm_batch_prepare(const epsm_batch *batch, epsm_batch_plan_t *out);
epsm_status epsm_batch_launch(epsm_batch_plan_t bp, void *stream);
void epsm_batch_destroy(epsm_batch_plan_t bp);
/* Work units (text tiles), (pair, tile) entries and tile bytes of a prepared
 * batch; any output pointer may be NULL. */
epsm_status epsm_batch_get_info(epsm_batch_plan_t bp, uint64_t *units, uint64_t *entries,
                                uint32_t *tile_bytes);

/* Select the batch tile (`waves` KiB per text tile: 4, 8 or 16) used by later
 * batch calls.  Output never depends on the choice. */
epsm_status epsm_set_batch_config(uint32_t waves);

/* ---- serving: continuous batching over resident texts ------------------- */

/*
 * A server keeps texts resident in device memory (the caller owns them and
 * keeps them alive) and answers queries: a text id plus a set of patterns,
 * every occurrence of every pattern as in epsm_search.  A scheduler thread
 * forms micro-batches from the queue of submitted queries as stream slots
 * and device memory free up, so queries that arrive while others are on the
 * device are admitted and run concurrently with them (continuous batching).
 * Device memory for a micro-batch's work and output is admitted against
 * hbm_budget; a query never fails for lack of budget: it waits, and work
 * larger than the whole budget runs when nothing else holds device memory.
 * Results are identical to searching each pattern alone.
 */
typedef struct epsm_server_s *epsm_server_t;

typedef struct {
    uint32_t slots;              /* micro-batches in flight, one HIP stream each (0 = 4, max 16) */
    uint32_t max_batch_queries;  /* queries per micro-batch (0 = 64) */
    uint64_t max_batch_entries;  /* (pattern, text tile) entries per micro-batch (0 = 2^25) */
    uint64_t hbm_budget;         /* device bytes for micro-batch work and outputs (0 = 16 GiB) */
    uint32_t flags;              /* EPSM_SERVER_* (0 for normal operation) */
} epsm_server_config;

/* Test hook: every write stage fails its output allocation as if the device
 * were out of memory; its queries complete with EPSM_ENOMEM and the slot's
 * device memory is released. */
#define EPSM_SERVER_FAIL_OUTPUT_ALLOC 0x1u

typedef struct {
    uint64_t query_id;
    uint32_t text_id;
    uint32_t n_patterns;
    int32_t status;              /* epsm_status of the query */
    uint32_t batch_queries;      /* queries that shared its micro-batch */
    uint64_t total;              /* positions over all its patterns */
    const uint64_t *counts;      /* host [n_patterns] */
    const uint64_t *offsets;     /* host [n_patterns]: pattern k's positions start here */
    const int64_t *positions;    /* host [total], ascending within each pattern */
    double submit_time;          /* server clock (seconds since creation) */
    double start_time;           /* its micro-batch was formed */
    double done_time;            /* its results were in host memory */
} epsm_query_result;

typedef struct {
    uint64_t submitted, completed, in_flight, queued, batches;
    uint64_t bytes_reserved, bytes_peak;  /* admitted device memory now / at most */
} epsm_server_stats;

/* Create a server on the current device (cfg may be NULL for defaults). */
epsm_status epsm_server_create(const epsm_server_config *cfg, epsm_server_t *out);
/* Register a resident text (device pointer, any alignment); returns its id. */
epsm_status epsm_server_add_text(epsm_server_t s, const uint8_t *d_text, uint64_t n,
                                 uint32_t *text_id);
/* Queue a query: n_patterns patterns given back to back in host memory
 * (copied), lengths[k] bytes each.  Thread safe; returns immediately. */
epsm_status epsm_server_submit(epsm_server_t s, uint32_t text_id, const uint8_t *patterns,
                               const uint64_t *lengths, uint32_t n_patterns, uint64_t *query_id);
/* Take up to max completed queries (in completion order), waiting up to
 * wait_us microseconds for the first one.  The result arrays stay valid
 * until epsm_server_release(query_id). */
epsm_status epsm_server_poll(epsm_server_t s, epsm_query_result *out, uint32_t max,
                             uint32_t *n_out, uint32_t wait_us);
/* Free the results of a query that epsm_server_poll has returned;
 * EPSM_EINVAL for an unknown id or a query not yet returned by a poll. */
epsm_status epsm_server_release(epsm_server_t s, uint64_t query_id);
/* Server clock in seconds (the time base of the result timestamps). */
double epsm_server_now(epsm_server_t s);
epsm_status epsm_server_get_stats(epsm_server_t s, epsm_server_stats *st);
/* Stop the scheduler, wait for in-flight work and free the server; queries
 * not yet started complete with EPSM_EDEVICE. */
void epsm_server_destroy(epsm_server_t s);

/* ---- workspace and diagnostics -------------------------------------------- */

/* Make sure the workspace tied to `stream` serves, without allocating
 * again, searches of texts of up to max_n bytes (packed DNA: max_n symbols)
 * with any tile and write strategy, and one-shot batches whose
 * epsm_batch_workspace is at most batch_bytes; also creates the stream's
 * fault word and, when batch_bytes > 0, makes sure a free pinned staging
 * block of batch_bytes exists (a batch call captured into a graph takes one
 * such block for the life of the graph: reserve once per captured batch
 * call).  Device allocation is stream ordered.  Call it before capturing the
 * stream into a graph (EPSM_EUNSUPPORTED if the stream is being captured). */
epsm_status epsm_reserve(void *stream, uint64_t max_n, uint64_t batch_bytes);

/* Free every cached workspace, fault word and staging block (synchronises
 * the device first).  Graphs that captured library calls must not be
 * replayed afterwards. */
void epsm_release(void);

/* Synchronise `stream` and report EPSM_EDEVICE if a kernel launched on it
 * gave up one of its bounded inter-workgroup waits since the last check (its
 * output is then not trustworthy; the report clears the stream's fault
 * word), or if an epsm_search_noalloc kernel on the current device did (that
 * word is shared by the device's no-allocation calls).  Such a wait is not expected to time out; the Python
 * helpers that synchronise (search, count and their DNA and batch forms)
 * call this and raise.  Returns EPSM_OK otherwise. */
epsm_status epsm_stream_check(void *stream);

/* Test hook (process-wide; 0 disables): while enabled, single-pass positions
 * searches make their first tile also wait on a status word that no tile
 * publishes, with a bound of a few polls, so the wait gives up and the
 * stream's fault word is set while every kernel exits normally.  The output
 * is unaffected (the wait is an extra one).  Lets tests check that give-ups
 * surface. */
void epsm_debug_force_giveup(int enable);

/* Thread-local description of the last error on this thread ("" if none). */
const char *epsm_last_error(void);

/* Static name of a status code. */
const char *epsm_status_string(epsm_status s);

/* Library version as major*10000 + minor*100 + patch. */
int epsm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EPSM_H */

// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epsm {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kPiece = 16;          // bytes per lane per load (one dwordx4)
constexpr int kWavePiece = kWave * kPiece;  // 1 KiB per wave per load

// Status word of the single-pass scan (decoupled look-back): flag in the two
// top bits, running count in the low 62.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagInclusive = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
// Upper bound on status polls per look-back step (each poll sleeps ~64
// cycles plus a memory round trip: several seconds in total).  Every wait is
// expected to end long before; the bound only guarantees the kernel drains.
constexpr uint32_t kSpinLimit = 1u << 22;
// Poll bound of the forced wait of epsm_debug_force_giveup (a test hook).
constexpr uint32_t kDebugSpinLimit = 64;

// Fingerprint hash of an aligned 8-byte text block (lo = bytes 0..3, hi =
// bytes 4..7, little endian), reduced to `bits` bits.  A two-multiply
// multiplicative hash: the top bits of the final product depend on every
// input bit.  Any deterministic function is correct because every candidate
// is verified exactly; this one is cheap on the VALU.
__host__ __device__ inline uint32_t fp_hash(uint32_t lo, uint32_t hi, uint32_t bits) {
    uint32_t x = lo ^ (hi * 0x85EBCA77u);
    return (x * 0x9E3779B1u) >> (32u - bits);
}

// Pattern as the kernels see it (kernel argument or device array element).
struct DevPlan {
    uint32_t pw[8];          // pattern bytes 4j..4j+3 (little endian), 0 past m
    uint32_t pmask[8];       // 0xFF byte lanes below m
    uint64_t m;
    uint32_t nw;             // words compared from registers: min(ceil(m/4), 4*NL)
                             // (DNA: 16-symbol words, min(ceil(m/16), 3))
    uint32_t variant;        // 1 direct, 2 fingerprint, 3 DNA (2-bit symbols)
    uint32_t pk;             // direct prefix kind: min(m, 4) (DNA: 16 if m >= 16, else 4)
    uint32_t hash_bits;      // fingerprint: k
    uint32_t collide;        // fingerprint: constant-0 hash (test mode)
    uint32_t nl;             // dwordx4 loads per lane per piece (2 or 3)
    const uint16_t *table;   // fingerprint table, 2^k entries (device)
    const uint8_t *pattern;  // full pattern (device), for m > 4*nw
    const uint16_t *stride_table;  // strided filter: [2^kStrideHashBits + 1] bucket
                                   // starts, then [stride] offsets (device)
    const uint2 *stride_blocks;    // strided filter: [stride] pattern blocks in offset order
    uint32_t stride;         // strided filter: bytes between inspected blocks
    uint32_t pad_;
};

// One search over one text.
struct ScanArgs {
    const uint8_t *base;     // 16-byte aligned address at or below the text start
    uint64_t delta;          // text start - base, 0..15
    uint64_t last;           // delta + n - m: largest valid start in base coordinates
    uint64_t load_end;       // round_up(delta + n, 16): readable bytes from base
    int64_t *out;            // positions (may be null when cap == 0)
    uint64_t cap;
    uint64_t *n_hits;        // full count (device)
    uint64_t *status;        // [num_tiles] look-back words, zeroed before launch
    uint32_t *tcnt;          // count only and two-phase: [num_tiles] hits of each tile
                             // (every entry written)
    uint32_t *fault;         // set to 1 if a bounded wait gave up (never expected)
    uint32_t *wcnt;          // two-phase: [num_tiles * waves] hits of each wave of each tile
    uint64_t *toff;          // two-phase: [num_tiles + 1] exclusive prefix of tcnt (tile_offsets_kernel)
    uint32_t *slots;         // two-phase: [num_tiles * tile_bytes / 32] list or masks per tile
    uint32_t num_tiles;
    uint32_t shift;          // coordinates per text byte, log2: 0 bytes, 2 packed DNA
    uint32_t write;          // kWriteNone, kWriteLookBack or kWriteTwoPhase
    uint32_t expand_tiles;   // two-phase: tiles per expand workgroup, 1..kExpandTiles
    uint32_t debug_giveup;   // single pass, test hook: tile 0 also waits (bounded) on
                             // status[num_tiles], which no tile publishes
    uint32_t pad_;
    DevPlan plan;
};

// Write strategies of epsm_search.  Single pass: each tile learns its output
// offset from a decoupled look-back and writes its positions itself.  Two
// phase: each tile parks its hits in its own slot (an ascending list of tile
// offsets if they fit in tile_bytes / 32 words, else its raw hit masks) and
// stores its tile and per-wave counts; one workgroup scans the tile counts
// into offsets, and an expand kernel turns slots into positions.
constexpr uint32_t kWriteNone = 0;
constexpr uint32_t kWriteLookBack = 1;
constexpr uint32_t kWriteTwoPhase = 2;
// The most tiles per expand workgroup of the two-phase write, and the
// workgroups the expand grid is sized to (about one resident round).
constexpr uint32_t kExpandTiles = 32;
constexpr uint32_t kExpandRound = 768;

// ---- strided fingerprint filter (long patterns) ----------------------------
constexpr int kStrideWaves = 8;
constexpr int kStrideThreads = kStrideWaves * kWave;
constexpr uint32_t kStrideBlocksPerLane = 4;
constexpr uint64_t kStrideBlocksPerTile = (uint64_t)kStrideThreads * kStrideBlocksPerLane;
// S: powers of two, S <= m - 7; at least kStrideMin unless a variant-table
// row asks for the strided filter, then at least kStrideMinRow
constexpr uint32_t kStrideMin = 256, kStrideMax = 2048, kStrideMinRow = 32;
constexpr uint32_t kStrideHashBits = 12;
// Packed DNA, m >= 16: buckets of the 8-symbol block filter (2^k u16 entries
// in LDS, as the byte fingerprint table).
constexpr uint32_t kDnaHashBits = 11;

struct StrideArgs {
    const uint8_t *base;      // 16-byte aligned address at or below the text start
    uint64_t delta, last;     // valid starts are [delta, last] (base coordinates)
    uint64_t load_end;        // readable bytes from base
    uint64_t stride;          // S
    uint32_t hash_bits;
    uint32_t write;           // 0: per-workgroup counts; 1: positions
    const uint16_t *table;    // bucket starts, then offsets
    const uint2 *blocks;      // [stride] pattern blocks p[j..j+7] (lo, hi) in offset order
    const uint8_t *pattern;
    uint64_t m;
    uint64_t first_block;     // inspected blocks are (first_block + b) * S, b < num_blocks
    uint64_t num_blocks;
    uint32_t *tile_count;     // [workgroups]
    const uint64_t *tile_offset;  // [workgroups + 1], exclusive scan of tile_count
    int64_t *out;
    uint64_t cap;
};
hipError_t launch_stride(const StrideArgs &a, uint32_t tiles, hipStream_t s);
hipError_t launch_copy_u64(const uint64_t *src, uint64_t *dst, hipStream_t s);

// ---- batched search -------------------------------------------------------
// A unit is one tile of one text; its workgroup loads the tile once and runs
// every pattern aimed at that text over it.

struct BatchTextDesc {
    const uint8_t *base;     // 16-byte aligned address at or below the text start
    uint64_t n;              // text length
    uint64_t entry_begin;    // first (pair, tile) entry of the text's pairs
    uint32_t delta;          // text start - base (< 16); readable to round_up(delta + n, 16)
    uint32_t tiles;          // tiles of the text: each of its pairs has one entry per tile
    // this text's pairs are kpairs[pair_begin, pair_end): first those the
    // count pass filters one by one, [pair_begin, solo_end), then those it
    // filters in groups of up to kGroupMax: the patterns of m = 4..7,
    // [solo_end, short_end), in the groups group_begin .. long_group - 1,
    // keyed by their first 4 bytes, then those of m >= 8, [short_end,
    // pair_end), in the groups long_group .. group_end - 1, keyed by their
    // first 8 bytes.  Entries follow the same order: pair q's entry for tile
    // i is entry_begin + (q - pair_begin) * tiles + i.
    uint32_t pair_begin;
    uint32_t solo_end;
    uint32_t short_end;
    uint32_t pair_end;
    uint32_t group_begin;
    uint32_t long_group;
    uint32_t group_end;
    uint32_t pad_;
};
static_assert(sizeof(BatchTextDesc) == 64, "one scalar load per text descriptor");

// Multi-pattern count (several patterns of one text through one filter).
// A group holds up to kGroupMax patterns aimed at one text; its bucket table
// maps the hash of a window to the set of group members (bit j) whose first
// bytes hash there: 4-byte windows for patterns of m = 4..7, 8-byte windows
// for m >= 8 (on small alphabets a 4-byte prefix matches too often to
// filter: over 4 symbols a text window equals one of 30 patterns' first
// words at about one position in eight).
constexpr uint32_t kGroupMax = 32;
constexpr int kGroupBits = 10;
constexpr uint32_t kGroupBuckets = 1u << kGroupBits;
// A group's table in memory: the kGroupBuckets member masks, then one flag
// byte per bucket (1: not empty), so testing a window's bucket is one LDS
// byte read at the bucket index, with no word and bit to extract.
constexpr uint32_t kGroupFlagWords = kGroupBuckets / 4;
constexpr uint32_t kGroupTableWords = kGroupBuckets + kGroupFlagWords;
// A text's word patterns are grouped only when it has at least this many.
constexpr uint32_t kGroupMin = 4;
// Parked group hits: the count pass lists up to kParkMax hits of a unit's
// grouped pairs, each as (member << 16) | (offset in the unit), member being
// the pair's index among its text's grouped pairs; sorted, these are the
// unit's grouped positions in output order, so the write pass places them
// without running the group filter again.  A unit with more hits (or a text
// with more than 65536 grouped pairs) stores kParkOverflow and the write
// pass recomputes its grouped pairs.
constexpr uint32_t kParkMax = 64;
constexpr uint32_t kParkOverflow = 0xFFFFFFFFu;

// Bucket of a 4-byte window x (little endian): fold the top byte into the
// low 24 bits, one 24-bit multiply, keep the top kGroupBits bits.
__host__ __device__ inline uint32_t group_bucket(uint32_t x) {
    const uint32_t y = (x ^ (x >> 16)) & 0xFFFFFFu;
    return (y * 0x9E3779u) >> (32 - kGroupBits);
}

// Bucket of an 8-byte window (lo, hi): the high word rotated by 7 bits and
// xor-ed into the low one, then the 4-byte bucket.
__host__ __device__ inline uint32_t group_bucket8(uint32_t lo, uint32_t hi) {
    return group_bucket(lo ^ ((hi << 7) | (hi >> 25)));
}

struct BatchPairDesc {
    DevPlan plan;
    uint64_t cnt_base;       // first (pair, tile) entry of this pair (entries are in kernel order)
    uint32_t text;
    uint32_t tiles;          // entries of this pair: tiles of its text, 0 if m > n
    uint32_t pad_[2];        // 160 bytes: copied to LDS as 16-byte elements
};

// Entries of a pair in the caller's order (for its count and offset).
struct BatchSpan {
    uint64_t cnt_base;
    uint32_t tiles;
    uint32_t kq;  // the pair's index in kernel order (kNoKq when it has no entries)
};
constexpr uint32_t kNoKq = 0xFFFFFFFFu;

struct BatchUnit {
    uint32_t text;
    uint32_t tile;
};

struct BatchArgs {
    const BatchTextDesc *texts;
    const BatchPairDesc *kpairs;   // descriptors in kernel order: pairs with entries, per text contiguous
    const uint32_t *group_tables;  // [groups][kGroupTableWords]
    const BatchUnit *units;
    uint32_t *park;            // [units][kParkMax] parked group hits, sorted
    uint32_t *park_n;          // [units] parked hits, or kParkOverflow
    uint32_t *pt_count;        // [entries] hits of each (pair, tile)
    const uint64_t *pt_offset; // [entries + 1] exclusive prefix of pt_count (write pass)
    const int64_t *shift;      // [pairs in kernel order] output offset of the pair minus
                               // pt_offset of its first entry (write pass)
    uint64_t entries;
    int64_t *out;
    uint64_t cap;
    uint32_t write;
};

// The launch helpers report errors with hipGetLastError, which returns the
// last error of any runtime call on this thread; each clears it first, so
// that an earlier failure of some other call (its own caller's to handle)
// is not taken for a failed launch.
inline void clear_launch_error() { (void)hipGetLastError(); }

hipError_t launch_batch(const BatchArgs &a, int waves, uint32_t n_units, hipStream_t s);
bool batch_waves_supported(int waves);
// Exclusive scan of entries u32 counts into offsets[0..entries] (u64), using
// block_sums (ceil(entries / kScanBlock) u64) as scratch.
constexpr uint32_t kScanBlock = 4096;
hipError_t launch_scan_counts(const uint32_t *counts, uint64_t entries, uint64_t *offsets,
                              uint64_t *block_sums, hipStream_t s);
// Per pair in the caller's order: its count, its output offset (exclusive
// prefix of the counts in that order), and the shift of its entries'
// offsets (entries are scanned in kernel order); block_sums holds
// ceil(n_pairs / kScanBlock) + 1 u64.
hipError_t launch_batch_finalize(const BatchSpan *spans, uint32_t n_pairs,
                                 const uint64_t *offsets, uint64_t entries, uint64_t *counts,
                                 uint64_t *pair_offsets, uint64_t *total, int64_t *shift,
                                 uint64_t *block_sums, hipStream_t s);

// Tile geometry of one kernel configuration.
struct TileConfig {
    int waves;   // waves per workgroup
    int pieces;  // 1 KiB pieces per wave per tile
    int bytes() const { return waves * pieces * kWavePiece; }
};

// Launchers (epsm_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_zero_u64(uint64_t *p, uint64_t count, hipStream_t s);
hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s);
// 2-bit packing of n symbol codes (low two bits of each byte) into
// ceil(n/4) bytes, symbol i at bits 2*(i%4) of byte i/4.
hipError_t launch_pack_dna(const uint8_t *codes, uint64_t n, uint8_t *packed, hipStream_t s);
// *out = the effective alphabet size of text[0, len) (one workgroup; len >= 1).
constexpr uint32_t kAlphabetSample = 65536;  // bytes epsm_estimate_alphabet samples
hipError_t launch_alphabet(const uint8_t *text, uint32_t len, uint32_t *out, hipStream_t s);
// *out = sum of tcnt[0 .. tiles) (one workgroup).
hipError_t launch_sum_tiles(const uint32_t *tcnt, uint32_t tiles, uint64_t *out, hipStream_t s);
// Packed DNA, m >= 16, wide lanes (a.num_tiles tiles of
// dna_wide_tile_symbols() symbols, dna_wide_waves() waves each).  mode 0:
// count per tile into a.tcnt; 1: also per wave into a.wcnt; 2: write the
// positions from a.toff (exclusive tile offsets) and a.wcnt.
uint64_t dna_wide_tile_symbols();
uint32_t dna_wide_waves();
uint32_t dna_wide_slot();  // parked hits per wave (mode 1 writes a.slots)
// Positions per tile (on average, from the output capacity) up to which
// packed searches take the wide-lane write: one per 16 symbols.  Measured
// on 2^32 uniform symbols, its re-read of waves with more hits than their
// slot, written through the LDS stage, beats the 16-start scan's write from
// 256 to 16384 positions per tile (m = 5, 4, 3, 2: 0.67 -> 0.32, 0.81 ->
// 0.61, 0.92 -> 0.68, 1.13 -> 0.99 ms) and ties it at 65536 (m = 1: 2.5 ms).
constexpr uint64_t kDnaWideMaxPerTile = 16384;
hipError_t launch_dna_wide(const ScanArgs &a, int mode, hipStream_t s);
// toff[i] = sum of tcnt[0 .. i) for i <= tiles, and *total = toff[tiles]
// (one workgroup).
hipError_t launch_tile_offsets(const uint32_t *tcnt, uint32_t tiles, uint64_t *toff, uint64_t *total,
                            hipStream_t s);
hipError_t launch_scan(const ScanArgs &a, TileConfig cfg, int grid, hipStream_t s);
// Third step of a two-phase search (after tile_offsets_kernel): slots -> positions.
hipError_t launch_expand(ScanArgs a, TileConfig cfg, hipStream_t s);
bool tile_config_supported(TileConfig cfg);
// The tile configurations compiled into the library, default first; returns
// how many there are (writes at most capacity of them).
int built_tile_configs(TileConfig *out, int capacity);

}  // namespace epsm

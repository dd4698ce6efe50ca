// gfx950 scan and expand kernels of the exact packed string matching search
// (templates; each built tile configuration is instantiated in a translation
// unit of its own, epsm_tile_*.hip).
//
// Layout.  A search runs over "base coordinates": base is the text start
// rounded down to 16 bytes and a text position s is base coordinate s+delta.
// A tile is WAVES * PIECES KiB of base coordinates; wave w of a workgroup
// owns the contiguous PIECES KiB at w*PIECES KiB inside the tile and walks
// it in chunks of U pieces, loading chunk c+1 while it computes chunk c.  In
// piece i lane L owns the 16 start positions [i*1024 + 16L, +16).  Each lane
// loads its 16 bytes plus the following 16 (32 for direct compares of
// patterns longer than 16 bytes) with dwordx4 buffer loads; the buffer descriptor's record count clamps reads at
// the 16-byte-rounded text end, so the (m-1)-byte halo past a piece (Section
// 3.3's reason for wsblend) is just the next bytes of the same coalesced
// stream.
//
// Filter.  Direct variant (m < 16, the job of EPSMa/EPSMb in Sections
// 3.2-3.3): for each of the lane's 16 starts, the 4-byte window at that start
// is cut from two registers with v_alignbyte and compared with the packed
// pattern prefix (masked for m < 4); candidates are checked on the next
// pattern words only when some lane of the wave still has one, so the common
// case costs one alignbyte and one compare per position.  Fingerprint variant
// (m >= 16, EPSMc of Section 3.4): every aligned 8-byte block q is hashed;
// the table entry of the hash lists the offsets j in [0,7] with
// h(p[j..j+7]) = h(block), and start q-j becomes a candidate.  With offsets
// 0..7 and m >= 15 every occurrence is hit by exactly one (block, offset)
// pair.  Candidates are then verified against the whole pattern.
//
// Output.  Each lane parks a 16-bit hit mask per piece in LDS; positions
// leave in ascending order in one of two ways.  Single pass: workgroup b
// owns tile b, publishes the tile's count, and a decoupled look-back over
// the predecessors' status words gives its exclusive prefix, so it writes
// its positions itself.  Two phase: the tile parks its hits in its own
// workspace slot (an ascending list of tile offsets when there are at most
// tile/32 of them, else the raw masks), stores its per-wave and tile counts
// and never waits; one workgroup then scans the tile counts into offsets, and
// a third kernel expands the slots.  No atomics and nothing to clear (in
// count mode, one atomic add per tile into 256 bins cost up to 10% of the
// rate when every tile had hits).  Measured on 1 GiB
// texts, the look-back costs about a quarter of the scan rate even when no
// position is written (a waiting workgroup issues no loads), while the two
// phase scan runs at the count-only rate; single pass stays ahead for dense
// output, whose writes it overlaps with other tiles' reads.
// Other measured constraints: a device-scope atomic on one address
// serialises its callers (one every ~12 ns), so no tile counter is used; the
// look-back's inclusive frontier advances by one window per memory round
// trip, so tiles are large (64 * 128 KiB per round trip); and a persistent
// workgroup that walks several consecutive tiles delays the counts of its
// later tiles behind the writes of its earlier ones, which serialises the
// chain, so workgroups are not persistent.  Count-only searches store one
// count per tile (no atomics, nothing to clear) and a second kernel sums them.
#pragma once

#include "epsm_device.h"

namespace epsm {

// Expand the 16-bit hit masks of one wave's span (piece i of lane L at
// masks[i / 2][tid], half i % 2) into ascending wave-relative offsets staged
// in LDS; sink(stage, fill, done) consumes each full stage, `done` being the
// number of entries consumed before it.  Used on LDS masks by the scan and on
// a slot's masks in global memory by the two-phase expand.
template <int PIECES, int THREADS, class Sink>
__device__ __forceinline__ void expand_masks(const uint32_t (*masks)[THREADS], uint32_t *stage,
                                             int tid, int lane, Sink sink) {
    uint32_t fill = 0, done = 0;
#pragma unroll 1
    for (int piece = 0; piece < PIECES; ++piece) {
        const uint32_t mk = (masks[piece >> 1][tid] >> ((piece & 1) * 16)) & 0xFFFFu;
        const uint32_t c = __popc(mk);
        if (!wave_any(c != 0)) continue;
        const uint32_t incl = wave_incl_scan32(c);
        const uint32_t tot = last_lane(incl);
        if (fill + tot > kStage) {
            sink(stage, fill, done);
            done += fill;
            fill = 0;
        }
        uint32_t at = fill + incl - c;
        const uint32_t rel0 = (uint32_t)piece * kWavePiece + (uint32_t)lane * kPiece;
        uint32_t bits = mk;
        while (bits) {
            const uint32_t k = __builtin_ctz(bits);
            bits &= bits - 1;
            stage[at++] = rel0 + k;
        }
        fill += tot;
    }
    if (fill) sink(stage, fill, done);
}

// Positions of one wave's span to out[obase ...] (entries past cap dropped).
template <int PIECES, int THREADS>
__device__ __forceinline__ void write_tile(const uint32_t (*masks)[THREADS], uint32_t *stage,
                                           const ScanArgs &a, uint64_t obase, int64_t wave_pos0,
                                           int tid, int lane) {
    expand_masks<PIECES, THREADS>(masks, stage, tid, lane,
                                  [&](const uint32_t *st, uint32_t fill, uint32_t done) {
                                      flush_stage(st, fill, a.out, a.cap, obase + done, wave_pos0, lane);
                                  });
}

// Buffer descriptor of a tile; tile_byte is the tile's first byte (its first
// coordinate >> a.shift), a.load_end the readable bytes from a.base.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const ScanArgs &a, uint64_t tile_byte) {
    const uint64_t avail = a.load_end - tile_byte;
    const uint32_t nrec = avail > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)avail;
    return make_rsrc(a.base + tile_byte, nrec);
}

// One workgroup per tile (workgroup index = tile index, no counter).  Every
// tile publishes its count as soon as it is computed, independently of the
// other tiles' look-back and write phases; a look-back only waits on lower
// workgroup indices, which in-order dispatch has already started.
// Six waves per SIMD (at most 80 VGPRs) for the one- and two-load kernels: one more
// resident wave per SIMD than 88 VGPRs would allow, which the streaming
// loads need.  The three-load direct kernel keeps its registers.  Tiles
// whose LDS admits fewer waves (4x32, 16x8, 16x16) do not reach the target;
// their register use is left as it is.
// CNT: the count-mode kernel of a plan held in registers (no tail check),
// which counts the filter's wave masks without per-lane masks.
template <int WAVES, int U, int C, int NL, int VAR, int PK, int NW, bool CNT>
__global__ __launch_bounds__(WAVES * kWave)
__attribute__((amdgpu_waves_per_eu(NL > 2 ? 4 : 6)))
void scan_kernel(ScanArgs a) {
    constexpr int kThreads = WAVES * kWave;
    constexpr int kPieces = U * C;  // pieces per wave per tile
    constexpr uint32_t kWaveSpan = kPieces * kWavePiece;
    constexpr uint32_t kTile = WAVES * kWaveSpan;
    static_assert(U % 2 == 0 && C % 2 == 0, "masks are packed in pairs; chunks ping-pong");
    extern __shared__ __attribute__((aligned(16))) uint16_t s_table[];
    __shared__ uint32_t s_mask[kPieces / 2][kThreads];
    __shared__ uint32_t s_stage[WAVES][kStage];
    __shared__ uint32_t s_wcnt[WAVES];
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

    // coordinates: text bytes, or 2-bit symbols for packed DNA (VAR == 3,
    // four to a byte); a piece is 1024 coordinates either way
    constexpr uint32_t kShift = VAR == 3 ? 2 : 0;
    const uint32_t tile = blockIdx.x;
    const uint64_t tile_start = (uint64_t)tile * kTile;
    const __amdgpu_buffer_rsrc_t rsrc = tile_rsrc(a, tile_start >> kShift);
    const uint32_t lane_off = (uint32_t)wave * kWaveSpan + (uint32_t)lane * kPiece;
    const uint64_t lane_start = tile_start + lane_off;
    const bool edge = tile == 0 || tile == a.num_tiles - 1;
    const bool tail = a.plan.m > (VAR == 3 ? 16u : 4u) * a.plan.nw;
    auto load = [&](uint32_t (&w)[U][NL * 4 + 1], uint32_t off) {
        if constexpr (VAR == 3) load_chunk_dna<U>(w, rsrc, off >> kShift);
        else load_chunk<U, NL>(w, rsrc, off);
    };

    uint32_t wa[U][NL * 4 + 1], wb[U][NL * 4 + 1];
    load(wa, lane_off);
    if constexpr (VAR == 2 || (VAR == 3 && PK == 16)) {
        const uint32_t rows = (1u << a.plan.hash_bits) / 8;  // 16-byte rows of the table
        const u32x4 *src = reinterpret_cast<const u32x4 *>(a.plan.table);
        u32x4 *dst = reinterpret_cast<u32x4 *>(s_table);
        for (uint32_t i = tid; i < rows; i += kThreads) dst[i] = src[i];
        __syncthreads();
    }

    // the loop body is two ping-pong rounds (four chunks), unrolled: with a
    // body of one round the register allocator kept 16 more bytes live in
    // the fingerprint and long-verify kernels and spilled them at 80 VGPRs
    uint32_t cnt = 0, wave_cnt = 0;  // per-lane hits; hits counted per wave (CNT)
    constexpr int kStep = C >= 4 ? 4 : 2;
    static_assert(C % kStep == 0, "whole loop bodies per tile");
#pragma unroll 1
    for (int c0 = 0; c0 < C; c0 += kStep) {
#pragma unroll
        for (int c = c0; c < c0 + kStep; c += 2) {
            load(wb, lane_off + (uint32_t)(c + 1) * U * kWavePiece);
            cnt += process_chunk<U, NL, VAR, PK, NW, CNT, kPieces / 2, kThreads>(
                wa, c, a, s_table, lane_start, edge, tail, s_mask, tid, wave_cnt);
            if (c + 2 < C) load(wa, lane_off + (uint32_t)(c + 2) * U * kWavePiece);
            cnt += process_chunk<U, NL, VAR, PK, NW, CNT, kPieces / 2, kThreads>(
                wb, c + 1, a, s_table, lane_start, edge, tail, s_mask, tid, wave_cnt);
        }
    }
    const uint32_t wtot = CNT ? wave_cnt : wave_sum32(cnt);
    if (lane == 0) s_wcnt[wave] = wtot;
    __syncthreads();
    uint64_t tile_cnt = 0;
#pragma unroll
    for (int i = 0; i < WAVES; ++i) tile_cnt += s_wcnt[i];

    if (CNT || a.write == kWriteNone) {
        // count only: a plain store per tile, summed by one more kernel
        if (tid == 0) a.tcnt[tile] = (uint32_t)tile_cnt;
        return;
    }
    if (a.write == kWriteTwoPhase) {
        // park the hits in the tile's slot; nothing waits on other tiles
        constexpr uint32_t kSlotWords = kTile / 32;  // = words of s_mask
        if (lane == 0) a.wcnt[(size_t)tile * WAVES + wave] = wtot;
        if (tid == 0) a.tcnt[tile] = (uint32_t)tile_cnt;
        if (tile_cnt == 0) return;
        uint32_t *slot = a.slots + (size_t)tile * kSlotWords;
        if (tile_cnt > kSlotWords) {
            const uint32_t *src = &s_mask[0][0];
            for (uint32_t i = tid; i < kSlotWords; i += kThreads) slot[i] = src[i];
            return;
        }
        if (wtot == 0) return;
        uint32_t before = 0;
        for (int i = 0; i < wave; ++i) before += s_wcnt[i];
        uint32_t *dst = slot + before;
        const uint32_t wave_off = (uint32_t)wave * kWaveSpan;
        const uint32_t room = kSlotWords - before;  // the slot's end bounds every write
        expand_masks<kPieces, kThreads>(s_mask, s_stage[wave], tid, lane,
                                        [&](const uint32_t *st, uint32_t fill, uint32_t done) {
                                            flush_list(st, fill, dst + done,
                                                       done < room ? room - done : 0u, wave_off, lane);
                                        });
        return;
    }
    if (wave == 0) {
        const uint64_t excl = look_back(a.status, tile, tile_cnt, lane, a.fault);
        if (lane == 0) {
            s_excl = excl;
            if (tile == a.num_tiles - 1) *a.n_hits = excl + tile_cnt;
        }
        // test hook: a wait on a word no tile publishes gives up after a few
        // polls and sets the fault word; the output is unaffected
        if (a.debug_giveup && tile == 0)
            (void)poll_status(a.status, (int64_t)a.num_tiles, a.fault, kDebugSpinLimit);
    }
    __syncthreads();
    if (wtot == 0) return;
    uint64_t obase = s_excl;
    for (int i = 0; i < wave; ++i) obase += s_wcnt[i];
    const int64_t wave_pos0 = (int64_t)(tile_start + (uint64_t)wave * kWaveSpan) - (int64_t)a.delta;
    write_tile<kPieces, kThreads>(s_mask, s_stage[wave], a, obase, wave_pos0, tid, lane);
}

// Last step of a two-phase search.  Workgroup b expands tiles [b * E, +E),
// E = a.expand_tiles <= kExpandTiles, from the output offset of its first
// tile (tile_offsets_kernel) and the tiles' counts, all loaded in one round
// trip; a run of tiles without hits returns at once.  The offset lists of its
// list tiles are copied as one flattened array, so every entry's load is in
// flight at once rather than one tile's list per memory round trip.  Mask
// tiles go through the same staged expansion as the scan, one after another,
// the next one's masks loaded while the current one is expanded.
template <int WAVES, int PIECES>
__global__ __launch_bounds__(WAVES * kWave) void expand_kernel(ScanArgs a) {
    constexpr int kThreads = WAVES * kWave;
    constexpr uint32_t kWaveSpan = PIECES * kWavePiece;
    constexpr uint32_t kTile = WAVES * kWaveSpan;
    constexpr uint32_t kSlotWords = kTile / 32;
    constexpr int kPairs = PIECES / 2;  // mask words per lane and tile
    static_assert(kExpandTiles * WAVES <= kThreads && kExpandTiles <= kWave, "counts per thread");
    __shared__ uint32_t s_stage[WAVES][kStage];
    __shared__ uint32_t s_mk[WAVES][kPairs][kWave];
    __shared__ uint32_t s_wc[kExpandTiles][WAVES];
    __shared__ uint32_t s_tot[kExpandTiles];
    __shared__ uint32_t s_rend[kExpandTiles], s_lend[kExpandTiles];  // inclusive ends
    __shared__ uint32_t s_dense;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t first = blockIdx.x * a.expand_tiles;  // num_tiles < 2^31
    const uint32_t cnt = min(first + a.expand_tiles, a.num_tiles) - first;
    const uint64_t pos0 = a.toff[first];
    const uint64_t pos_end = a.toff[first + cnt];
    const uint32_t wc = (uint32_t)tid < cnt * WAVES ? a.wcnt[(uint64_t)first * WAVES + tid] : 0u;
    const uint32_t tc = (uint32_t)tid < cnt ? a.tcnt[first + tid] : 0u;
    if (pos_end == pos0) return;  // no hits in these tiles
    if (tid < kExpandTiles * WAVES) (&s_wc[0][0])[tid] = wc;
    if (wave == 0) {
        // per tile: end of its positions (relative to pos0) and of its list
        // in the flattened array (mask tiles add no list entries)
        const bool list = tc <= kSlotWords;
        const uint32_t rend = wave_incl_scan32(tc);
        const uint32_t lend = wave_incl_scan32(list ? tc : 0u);
        const uint64_t dense = ballot(!list);
        if (lane < (int)kExpandTiles) {
            s_tot[lane] = tc;
            s_rend[lane] = rend;
            s_lend[lane] = lend;
        }
        if (lane == 0) s_dense = dense != 0;
    }
    __syncthreads();
    const uint32_t l = s_lend[kExpandTiles - 1];  // list entries in all

    // list tiles: entry e of the flattened array lies in the first tile whose
    // list ends past e; a thread's entries ascend, so its tile index does too
    uint32_t ti = 0;
#pragma unroll 1
    for (uint32_t e0 = 0; e0 < l; e0 += 8 * kThreads) {
        uint32_t v[8];
        uint64_t at[8];
        int64_t base[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t e = e0 + u * kThreads + tid;
            if (e < l)
                while (s_lend[ti] <= e) ++ti;  // ends at the last list tile
            const uint32_t lb = ti ? s_lend[ti - 1] : 0u, rb = ti ? s_rend[ti - 1] : 0u;
            const uint64_t t = (uint64_t)first + ti;
            const uint32_t j = e - lb;
            v[u] = e < l ? a.slots[t * kSlotWords + j] : 0u;
            at[u] = pos0 + rb + j;
            base[u] = (int64_t)(t * kTile) - (int64_t)a.delta;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t e = e0 + u * kThreads + tid;
            if (e < l && at[u] < a.cap) a.out[at[u]] = base[u] + v[u];
        }
    }
    if (!s_dense) return;

    auto next_dense = [&](uint32_t i) {
        while (i < cnt && s_tot[i] <= kSlotWords) ++i;
        return i;
    };
    auto load_masks = [&](uint32_t i, uint32_t (&dst)[kPairs]) {
        const uint32_t *slot = a.slots + ((uint64_t)first + i) * kSlotWords;
#pragma unroll
        for (int p = 0; p < kPairs; ++p) dst[p] = slot[p * kThreads + tid];
    };
    uint32_t pre[kPairs];
    uint32_t nd = next_dense(0);
    if (nd < cnt) load_masks(nd, pre);
#pragma unroll 1
    for (uint32_t i = nd; i < cnt; i = nd) {
        // tile i is the dense tile whose masks are in pre
        const uint64_t t = (uint64_t)first + i;
        const int64_t tile_pos0 = (int64_t)(t * kTile) - (int64_t)a.delta;
        const uint64_t pos = pos0 + (i ? s_rend[i - 1] : 0u);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) s_mk[wave][p][lane] = pre[p];
        nd = next_dense(i + 1);
        if (nd < cnt) load_masks(nd, pre);
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += s_wc[i][w];
        if (s_wc[i][wave])
            write_tile<PIECES, kWave>(s_mk[wave], s_stage[wave], a, pos + before,
                                      tile_pos0 + (int64_t)wave * kWaveSpan, lane, lane);
    }
}

typedef void (*ScanFn)(ScanArgs);

// Chunks of 2 pieces (two or three dwordx4 loads per piece and lane, two
// chunks in flight) keep the kernels within about 100 VGPRs.
template <int WAVES, int PIECES, bool CNT>
static ScanFn pick_direct(const DevPlan &p) {
    constexpr int C = PIECES / 2;
    switch (p.pk) {
        case 2: return scan_kernel<WAVES, 2, C, 2, 1, 2, 1, CNT>;
        case 3: return scan_kernel<WAVES, 2, C, 2, 1, 3, 1, CNT>;
        case 5:
        case 6:
        case 7: return scan_kernel<WAVES, 2, C, 2, 1, 7, 2, CNT>;
        case 8:
            switch (p.nw) {
                case 2: return scan_kernel<WAVES, 2, C, 2, 1, 8, 2, CNT>;
                case 3: return scan_kernel<WAVES, 2, C, 2, 1, 8, 3, CNT>;
                default: return scan_kernel<WAVES, 2, C, 2, 1, 8, 4, CNT>;
            }
        default: break;
    }
    switch (p.nw) {
        case 1: return scan_kernel<WAVES, 2, C, 2, 1, 4, 1, CNT>;
        case 2: return scan_kernel<WAVES, 2, C, 2, 1, 4, 2, CNT>;
        case 3: return scan_kernel<WAVES, 2, C, 2, 1, 4, 3, CNT>;
        default: return scan_kernel<WAVES, 2, C, 2, 1, 4, 4, CNT>;
    }
}

// Kernel of a plan; count_only selects the counting kernels where the
// pattern is held in registers (m <= 4 * nw: no tail check).
template <int WAVES, int PIECES>
static ScanFn pick(const DevPlan &p, bool count_only) {
    constexpr int C = PIECES / 2;
    if (p.variant == 3)
        return p.pk == 16 ? scan_kernel<WAVES, 2, C, 1, 3, 16, 0, false>
                          : scan_kernel<WAVES, 2, C, 1, 3, 4, 0, false>;
    const bool cnt = count_only && p.nl == 2 && p.m <= 4ull * p.nw;
    if (p.variant == 2)
        return cnt ? scan_kernel<WAVES, 2, C, 2, 2, 4, 0, true> : scan_kernel<WAVES, 2, C, 2, 2, 4, 0, false>;
    if (p.nl == 3) return scan_kernel<WAVES, 2, C, 3, 1, 4, 0, false>;
    if (p.pk == 1) return scan_kernel<WAVES, 2, C, 2, 1, 1, 1, false>;
    return cnt ? pick_direct<WAVES, PIECES, true>(p) : pick_direct<WAVES, PIECES, false>(p);
}

typedef void (*ExpandFn)(ScanArgs);

// Scan kernel of a plan and expand kernel, per built tile configuration.
#define EPSM_TILE_FNS(W, P)                              \
    ScanFn scan_fn_##W##x##P(const DevPlan &p, bool count_only); \
    ExpandFn expand_fn_##W##x##P();
EPSM_TILE_FNS(8, 16)
EPSM_TILE_FNS(8, 8)
EPSM_TILE_FNS(4, 16)
EPSM_TILE_FNS(4, 32)
EPSM_TILE_FNS(16, 8)
EPSM_TILE_FNS(16, 16)
#undef EPSM_TILE_FNS

// Body of a tile translation unit: instantiates every scan kernel variant
// and the expand kernel of one tile configuration.
#define EPSM_TILE_TU(W, P)                                                     \
    namespace epsm {                                                           \
    ScanFn scan_fn_##W##x##P(const DevPlan &p, bool count_only) {              \
        return pick<W, P>(p, count_only);                                      \
    }                                                                          \
    ExpandFn expand_fn_##W##x##P() { return expand_kernel<W, P>; }             \
    }

}  // namespace epsm

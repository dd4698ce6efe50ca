// gfx950 kernels of the exact packed string matching scan.
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
template <int WAVES, int U, int C, int NL, int VAR, int PK, int NW>
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
    uint32_t cnt = 0;
    constexpr int kStep = C >= 4 ? 4 : 2;
    static_assert(C % kStep == 0, "whole loop bodies per tile");
#pragma unroll 1
    for (int c0 = 0; c0 < C; c0 += kStep) {
#pragma unroll
        for (int c = c0; c < c0 + kStep; c += 2) {
            load(wb, lane_off + (uint32_t)(c + 1) * U * kWavePiece);
            cnt += process_chunk<U, NL, VAR, PK, NW, kPieces / 2, kThreads>(
                wa, c, a, s_table, lane_start, edge, tail, s_mask, tid);
            if (c + 2 < C) load(wa, lane_off + (uint32_t)(c + 2) * U * kWavePiece);
            cnt += process_chunk<U, NL, VAR, PK, NW, kPieces / 2, kThreads>(
                wb, c + 1, a, s_table, lane_start, edge, tail, s_mask, tid);
        }
    }
    const uint32_t wtot = wave_sum32(cnt);
    if (lane == 0) s_wcnt[wave] = wtot;
    __syncthreads();
    uint64_t tile_cnt = 0;
#pragma unroll
    for (int i = 0; i < WAVES; ++i) tile_cnt += s_wcnt[i];

    if (a.write == kWriteNone) {
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

// One workgroup reads the per-tile counts in chunks of kRunTiles rows of
// kSumThreads tiles: thread i holds tiles c0 + j * kSumThreads + i, j <
// kRunTiles, so every load and store of a wave covers consecutive words.
// The loads are independent buffer loads (zero past the last tile), all in
// flight before the first is used.  A tile holds at most 2^20 hits (tiles are
// at most 2^20 coordinates), a wave's row at most 2^26, a chunk at most 2^34.
constexpr int kSumThreads = 1024;
constexpr int kSumWaves = kSumThreads / kWave;
constexpr uint32_t kRunTiles = 16;
constexpr uint32_t kChunkTiles = kSumThreads * kRunTiles;

__device__ __forceinline__ void load_rows(const uint32_t *tcnt, uint32_t tiles, uint32_t c0, int tid,
                                          uint32_t (&v)[kRunTiles]) {
    const uint32_t left = tiles - c0;
    const __amdgpu_buffer_rsrc_t r = make_rsrc(reinterpret_cast<const uint8_t *>(tcnt + c0),
                                               (left < kChunkTiles ? left : kChunkTiles) * 4u);
#pragma unroll
    for (uint32_t j = 0; j < kRunTiles; ++j)
        v[j] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)((j * kSumThreads + (uint32_t)tid) * 4u), 0, 0);
}

// Sum of the per-tile counts into *out (one workgroup).
__global__ __launch_bounds__(kSumThreads) void sum_tiles_kernel(const uint32_t *tcnt, uint32_t tiles,
                                                                 uint64_t *out) {
    __shared__ uint64_t s_wave[kSumWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint64_t v = 0;
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < tiles; c0 += kChunkTiles) {
        uint32_t r[kRunTiles];
        load_rows(tcnt, tiles, c0, tid, r);
#pragma unroll
        for (uint32_t j = 0; j < kRunTiles; ++j) v += r[j];
    }
    v = wave_sum64(v);
    if (lane == 0) s_wave[wave] = v;
    __syncthreads();
    if (tid == 0) {
        uint64_t total = 0;
#pragma unroll
        for (int i = 0; i < kSumWaves; ++i) total += s_wave[i];
        *out = total;
    }
}

// Exclusive scan of the per-tile counts, toff[i] = sum of tcnt[0 .. i) for
// i <= tiles, and *total = toff[tiles] (one workgroup).  Per chunk: a wave
// scan of each row; the (row, wave) totals in row-major order are scanned by
// the first kRunTiles * kSumWaves / kWave waves; each thread then adds its
// (row, wave) prefix to its in-wave prefix and stores the offsets.
__global__ __launch_bounds__(kSumThreads) void tile_offsets_kernel(const uint32_t *tcnt, uint32_t tiles,
                                                                   uint64_t *toff, uint64_t *total) {
    constexpr int kCells = kRunTiles * kSumWaves;  // (row, wave) totals per chunk
    constexpr int kCellWaves = kCells / kWave;
    static_assert(kCells % kWave == 0 && kCells <= kSumThreads, "one cell per thread");
    __shared__ uint32_t s_cell[kCells];
    __shared__ uint64_t s_pre[kCells];
    __shared__ uint64_t s_part[kCellWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint64_t carry = 0;
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < tiles; c0 += kChunkTiles) {
        uint32_t v[kRunTiles], incl[kRunTiles];
        load_rows(tcnt, tiles, c0, tid, v);
#pragma unroll
        for (uint32_t j = 0; j < kRunTiles; ++j) incl[j] = wave_incl_scan32(v[j]);
        if (lane == kWave - 1) {
#pragma unroll
            for (uint32_t j = 0; j < kRunTiles; ++j) s_cell[j * kSumWaves + wave] = incl[j];
        }
        __syncthreads();
        uint64_t x = 0, xi = 0;
        if (tid < kCells) {
            x = s_cell[tid];
            xi = x;  // inclusive scan of the cells in this wave
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint64_t t = __shfl_up(xi, d, kWave);
                if (lane >= d) xi += t;
            }
            if (lane == kWave - 1) s_part[wave] = xi;
        }
        __syncthreads();
        uint64_t chunk = 0;
#pragma unroll
        for (int i = 0; i < kCellWaves; ++i) chunk += s_part[i];
        if (tid < kCells) {
            uint64_t before = xi - x;
            for (int i = 0; i < wave; ++i) before += s_part[i];
            s_pre[tid] = before;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < kRunTiles; ++j) {
            const uint64_t i = (uint64_t)c0 + j * kSumThreads + (uint32_t)tid;
            if (i < tiles) toff[i] = carry + s_pre[j * kSumWaves + wave] + (incl[j] - v[j]);
        }
        carry += chunk;
        __syncthreads();
    }
    if (tid == 0) {
        toff[tiles] = carry;
        *total = carry;
    }
}

hipError_t launch_tile_offsets(const uint32_t *tcnt, uint32_t tiles, uint64_t *toff, uint64_t *total,
                            hipStream_t s) {
    hipLaunchKernelGGL(tile_offsets_kernel, dim3(1), dim3(kSumThreads), 0, s, tcnt, tiles, toff, total);
    return hipGetLastError();
}

hipError_t launch_sum_tiles(const uint32_t *tcnt, uint32_t tiles, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_tiles_kernel, dim3(1), dim3(kSumThreads), 0, s, tcnt, tiles, out);
    return hipGetLastError();
}

// Packed DNA, m >= 16: the block filter with wide lanes.  A piece is 4096
// symbols (1 KiB); lane L owns starts [64 L, 64 L + 64), the 16 bytes it
// loads (one non-temporal load, no overlap between lanes); the 64 symbols
// after them are lane L + 1's (DPP wave_shl:1), lane 63's the next piece's
// first bytes, one wave-uniform address.  The nine aligned 8-symbol blocks
// at symbols 0, 8, ..., 64 of the run cover the lane's starts: bit j of the
// block at 8i marks start 8i - j.  Candidates are checked per lane, the
// run's words picked by selects (a runtime register index would move the
// run to scratch).
// Modes: kWideCount stores each tile's count; kWideCountWaves also each
// wave's, and parks up to kWideSlot of a wave's hits (offsets in the tile,
// ascending) in its slot; kWideWrite writes the positions of the tiles with
// hits from the tile offsets and wave counts: a wave whose hits fit its slot
// copies them, a wave with more re-scans its span.  Within a piece the
// starts are ordered by lane, then bit, so a lane's hits are consecutive in
// the output and each lane writes its own run.
constexpr int kWideWaves = 8;
constexpr int kWidePieces = 8;                      // pieces per wave and tile
constexpr uint32_t kWidePieceSym = 64 * kWave;      // 4096 symbols = 1 KiB
constexpr uint64_t kWideTileSym = (uint64_t)kWideWaves * kWidePieces * kWidePieceSym;
constexpr int kWideCount = 0, kWideCountWaves = 1, kWideWrite = 2;
constexpr uint32_t kWideSlot = 64;  // parked hit offsets per wave
// write pass: a wave's hits are staged in LDS (offsets in its span) and
// written by consecutive lanes; a piece with more hits than this is
// written lane by lane
constexpr uint32_t kWideStage = 1536;

__device__ __forceinline__ uint32_t pick4(const uint32_t (&w)[9], uint32_t q, int j) {
    // w[q + j] for q in 0..3 (j fixed), without a runtime register index
    const uint32_t a = w[j], b = w[j + 1], c = w[j + 2], d = w[j + 3];
    return q == 0 ? a : q == 1 ? b : q == 2 ? c : d;
}

// Packed DNA, m < 8: every start compared directly, the 16 starts of a word
// at once.  For pattern symbol j the run shifted by j symbols is XOR-ed with
// p[j] repeated in every 2-bit field; start i of word q matches iff field i
// of the OR of these differences over j < m is zero.  The zero fields are
// then gathered into 16 bits (the inverse of a 2-bit Morton spread).
__device__ __forceinline__ uint64_t dna_direct_hits(const uint32_t (&w)[9], const DevPlan &p) {
    uint32_t rep[7], keep[7];  // wave-uniform
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        rep[j] = ((p.pw[0] >> (2 * j)) & 3u) * 0x55555555u;
        keep[j] = (uint32_t)j < p.m ? ~0u : 0u;
    }
    uint64_t hits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t acc = w[q] ^ rep[0];
#pragma unroll
        for (int j = 1; j < 7; ++j)
            acc |= (__builtin_amdgcn_alignbit(w[q + 1], w[q], 2 * j) ^ rep[j]) & keep[j];
        uint32_t z = ~(acc | (acc >> 1)) & 0x55555555u;
        z = (z | (z >> 1)) & 0x33333333u;
        z = (z | (z >> 2)) & 0x0F0F0F0Fu;
        z = (z | (z >> 4)) & 0x00FF00FFu;
        z = (z | (z >> 8)) & 0x0000FFFFu;
        hits |= (uint64_t)z << (16 * q);
    }
    return hits;
}

// BLOCK: 8 (m >= 16, hashed 8-symbol blocks), 4 (8 <= m < 16, 4-symbol
// blocks indexing the table directly) or 0 (m < 8, dna_direct_hits).
template <int MODE, int BLOCK>
__global__ __launch_bounds__(kWideWaves * kWave) void dna_wide_kernel(ScanArgs a) {
    static_assert(BLOCK == 0 || BLOCK == 4 || BLOCK == 8, "direct, 4-symbol or 8-symbol blocks");
    constexpr int kBlocks = BLOCK ? 64 / BLOCK : 0;  // blocks at symbols BLOCK * i, i = 0..kBlocks
    constexpr uint32_t kBlockMask = BLOCK == 8 ? 0xFFFFu : 0xFFu;
    extern __shared__ __attribute__((aligned(16))) uint16_t s_table[];
    __shared__ uint32_t s_wave[kWideWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t tile = blockIdx.x;
    const uint64_t tile_sym = (uint64_t)tile * kWideTileSym;
    uint32_t *slot = a.slots + ((uint64_t)tile * kWideWaves + wave) * kWideSlot;
    uint64_t pos = 0;  // write: output index of this wave's first hit
    uint32_t mine = 0;  // write: this wave's hits
    if constexpr (MODE == kWideWrite) {
        pos = a.toff[tile];
        if (a.toff[tile + 1] == pos) return;  // no hits in this tile (uniform)
        for (int i = 0; i < wave; ++i) pos += a.wcnt[(uint64_t)tile * kWideWaves + i];
        mine = a.wcnt[(uint64_t)tile * kWideWaves + wave];
    }
    const __amdgpu_buffer_rsrc_t rsrc = tile_rsrc(a, tile_sym >> 2);
    if constexpr (BLOCK != 0) {
        const uint32_t rows = (1u << a.plan.hash_bits) / 8;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(a.plan.table);
        u32x4 *dst = reinterpret_cast<u32x4 *>(s_table);
        for (uint32_t i = tid; i < rows; i += kWideWaves * kWave) dst[i] = src[i];
    }
    __syncthreads();  // the last barrier: waves may leave after it
    if constexpr (MODE == kWideWrite) {
        if (mine <= kWideSlot) {
            // the wave's hits are parked: copy them, no text read
            const int64_t p0 = (int64_t)tile_sym - (int64_t)a.delta;
            for (uint32_t i = lane; i < mine; i += kWave)
                if (pos + i < a.cap) a.out[pos + i] = p0 + slot[i];
            return;
        }
    }
    const uint32_t wave_byte = (uint32_t)wave * kWidePieces * (kWidePieceSym / 4);
    const uint32_t lane_byte = wave_byte + (uint32_t)lane * 16;
    const bool edge = tile == 0 || tile == a.num_tiles - 1;
    const uint32_t nw = a.plan.nw;
    auto load = [&](uint32_t (&w)[9], int p) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(lane_byte + p * 1024), 0, kStreamLoad);
        const u32x4 h = __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(wave_byte + (p + 1) * 1024), 0,
                                                              kStreamLoad);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        w[4] = h.x; w[5] = h.y; w[6] = h.z; w[7] = h.w;
        w[8] = 0;
    };
    // hits of the lane's 64 starts in piece p (base coordinate s0 = bit 0)
    auto piece = [&](uint32_t (&w)[9], uint64_t s0) -> uint64_t {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[4 + j] = (uint32_t)__builtin_amdgcn_update_dpp((int)w[4 + j], (int)w[j], 0x130, 0xF, 0xF, false);
        uint64_t cand = 0;
        if constexpr (BLOCK == 0) {
            cand = dna_direct_hits(w, a.plan);
        } else {
            auto entry = [&](uint32_t block) -> uint32_t {
                return s_table[BLOCK == 8 ? fp_hash(block, 0, a.plan.hash_bits) : block];
            };
            cand = entry(w[0] & kBlockMask) & 1u;
#pragma unroll
            for (int i = 1; i <= kBlocks; ++i) {
                constexpr int kPerWord = 16 / BLOCK;
                const uint32_t block = (w[i / kPerWord] >> (2 * BLOCK * (i % kPerWord))) & kBlockMask;
                // bit j -> start BLOCK * i - j: reverse the BLOCK low bits, then shift
                cand |= (uint64_t)(__builtin_bitreverse32(entry(block)) >> (32 - BLOCK))
                        << (BLOCK * i - (BLOCK - 1));
            }
        }
        if (edge) {
            uint32_t lo = 0, hi = 64;
            if (a.delta > s0) lo = a.delta - s0 > 64 ? 64u : (uint32_t)(a.delta - s0);
            if (a.last < s0) hi = 0;
            else if (a.last - s0 < 63) hi = (uint32_t)(a.last - s0) + 1;
            const uint64_t below_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1);
            const uint64_t below_lo = lo >= 64 ? ~0ull : ((1ull << lo) - 1);
            cand &= below_hi & ~below_lo;
        }
        if constexpr (BLOCK == 0) return cand;  // exact already
        uint64_t hits = 0;
        while (cand) {
            const uint32_t k = (uint32_t)__builtin_ctzll(cand);
            cand &= cand - 1;
            const uint32_t q = k >> 4, sh = 2 * (k & 15);
            bool ok = true;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j < (int)nw) {
                    const uint32_t x = __builtin_amdgcn_alignbit(pick4(w, q, j + 1), pick4(w, q, j), sh);
                    ok = ok && (x & a.plan.pmask[j]) == a.plan.pw[j];
                }
            if (ok && a.plan.m > 48) {
                const uint64_t s = s0 + k;
                for (uint64_t j = 48; j < a.plan.m && ok; ++j) {
                    const uint64_t c = s + j;
                    ok = ((a.base[c >> 2] >> (2 * (c & 3))) & 3u) == a.plan.pattern[j];
                }
            }
            hits |= ok ? 1ull << k : 0ull;
        }
        return hits;
    };
    const uint64_t wave_base = tile_sym + (uint64_t)wave * kWidePieces * kWidePieceSym;
    const uint64_t wave_sym = wave_base + (uint64_t)lane * 64;
    // write pass: the wave's LDS stage (after the table), its fill, and the
    // hits already written from this wave's output base `pos`
    uint32_t *stage = reinterpret_cast<uint32_t *>(s_table + (BLOCK ? (1u << a.plan.hash_bits) : 0u)) +
                      (uint32_t)wave * kWideStage;
    const int64_t wave_p0 = (int64_t)wave_base - (int64_t)a.delta;
    uint32_t fill = 0;
    uint64_t done = 0;
    uint32_t cnt = 0, parked = 0;  // parked: the wave's hits so far (count pass for a write)
    auto consume = [&](uint64_t hits, uint64_t s0) {
        const uint32_t c = (uint32_t)__popcll(hits);
        if constexpr (MODE != kWideWrite) {
            cnt += c;
            if constexpr (MODE == kWideCountWaves) {
                if (wave_any(c != 0)) {
                    const uint32_t incl = wave_incl_scan32(c);
                    uint32_t at = parked + (incl - c);
                    parked += last_lane(incl);
                    const uint32_t rel = (uint32_t)(s0 - tile_sym);
                    while (hits) {
                        const uint32_t k = (uint32_t)__builtin_ctzll(hits);
                        hits &= hits - 1;
                        if (at < kWideSlot) slot[at] = rel + k;
                        ++at;
                    }
                }
            }
        } else {
            const uint32_t incl = wave_incl_scan32(c);
            const uint32_t tot = last_lane(incl);
            if (tot == 0) return;
            if (fill + tot > kWideStage) {
                flush_stage(stage, fill, a.out, a.cap, pos + done, wave_p0, lane);
                done += fill;
                fill = 0;
            }
            if (tot > kWideStage) {
                uint64_t at = pos + done + (incl - c);
                const int64_t p0 = (int64_t)s0 - (int64_t)a.delta;
                while (hits) {
                    const uint32_t k = (uint32_t)__builtin_ctzll(hits);
                    hits &= hits - 1;
                    if (at < a.cap) a.out[at] = p0 + k;
                    ++at;
                }
                done += tot;
                return;
            }
            uint32_t at = fill + (incl - c);
            const uint32_t rel = (uint32_t)(s0 - wave_base);
            while (hits) {
                const uint32_t k = (uint32_t)__builtin_ctzll(hits);
                hits &= hits - 1;
                stage[at++] = rel + k;
            }
            fill += tot;
        }
    };
    uint32_t wa[9], wb[9];
    load(wa, 0);
#pragma unroll 1
    for (int p = 0; p < kWidePieces; p += 2) {
        load(wb, p + 1);
        const uint64_t sa = wave_sym + (uint64_t)p * kWidePieceSym;
        consume(piece(wa, sa), sa);
        if (p + 2 < kWidePieces) load(wa, p + 2);
        consume(piece(wb, sa + kWidePieceSym), sa + kWidePieceSym);
    }
    if constexpr (MODE == kWideWrite)
        if (fill) flush_stage(stage, fill, a.out, a.cap, pos + done, wave_p0, lane);
    if constexpr (MODE != kWideWrite) {
        const uint32_t wt = wave_sum32(cnt);
        if constexpr (MODE == kWideCountWaves)
            if (lane == 0) a.wcnt[(uint64_t)tile * kWideWaves + wave] = wt;
        if (lane == 0) s_wave[wave] = wt;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
#pragma unroll
            for (int i = 0; i < kWideWaves; ++i) t += s_wave[i];
            a.tcnt[tile] = t;
        }
    }
}

uint64_t dna_wide_tile_symbols() { return kWideTileSym; }
uint32_t dna_wide_waves() { return kWideWaves; }
uint32_t dna_wide_slot() { return kWideSlot; }

template <int BLOCK>
static void launch_dna_wide_block(const ScanArgs &a, int mode, hipStream_t s) {
    const dim3 grid(a.num_tiles), block(kWideWaves * kWave);
    const size_t table = BLOCK ? (size_t)2 << a.plan.hash_bits : 0;
    const size_t lds = table + (mode == kWideWrite ? (size_t)kWideWaves * kWideStage * sizeof(uint32_t) : 0);
    if (mode == kWideCount) hipLaunchKernelGGL((dna_wide_kernel<kWideCount, BLOCK>), grid, block, lds, s, a);
    else if (mode == kWideCountWaves)
        hipLaunchKernelGGL((dna_wide_kernel<kWideCountWaves, BLOCK>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((dna_wide_kernel<kWideWrite, BLOCK>), grid, block, lds, s, a);
}

hipError_t launch_dna_wide(const ScanArgs &a, int mode, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (a.plan.pk == 16) launch_dna_wide_block<8>(a, mode, s);
    else if (a.plan.pk == 8) launch_dna_wide_block<4>(a, mode, s);
    else launch_dna_wide_block<0>(a, mode, s);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(uint64_t *p, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

// 16 symbols per thread: codes[16i .. 16i+16) -> packed bytes [4i, 4i+4).
__global__ __launch_bounds__(256) void pack_dna_kernel(const uint8_t *codes, uint64_t n,
                                                       uint8_t *packed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t first = i * 16;
    if (first >= n) return;
    uint32_t v = 0;
    for (int t = 0; t < 16; ++t)
        if (first + t < n) v |= (uint32_t)(codes[first + t] & 3u) << (2 * t);
    const uint64_t bytes = (n + 3) / 4;
    for (int b = 0; b < 4; ++b)
        if (4 * i + b < bytes) packed[4 * i + b] = (uint8_t)(v >> (8 * b));
}

hipError_t launch_pack_dna(const uint8_t *codes, uint64_t n, uint8_t *packed, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t threads = (n + 15) / 16;
    hipLaunchKernelGGL(pack_dna_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, codes,
                       n, packed);
    return hipGetLastError();
}

__global__ void set_u64_kernel(uint64_t *p, uint64_t value) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

hipError_t launch_zero_u64(uint64_t *p, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s) {
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, value);
    return hipGetLastError();
}

typedef void (*ScanFn)(ScanArgs);

// Chunks of 2 pieces (two or three dwordx4 loads per piece and lane, two
// chunks in flight) keep the kernels within about 100 VGPRs.
template <int WAVES, int PIECES>
static ScanFn pick(const DevPlan &p) {
    if (p.variant == 3)
        return p.pk == 16 ? scan_kernel<WAVES, 2, PIECES / 2, 1, 3, 16, 0>
                          : scan_kernel<WAVES, 2, PIECES / 2, 1, 3, 4, 0>;
    if (p.variant == 2) return scan_kernel<WAVES, 2, PIECES / 2, 2, 2, 4, 0>;
    if (p.nl == 3) return scan_kernel<WAVES, 2, PIECES / 2, 3, 1, 4, 0>;
    switch (p.pk) {
        case 1: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 1, 1>;
        case 2: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 2, 1>;
        case 3: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 3, 1>;
        case 5:
        case 6:
        case 7: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 7, 2>;
        case 8:
            switch (p.nw) {
                case 2: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 8, 2>;
                case 3: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 8, 3>;
                default: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 8, 4>;
            }
        default: break;
    }
    switch (p.nw) {
        case 1: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 4, 1>;
        case 2: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 4, 2>;
        case 3: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 4, 3>;
        default: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 4, 4>;
    }
}

// Built tiles, default first.  4x32 has the default's 128 KiB tile with half
// the LDS per workgroup (masks and stages of 4 waves), so about twice as many
// workgroups fit on a CU.
static const TileConfig kBuiltTiles[] = {{8, 16}, {8, 8}, {4, 16}, {4, 32}, {16, 8}, {16, 16}};

static ScanFn pick_fn(TileConfig cfg, const DevPlan &p) {
    if (cfg.waves == 8 && cfg.pieces == 16) return pick<8, 16>(p);
    if (cfg.waves == 8 && cfg.pieces == 8) return pick<8, 8>(p);
    if (cfg.waves == 4 && cfg.pieces == 16) return pick<4, 16>(p);
    if (cfg.waves == 4 && cfg.pieces == 32) return pick<4, 32>(p);
    if (cfg.waves == 16 && cfg.pieces == 8) return pick<16, 8>(p);
    if (cfg.waves == 16 && cfg.pieces == 16) return pick<16, 16>(p);
    return nullptr;
}

int built_tile_configs(TileConfig *out, int capacity) {
    const int n = (int)(sizeof(kBuiltTiles) / sizeof(kBuiltTiles[0]));
    for (int i = 0; i < n && i < capacity; ++i) out[i] = kBuiltTiles[i];
    return n;
}

bool tile_config_supported(TileConfig cfg) {
    DevPlan p{};
    p.variant = 1;
    p.nl = 2;
    p.pk = 4;
    return pick_fn(cfg, p) != nullptr;
}

static size_t table_bytes(const DevPlan &p) {
    return (p.variant == 2 || (p.variant == 3 && p.pk == 16)) ? ((size_t)2 << p.hash_bits) : 0;
}

typedef void (*ExpandFn)(ScanArgs);

static ExpandFn pick_expand(TileConfig cfg) {
    if (cfg.waves == 8 && cfg.pieces == 16) return expand_kernel<8, 16>;
    if (cfg.waves == 8 && cfg.pieces == 8) return expand_kernel<8, 8>;
    if (cfg.waves == 4 && cfg.pieces == 16) return expand_kernel<4, 16>;
    if (cfg.waves == 4 && cfg.pieces == 32) return expand_kernel<4, 32>;
    if (cfg.waves == 16 && cfg.pieces == 8) return expand_kernel<16, 8>;
    if (cfg.waves == 16 && cfg.pieces == 16) return expand_kernel<16, 16>;
    return nullptr;
}

hipError_t launch_expand(ScanArgs a, TileConfig cfg, hipStream_t s) {
    ExpandFn fn = pick_expand(cfg);
    if (!fn) return hipErrorInvalidValue;
    // Lists: 8 to kExpandTiles tiles per workgroup, copied together, enough
    // that the grid fits in about one round of resident workgroups (three
    // per CU).  Outputs dense enough that most tiles park masks: one tile
    // each, so that different tiles' masks are expanded in parallel.
    const uint64_t slot_words = (uint64_t)cfg.waves * cfg.pieces * kWavePiece / 32;
    uint32_t e = (uint32_t)((a.num_tiles + kExpandRound - 1) / kExpandRound);
    e = e < 8 ? 8 : (e > kExpandTiles ? kExpandTiles : e);
    a.expand_tiles = a.cap <= (uint64_t)a.num_tiles * (slot_words / 2) ? e : 1;
    const uint32_t grid = (a.num_tiles + a.expand_tiles - 1) / a.expand_tiles;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs &a, TileConfig cfg, int grid, hipStream_t s) {
    ScanFn fn = pick_fn(cfg, a.plan);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * kWave), table_bytes(a.plan), s, a);
    return hipGetLastError();
}

}  // namespace epsm

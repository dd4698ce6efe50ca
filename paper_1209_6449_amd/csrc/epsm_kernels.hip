// gfx950 kernels of the exact packed string matching scan.
//
// Layout.  A search runs over "base coordinates": base is the text start
// rounded down to 16 bytes and a text position s is base coordinate s+delta.
// A tile is WAVES * PIECES KiB of base coordinates; wave w of a workgroup
// owns the contiguous PIECES KiB at w*PIECES KiB inside the tile and walks
// it in chunks of U pieces, loading chunk c+1 while it computes chunk c.  In
// piece i lane L owns the 16 start positions [i*1024 + 16L, +16).  Each lane
// loads its 16 bytes plus the following 16 (32 for long patterns) with
// dwordx4 buffer loads; the buffer descriptor's record count clamps reads at
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
// Output.  Each lane parks a 16-bit hit mask per piece in LDS.  Workgroup b
// owns tile b; it publishes the tile's count and a single-pass decoupled
// look-back over the predecessors' status words gives its exclusive prefix,
// so positions are written in ascending order in one pass over the text.
// Measured constraints shape the schedule: a device-scope atomic on one
// address serialises its callers (one every ~12 ns), so no tile counter is
// used; the inclusive-prefix frontier advances by one look-back window per
// memory round trip, so tiles are large (64 * 128 KiB per round trip);
// and a persistent workgroup that walks several consecutive tiles delays the
// counts of its later tiles behind the writes of its earlier ones, which
// serialises the chain, so workgroups are not persistent.  Count-only
// searches skip the look-back.
#include "epsm_device.h"

namespace epsm {

// Write phase of one tile, run by each wave on its own span: expand the
// parked masks into wave-relative offsets staged in LDS (ascending), and
// flush the stage with consecutive lanes writing consecutive int64 entries.
template <int PIECES, int THREADS>
__device__ __forceinline__ void write_tile(const uint32_t (*s_mask)[THREADS], uint32_t *stage,
                                           const ScanArgs &a, uint64_t obase, int64_t wave_pos0,
                                           int tid, int lane) {
    uint32_t fill = 0;
#pragma unroll 1
    for (int piece = 0; piece < PIECES; ++piece) {
        const uint32_t mk = (s_mask[piece >> 1][tid] >> ((piece & 1) * 16)) & 0xFFFFu;
        const uint32_t c = __popc(mk);
        if (!wave_any(c != 0)) continue;
        const uint32_t incl = wave_incl_scan32(c, lane);
        const uint32_t tot = __shfl(incl, kWave - 1, kWave);
        if (fill + tot > kStage) {
            flush_stage(stage, fill, a.out, a.cap, obase, wave_pos0, lane);
            obase += fill;
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
    if (fill) flush_stage(stage, fill, a.out, a.cap, obase, wave_pos0, lane);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const ScanArgs &a, uint64_t tile_start) {
    const uint64_t avail = a.load_end - tile_start;
    const uint32_t nrec = avail > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)avail;
    return make_rsrc(a.base + tile_start, nrec);
}

// One workgroup per tile (workgroup index = tile index, no counter).  Every
// tile publishes its count as soon as it is computed, independently of the
// other tiles' look-back and write phases; a look-back only waits on lower
// workgroup indices, which in-order dispatch has already started.
template <int WAVES, int U, int C, int NL, int VAR, int PK, int NW>
__global__ __launch_bounds__(WAVES * kWave, 4) void scan_kernel(ScanArgs a) {
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

    const uint32_t tile = blockIdx.x;
    const uint64_t tile_start = (uint64_t)tile * kTile;
    const __amdgpu_buffer_rsrc_t rsrc = tile_rsrc(a, tile_start);
    const uint32_t lane_off = (uint32_t)wave * kWaveSpan + (uint32_t)lane * kPiece;
    const uint64_t lane_start = tile_start + lane_off;
    const bool edge = tile == 0 || tile == a.num_tiles - 1;
    const bool tail = a.plan.m > 4u * a.plan.nw;

    uint32_t wa[U][NL * 4 + 1], wb[U][NL * 4 + 1];
    load_chunk<U, NL>(wa, rsrc, lane_off);
    if constexpr (VAR == 2) {
        const uint32_t rows = (1u << a.plan.hash_bits) / 8;  // 16-byte rows of the table
        const u32x4 *src = reinterpret_cast<const u32x4 *>(a.plan.table);
        u32x4 *dst = reinterpret_cast<u32x4 *>(s_table);
        for (uint32_t i = tid; i < rows; i += kThreads) dst[i] = src[i];
        __syncthreads();
    }

    uint32_t cnt = 0;
#pragma unroll 1
    for (int c = 0; c < C; c += 2) {
        load_chunk<U, NL>(wb, rsrc, lane_off + (uint32_t)(c + 1) * U * kWavePiece);
        cnt += process_chunk<U, NL, VAR, PK, NW, kPieces / 2, kThreads>(
            wa, c, a, s_table, lane_start, edge, tail, s_mask, tid);
        if (c + 2 < C) load_chunk<U, NL>(wa, rsrc, lane_off + (uint32_t)(c + 2) * U * kWavePiece);
        cnt += process_chunk<U, NL, VAR, PK, NW, kPieces / 2, kThreads>(
            wb, c + 1, a, s_table, lane_start, edge, tail, s_mask, tid);
    }
    const uint32_t wtot = wave_sum32(cnt);
    if (lane == 0) s_wcnt[wave] = wtot;
    __syncthreads();
    uint64_t tile_cnt = 0;
#pragma unroll
    for (int i = 0; i < WAVES; ++i) tile_cnt += s_wcnt[i];

    if (!a.write) {
        // count only: no ordering needed; spread the adds over kCountBins words
        if (tid == 0 && tile_cnt)
            atomicAdd((unsigned long long *)&a.bins[tile & (kCountBins - 1)],
                      (unsigned long long)tile_cnt);
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

// Sum of the count bins into *out (one workgroup of kCountBins threads).
__global__ __launch_bounds__(kCountBins) void sum_bins_kernel(const uint64_t *bins, uint64_t *out) {
    __shared__ uint64_t s_part[kCountBins / kWave];
    const int tid = threadIdx.x;
    const uint64_t v = wave_sum64(bins[tid]);
    if ((tid & (kWave - 1)) == 0) s_part[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        uint64_t total = 0;
        for (int i = 0; i < kCountBins / kWave; ++i) total += s_part[i];
        *out = total;
    }
}

hipError_t launch_sum_bins(const uint64_t *bins, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_bins_kernel, dim3(1), dim3(kCountBins), 0, s, bins, out);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(uint64_t *p, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
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
    if (p.variant == 2) return scan_kernel<WAVES, 2, PIECES / 2, 3, 2, 4, 0>;
    if (p.nl == 3) return scan_kernel<WAVES, 2, PIECES / 2, 3, 1, 4, 0>;
    switch (p.pk) {
        case 1: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 1, 1>;
        case 2: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 2, 1>;
        case 3: return scan_kernel<WAVES, 2, PIECES / 2, 2, 1, 3, 1>;
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
    return p.variant == 2 ? ((size_t)2 << p.hash_bits) : 0;
}

int scan_blocks_per_cu(TileConfig cfg, const DevPlan &p) {
    ScanFn fn = pick_fn(cfg, p);
    if (!fn) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, cfg.waves * kWave,
                                                     table_bytes(p)) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_scan(const ScanArgs &a, TileConfig cfg, int grid, hipStream_t s) {
    ScanFn fn = pick_fn(cfg, a.plan);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * kWave), table_bytes(a.plan), s, a);
    return hipGetLastError();
}

}  // namespace epsm

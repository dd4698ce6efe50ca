// gfx950 kernels of the exact packed string matching search other than the
// scan and expand templates (epsm_scan.h): tile-count sums and offsets, the
// packed-DNA wide-lane kernel, small helpers, and the launchers.
#include "epsm_scan.h"

namespace epsm {
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
    clear_launch_error();
    hipLaunchKernelGGL(tile_offsets_kernel, dim3(1), dim3(kSumThreads), 0, s, tcnt, tiles, toff, total);
    return hipGetLastError();
}

hipError_t launch_sum_tiles(const uint32_t *tcnt, uint32_t tiles, uint64_t *out, hipStream_t s) {
    clear_launch_error();
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
    clear_launch_error();
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
    clear_launch_error();
    if (n == 0) return hipSuccess;
    const uint64_t threads = (n + 15) / 16;
    hipLaunchKernelGGL(pack_dna_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, codes,
                       n, packed);
    return hipGetLastError();
}

// Effective alphabet of text[0, len): one workgroup histograms the bytes in
// LDS, then *out = round(len^2 / sum_c count_c^2), clamped to 1..256.
__global__ __launch_bounds__(256) void alphabet_kernel(const uint8_t *text, uint32_t len, uint32_t *out) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t part[4];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < len; i += 256) atomicAdd(&hist[text[i]], 1u);
    __syncthreads();
    const uint64_t c = hist[tid];
    uint64_t sq = c * c;
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if ((tid & 63) == 0) part[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
        const uint64_t sum = part[0] + part[1] + part[2] + part[3];
        const uint64_t l2 = (uint64_t)len * len;
        uint64_t v = (l2 + sum / 2) / sum;
        *out = (uint32_t)(v < 1 ? 1 : (v > 256 ? 256 : v));
    }
}

hipError_t launch_alphabet(const uint8_t *text, uint32_t len, uint32_t *out, hipStream_t s) {
    clear_launch_error();
    hipLaunchKernelGGL(alphabet_kernel, dim3(1), dim3(256), 0, s, text, len, out);
    return hipGetLastError();
}

__global__ void set_u64_kernel(uint64_t *p, uint64_t value) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

hipError_t launch_zero_u64(uint64_t *p, uint64_t count, hipStream_t s) {
    clear_launch_error();
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t value, hipStream_t s) {
    clear_launch_error();
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, value);
    return hipGetLastError();
}

// Built tiles, default first.  4x32 has the default's 128 KiB tile with half
// the LDS per workgroup (masks and stages of 4 waves), so about twice as many
// workgroups fit on a CU.
static const TileConfig kBuiltTiles[] = {{8, 16}, {8, 8}, {4, 16}, {4, 32}, {16, 8}, {16, 16}};

static ScanFn pick_fn(TileConfig cfg, const DevPlan &p, bool count_only = false) {
    if (cfg.waves == 8 && cfg.pieces == 16) return scan_fn_8x16(p, count_only);
    if (cfg.waves == 8 && cfg.pieces == 8) return scan_fn_8x8(p, count_only);
    if (cfg.waves == 4 && cfg.pieces == 16) return scan_fn_4x16(p, count_only);
    if (cfg.waves == 4 && cfg.pieces == 32) return scan_fn_4x32(p, count_only);
    if (cfg.waves == 16 && cfg.pieces == 8) return scan_fn_16x8(p, count_only);
    if (cfg.waves == 16 && cfg.pieces == 16) return scan_fn_16x16(p, count_only);
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

static ExpandFn pick_expand(TileConfig cfg) {
    if (cfg.waves == 8 && cfg.pieces == 16) return expand_fn_8x16();
    if (cfg.waves == 8 && cfg.pieces == 8) return expand_fn_8x8();
    if (cfg.waves == 4 && cfg.pieces == 16) return expand_fn_4x16();
    if (cfg.waves == 4 && cfg.pieces == 32) return expand_fn_4x32();
    if (cfg.waves == 16 && cfg.pieces == 8) return expand_fn_16x8();
    if (cfg.waves == 16 && cfg.pieces == 16) return expand_fn_16x16();
    return nullptr;
}

hipError_t launch_expand(ScanArgs a, TileConfig cfg, hipStream_t s) {
    clear_launch_error();
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
    clear_launch_error();
    ScanFn fn = pick_fn(cfg, a.plan, a.write == kWriteNone);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * kWave), table_bytes(a.plan), s, a);
    return hipGetLastError();
}

}  // namespace epsm

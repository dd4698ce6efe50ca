// Batched search: many (text, pattern) pairs in one stream-ordered submission.
//
// Work is cut into units, one unit = one tile of one text.  The unit's
// workgroup loads the tile once (each lane 16 bytes plus a 32-byte halo) and
// runs every pattern aimed at that text over it, so a text read from HBM
// serves all of its patterns.  Output is pair-major: pair k's positions,
// ascending, fill d_out[offsets[k] .. offsets[k] + counts[k]).  That order is
// produced in three steps: a count pass writes the hits of every
// (pair, tile) entry, a device exclusive scan turns the entries (in pair
// order) into output offsets, and a write pass recomputes only the entries
// that have hits and writes their positions.  No step needs a host round
// trip, so the whole sequence can be captured once into a graph.
#include "epsm_device.h"

namespace epsm {

constexpr int kBatchNL = 3;  // 48 bytes per lane: any m <= 32 verified from registers

// Mask of one lane piece for a runtime-described pattern.
__device__ __forceinline__ uint32_t any_mask(const uint32_t (&w)[kBatchNL * 4 + 1], const DevPlan &p) {
    if (p.variant == 2) return fingerprint_mask<kBatchNL>(w, p, p.table);
    if (p.nl == 3) return direct_mask<kBatchNL, 4, 0>(w, p);
    switch (p.pk) {
        case 1: return direct_mask<kBatchNL, 1, 1>(w, p);
        case 2: return direct_mask<kBatchNL, 2, 1>(w, p);
        case 3: return direct_mask<kBatchNL, 3, 1>(w, p);
        default: break;
    }
    switch (p.nw) {
        case 1: return direct_mask<kBatchNL, 4, 1>(w, p);
        case 2: return direct_mask<kBatchNL, 4, 2>(w, p);
        case 3: return direct_mask<kBatchNL, 4, 3>(w, p);
        default: return direct_mask<kBatchNL, 4, 4>(w, p);
    }
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void batch_kernel(BatchArgs a) {
    constexpr uint32_t kTileB = WAVES * kWavePiece;
    __shared__ uint32_t s_wcnt[WAVES];
    __shared__ uint32_t s_stage[WAVES][kStage];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

    const BatchUnit unit = a.units[blockIdx.x];
    const BatchTextDesc t = a.texts[unit.text];
    const uint64_t tile_start = (uint64_t)unit.tile * kTileB;
    const uint64_t avail = t.load_end - tile_start;
    const uint32_t nrec = avail > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)avail;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(t.base + tile_start, nrec);
    const uint32_t lane_off = (uint32_t)wave * kWavePiece + (uint32_t)lane * kPiece;
    const uint64_t s0 = tile_start + lane_off;

    uint32_t w[kBatchNL * 4 + 1];
#pragma unroll
    for (int l = 0; l < kBatchNL; ++l) {
        const u32x4 v = load16(rsrc, lane_off + l * kPiece);
        w[4 * l + 0] = v.x;
        w[4 * l + 1] = v.y;
        w[4 * l + 2] = v.z;
        w[4 * l + 3] = v.w;
    }
    w[kBatchNL * 4] = 0;

    const int64_t wave_pos0 = (int64_t)(tile_start + (uint64_t)wave * kWavePiece) - (int64_t)t.delta;
#pragma unroll 1
    for (uint32_t pi = t.pair_begin; pi < t.pair_end; ++pi) {
        const uint32_t pidx = a.pair_order[pi];
        const BatchPairDesc &pd = a.pairs[pidx];
        if (pd.tiles == 0) continue;  // m > n: the pair has no entries
        const uint64_t entry = pd.cnt_base + unit.tile;
        if (a.write && a.pt_count[entry] == 0) continue;
        const DevPlan &p = pd.plan;
        uint32_t mk = any_mask(w, p);
        const uint64_t last = t.delta + t.n - p.m;  // m <= n here
        if (tile_start + kTileB > last || tile_start < t.delta) mk &= valid_mask(s0, t.delta, last);
        if (p.m > 4u * p.nw && wave_any(mk != 0))
            mk = tail_check(mk, s0, t.base, p.pattern, p.m, 4u * p.nw);
        const uint32_t c = __popc(mk);
        const uint32_t incl = wave_incl_scan32(c);
        const uint32_t wtot = last_lane(incl);
        if (lane == 0) s_wcnt[wave] = wtot;
        __syncthreads();
        if (!a.write) {
            if (tid == 0) {
                uint32_t total = 0;
#pragma unroll
                for (int i = 0; i < WAVES; ++i) total += s_wcnt[i];
                a.pt_count[entry] = total;
            }
        } else if (wtot) {
            uint64_t obase = a.pt_offset[entry];
            for (int i = 0; i < wave; ++i) obase += s_wcnt[i];
            uint32_t at = incl - c;
            const uint32_t rel0 = (uint32_t)lane * kPiece;
            uint32_t bits = mk;
            while (bits) {
                const uint32_t k = __builtin_ctz(bits);
                bits &= bits - 1;
                s_stage[wave][at++] = rel0 + k;
            }
            flush_stage(s_stage[wave], wtot, a.out, a.cap, obase, wave_pos0, lane);
        }
        __syncthreads();  // s_wcnt is rewritten by the next pattern
    }
}

bool batch_waves_supported(int waves) { return waves == 4 || waves == 8 || waves == 16; }

hipError_t launch_batch(const BatchArgs &a, int waves, uint32_t n_units, hipStream_t s) {
    if (n_units == 0) return hipSuccess;
    switch (waves) {
        case 4: hipLaunchKernelGGL(batch_kernel<4>, dim3(n_units), dim3(4 * kWave), 0, s, a); break;
        case 8: hipLaunchKernelGGL(batch_kernel<8>, dim3(n_units), dim3(8 * kWave), 0, s, a); break;
        case 16: hipLaunchKernelGGL(batch_kernel<16>, dim3(n_units), dim3(16 * kWave), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- exclusive scan of the (pair, tile) counts ------------------------------
// kScanBlock entries per workgroup of 256 threads (16 per thread).

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t *counts, uint64_t entries,
                                                          uint64_t *block_sums) {
    __shared__ uint64_t s_part[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t v = 0;
    for (uint32_t i = threadIdx.x; i < kScanBlock; i += 256) {
        const uint64_t j = base + i;
        if (j < entries) v += counts[j];
    }
    v = wave_sum64(v);
    if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

// Exclusive scan of block_sums in place by one workgroup; the grand total is
// written to offsets[entries].
__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint64_t *block_sums, uint64_t n_blocks,
                                                           uint64_t *offsets, uint64_t entries) {
    __shared__ uint64_t s_wave[16];
    __shared__ uint64_t s_carry;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < n_blocks; base += 1024) {
        const uint64_t j = base + tid;
        const uint64_t v = j < n_blocks ? block_sums[j] : 0;
        uint64_t x = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint64_t t = __shfl_up(x, d, kWave);
            if (lane >= d) x += t;
        }
        if (lane == kWave - 1) s_wave[wave] = x;
        __syncthreads();
        uint64_t before = s_carry;
        for (int w2 = 0; w2 < wave; ++w2) before += s_wave[w2];
        if (j < n_blocks) block_sums[j] = before + x - v;
        __syncthreads();
        if (tid == 1023) s_carry = before + x;
        __syncthreads();
    }
    if (tid == 0) offsets[entries] = s_carry;
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const uint32_t *counts, uint64_t entries,
                                                         const uint64_t *block_sums, uint64_t *offsets) {
    __shared__ uint64_t s_wave[4];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)tid * 16;
    uint32_t v[16];
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < entries ? counts[base + i] : 0u;
        sum += v[i];
    }
    uint64_t x = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t t = __shfl_up(x, d, kWave);
        if (lane >= d) x += t;
    }
    if (lane == kWave - 1) s_wave[wave] = x;
    __syncthreads();
    uint64_t run = block_sums[blockIdx.x] + x - sum;
    for (int w2 = 0; w2 < wave; ++w2) run += s_wave[w2];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (base + i < entries) offsets[base + i] = run;
        run += v[i];
    }
}

hipError_t launch_scan_counts(const uint32_t *counts, uint64_t entries, uint64_t *offsets,
                              uint64_t *block_sums, hipStream_t s) {
    const uint64_t blocks = (entries + kScanBlock - 1) / kScanBlock;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (blocks) hipLaunchKernelGGL(scan_reduce_kernel, dim3((uint32_t)blocks), dim3(256), 0, s,
                                   counts, entries, block_sums);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, block_sums, blocks, offsets,
                       entries);
    if (blocks) hipLaunchKernelGGL(scan_apply_kernel, dim3((uint32_t)blocks), dim3(256), 0, s,
                                   counts, entries, block_sums, offsets);
    return hipGetLastError();
}

__global__ void batch_finalize_kernel(const BatchPairDesc *pairs, uint32_t n_pairs,
                                      const uint64_t *offsets, uint64_t entries, uint64_t *counts,
                                      uint64_t *pair_offsets, uint64_t *total) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_pairs) {
        const uint64_t b = pairs[k].cnt_base;
        const uint64_t begin = offsets[b], end = offsets[b + pairs[k].tiles];
        pair_offsets[k] = begin;
        counts[k] = end - begin;
    }
    if (k == 0 && total) *total = offsets[entries];
}

hipError_t launch_batch_finalize(const BatchPairDesc *pairs, uint32_t n_pairs,
                                 const uint64_t *offsets, uint64_t entries, uint64_t *counts,
                                 uint64_t *pair_offsets, uint64_t *total, hipStream_t s) {
    const uint32_t blocks = n_pairs ? (n_pairs + 255) / 256 : 1;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(blocks), dim3(256), 0, s, pairs, n_pairs, offsets,
                       entries, counts, pair_offsets, total);
    return hipGetLastError();
}

}  // namespace epsm

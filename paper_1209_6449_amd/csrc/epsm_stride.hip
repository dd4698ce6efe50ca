// Strided fingerprint filter for long patterns: EPSMc (Section 3.4) with the
// stride it is defined with, one inspected block per S text bytes.
//
// With S a power of two, 256 <= S <= m - 7, only the aligned 8-byte blocks at
// multiples of S are read.  An occurrence at s has exactly one such block q
// with s <= q < s + S, and q + 8 <= s + m, so the block lies inside the
// occurrence at pattern offset j = q - s in [0, S).  The plan's table lists,
// for each hash value, the offsets j whose pattern block p[j..j+7] hashes
// there; a block of hash h makes q - j a candidate for every listed j whose
// pattern block equals the text block, and a candidate is checked against the
// whole pattern.  Text lines between inspected blocks are never fetched, so
// the scan moves about one 128-byte line per S bytes of text, plus the
// candidates' checks.
//
// Work and order.  Lane L of wave w of workgroup t inspects the blocks
// b = ((t * waves + w) * 64 + L) * kStrideBlocksPerLane + i, in order; a block
// lists its candidates by descending j, i.e. ascending s.  Positions are thus
// ascending in (t, w, L, i, s).  A count pass stores each workgroup's hits;
// after an exclusive scan of those counts, the write pass (only workgroups
// with hits) recomputes the candidates, counts a lane's hits once more for
// its offset in the wave, and writes them.  Candidates are checked by the
// whole wave together, so a long pattern costs about m / 512 memory round
// trips per check instead of m.
#include "epsm_device.h"

namespace epsm {

// Exact check of the whole pattern at base coordinate s by the whole wave:
// lane L compares bytes L, L + 64, ... (consecutive lanes read consecutive
// bytes), eight loads in flight per lane, stopping at the first chunk with a
// mismatch.  s is the same on every lane.
__device__ __forceinline__ bool wave_check(const uint8_t *base, uint64_t s, const uint8_t *pattern,
                                           uint64_t m, int lane) {
    const uint8_t *t = base + s;
    for (uint64_t j0 = 0; j0 < m; j0 += 8 * kWave) {
        uint32_t tv[8], pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t j = j0 + (uint64_t)u * kWave + lane;
            tv[u] = j < m ? t[j] : 0u;
            pv[u] = j < m ? pattern[j] : 0u;
        }
        bool ok = true;
#pragma unroll
        for (int u = 0; u < 8; ++u) ok = ok && tv[u] == pv[u];
        if (wave_any(!ok)) return false;
    }
    return true;
}

// Visit the hits of each lane, in ascending position, calling hit(s) on the
// lane that owns s.  A listed offset j is a candidate only if the pattern
// block p[j..j+7] equals the text block (not only its hash).  Each lane walks
// its block's list until it holds a candidate; the wave then checks the held
// candidates one at a time together, and the lanes walk on.  Called by full
// waves (the checks are wave-wide).
template <class Hit>
__device__ __forceinline__ void stride_wave(const StrideArgs &a, __amdgpu_buffer_rsrc_t rsrc,
                                            uint64_t tile_q0, uint64_t b0, const uint16_t *s_start,
                                            const uint16_t *s_off, const uint2 *s_blk, int lane,
                                            Hit hit) {
#pragma unroll 1
    for (uint32_t i = 0; i < kStrideBlocksPerLane; ++i) {
        const uint64_t b = b0 + i;
        uint64_t q = 0;
        uint32_t lo = 0, hi = 0;
        int first = 0, cur = -1;
        if (b < a.num_blocks) {
            q = (a.first_block + b) * a.stride;
            const uint32_t off = (uint32_t)(q - tile_q0);
            lo = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off, 0, 0);
            hi = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off + 4, 0, 0);
            const uint32_t h = fp_hash(lo, hi, a.hash_bits);
            first = s_start[h];
            cur = (int)s_start[h + 1] - 1;
        }
#pragma unroll 1
        for (;;) {
            bool have = false;
            uint64_t s = 0;
            while (cur >= first) {  // descending j: ascending s
                const int idx = cur--;
                const uint2 pb = s_blk[idx];
                if (pb.x != lo || pb.y != hi) continue;
                const uint64_t j = s_off[idx];
                if (j > q) continue;  // s would be negative
                const uint64_t sc = q - j;
                if (sc < a.delta || sc > a.last) continue;
                s = sc;
                have = true;
                break;
            }
            uint64_t held = ballot(have);
            if (held == 0) break;
            while (held) {
                const int owner = __builtin_ctzll(held);
                held &= held - 1;
                const uint32_t so_hi = (uint32_t)__builtin_amdgcn_readlane((int)(s >> 32), owner);
                const uint32_t so_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s, owner);
                const uint64_t so = ((uint64_t)so_hi << 32) | so_lo;
                const bool ok = wave_check(a.base, so, a.pattern, a.m, lane);
                if (lane == owner && ok) hit(s);
            }
        }
    }
}

__global__ __launch_bounds__(kStrideThreads) void stride_kernel(StrideArgs a) {
    // LDS: [S] pattern blocks (u32 pairs) in offset order, then [2^k + 1]
    // bucket starts and [S] offsets (u16)
    extern __shared__ __attribute__((aligned(16))) uint2 s_blk[];
    __shared__ uint32_t s_wave[kStrideWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t tile = blockIdx.x;
    // the write pass skips workgroups without hits: their blocks are not read again
    if (a.write && a.tile_count[tile] == 0) return;
    const uint32_t buckets = 1u << a.hash_bits;
    const uint32_t S = (uint32_t)a.stride;
    for (uint32_t i = tid; i < S; i += kStrideThreads) s_blk[i] = a.blocks[i];
    uint16_t *s_tab = reinterpret_cast<uint16_t *>(s_blk + S);
    const uint32_t tab_words = buckets + 1 + S;
    for (uint32_t i = tid; i < tab_words; i += kStrideThreads) s_tab[i] = a.table[i];
    __syncthreads();
    const uint16_t *s_start = s_tab, *s_off = s_tab + buckets + 1;

    // the workgroup's blocks: one buffer descriptor from its first block
    const uint64_t tb0 = (uint64_t)tile * kStrideBlocksPerTile;
    const uint64_t tile_q0 = (a.first_block + tb0) * a.stride;
    const uint64_t avail = a.load_end > tile_q0 ? a.load_end - tile_q0 : 0;
    const __amdgpu_buffer_rsrc_t rsrc =
        make_rsrc(a.base + tile_q0, avail > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)avail);
    const uint64_t b0 = tb0 + (uint64_t)tid * kStrideBlocksPerLane;

    uint32_t c = 0;
    stride_wave(a, rsrc, tile_q0, b0, s_start, s_off, s_blk, lane, [&](uint64_t) { ++c; });
    if (!a.write) {
        const uint32_t wt = wave_sum32(c);
        if (lane == 0) s_wave[wave] = wt;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int i = 0; i < kStrideWaves; ++i) t += s_wave[i];
            a.tile_count[tile] = t;
        }
        return;
    }
    const uint32_t incl = wave_incl_scan32(c);
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint64_t pos = a.tile_offset[tile] + incl - c;
    for (int i = 0; i < wave; ++i) pos += s_wave[i];
    stride_wave(a, rsrc, tile_q0, b0, s_start, s_off, s_blk, lane, [&](uint64_t s) {
        if (pos < a.cap) a.out[pos] = (int64_t)(s - a.delta);
        ++pos;
    });
}

__global__ void copy_u64_kernel(const uint64_t *src, uint64_t *dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = *src;
}

hipError_t launch_stride(const StrideArgs &a, uint32_t tiles, hipStream_t s) {
    clear_launch_error();
    if (tiles == 0) return hipSuccess;
    const size_t lds =
        a.stride * sizeof(uint2) + ((size_t)(1u << a.hash_bits) + 1 + a.stride) * sizeof(uint16_t);
    hipLaunchKernelGGL(stride_kernel, dim3(tiles), dim3(kStrideThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_copy_u64(const uint64_t *src, uint64_t *dst, hipStream_t s) {
    clear_launch_error();
    hipLaunchKernelGGL(copy_u64_kernel, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

}  // namespace epsm

// Batched search: many (text, pattern) pairs in one stream-ordered submission.
//
// Work is cut into units, one unit = one tile of one text.  The unit's
// workgroup loads the tile once (each lane its 16 bytes, the 32-byte halo
// from its neighbours) and runs every pattern aimed at that text over it, so
// a text read from HBM serves all of its patterns.  Output is pair-major:
// pair k's positions, ascending, fill d_out[offsets[k] .. offsets[k] +
// counts[k]).  That order is produced in three steps: a count pass writes
// the hits of every (pair, tile) entry (and lists the unit's hits of grouped
// patterns, up to kParkMax), a device exclusive scan turns the entries (in
// kernel order, a pair's tiles consecutive) into offsets and a scan of the
// pairs' totals in the caller's order gives each pair its output offset and
// shift, and a write pass places the listed hits and recomputes only the
// other entries that have hits.  No step needs a host round trip, so the
// whole sequence can be captured once into a graph.
#include "epsm_device.h"

namespace epsm {

constexpr int kBatchNL = 3;  // 48 bytes per lane: any m <= 32 verified from registers
constexpr uint32_t kPairChunk = 32;  // pair descriptors staged in LDS at a time

// Mask of one lane piece for a runtime-described pattern.  Plans with a
// 64-bit prefix (pk 5..8) are filtered on their first word and verified:
// this kernel holds every variant at once, and the 64-bit variants cost
// more registers than the occupancy the batch needs allows (measured: 105
// -> 153 VGPRs when they were added).
// WIDE: plans with three loads per lane (m > 16) compare up to 32 bytes
// from registers; otherwise their first 16, and the tail check reads the
// rest of the pattern from device memory (a batch uploads the pattern of
// every plan with m > 16).  The write pass, which runs only entries with
// hits, takes the narrow form to stay at six waves per SIMD.
// F gives the plan fields the choice branches on (and the first pattern
// word): PlanFields reads them from the plan (in LDS) where they are used,
// HeldFields holds them in scalar registers, read together beforehand.
struct PlanFields {
    const DevPlan &p;
    __device__ uint32_t var() const { return p.variant; }
    __device__ uint32_t nl() const { return p.nl; }
    __device__ uint32_t pk() const { return p.pk; }
    __device__ uint32_t nw() const { return p.nw; }
    __device__ uint32_t pw0() const { return p.pw[0]; }
};
struct HeldFields {
    uint32_t var_, nl_, pk_, nw_, pw0_;
    __device__ uint32_t var() const { return var_; }
    __device__ uint32_t nl() const { return nl_; }
    __device__ uint32_t pk() const { return pk_; }
    __device__ uint32_t nw() const { return nw_; }
    __device__ uint32_t pw0() const { return pw0_; }  // the first pattern word (m <= 3)
};
template <bool WIDE, class F>
__device__ __forceinline__ uint32_t any_mask(const uint32_t (&w)[kBatchNL * 4 + 1], const DevPlan &p, const F &f) {
    if (f.var() == 2) return fingerprint_mask<kBatchNL>(w, p, p.table);
    if (WIDE && f.nl() == 3) return direct_mask<kBatchNL, 4, 0>(w, p);
    switch (f.pk()) {
        case 1: return byte_mask(w, f.pw0());
        case 2: return short_mask<2>(w, f.pw0());  // per-lane byte runs: no wave masks
        case 3: return short_mask<3>(w, f.pw0());
        default: break;  // 64-bit prefixes (pk 5..8) take the 4-byte path here
    }
    switch (f.nw()) {
        case 1: return direct_mask<kBatchNL, 4, 1>(w, p);
        case 2: return direct_mask<kBatchNL, 4, 2>(w, p);
        case 3: return direct_mask<kBatchNL, 4, 3>(w, p);
        default: return direct_mask<kBatchNL, 4, 4>(w, p);
    }
}

// Window of 4 text bytes at byte `off` of a wave's LDS copy of its piece.
__device__ __forceinline__ uint32_t lds_window(const uint32_t *tw, uint32_t off) {
    const uint32_t q = off >> 2, r = off & 3;
    return r == 0 ? tw[q] : __builtin_amdgcn_alignbyte(tw[q + 1], tw[q], r);
}

// Words of a wave's LDS copy of its text piece: the piece's 1024 bytes, the
// 32 bytes after it, and one zero word for the last window.
constexpr uint32_t kTextWords = kWavePiece / 4 + 8 + 1;

// Multi-pattern count of one lane piece against a group (staged in LDS):
// each of the 16 windows (4 bytes, or 8 for a group of m >= 8 patterns) is
// hashed to its bucket and the bucket's flag byte read; a window whose
// bucket is not empty is compared with the first word of every member in it,
// then with the member's remaining words (from the LDS copy of the piece,
// up to 32 bytes) and, past 32 bytes, the tail check.  Hits of member j are
// added to s_cnt[j] and listed in s_park (up to kParkMax; s_npark counts
// them all).
__device__ __forceinline__ void group_count(const uint32_t (&w)[kBatchNL * 4 + 1], const uint32_t *tw,
                                            const uint32_t *s_tab, const BatchPairDesc *s_gd, uint32_t *s_cnt,
                                            uint32_t *s_park, uint32_t *s_npark, uint32_t member0,
                                            bool long_keys, const BatchTextDesc &t, uint64_t s0,
                                            uint32_t lane_byte, uint32_t unit_off) {
    // first the flag bytes of non-empty buckets, then, for the rare windows
    // whose bucket holds members, the member masks.  long_keys: the group's
    // keys are 8-byte windows (all members have m >= 8)
    const uint8_t *s_flag = reinterpret_cast<const uint8_t *>(s_tab + kGroupBuckets);
    uint32_t cand = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t b = long_keys ? group_bucket8(window(w, k), window(w, k + 4)) : group_bucket(window(w, k));
        cand |= (uint32_t)s_flag[b] << k;
    }
    while (cand) {
        const uint32_t k = __builtin_ctz(cand);
        cand &= cand - 1;
        const uint32_t off = lane_byte + k;
        const uint32_t x = lds_window(tw, off);
        uint32_t members = s_tab[long_keys ? group_bucket8(x, lds_window(tw, off + 4)) : group_bucket(x)];
        const uint64_t s = s0 + k;
        while (members) {
            const uint32_t j = __builtin_ctz(members);
            members &= members - 1;
            const DevPlan &p = s_gd[j].plan;
            if (x != p.pw[0]) continue;
            const uint64_t m = p.m;
            if (s < t.delta || s > t.delta + t.n - m) continue;
            const uint32_t nw = m >= 32 ? 8u : (uint32_t)((m + 3) / 4);
            bool ok = true;
            for (uint32_t i = 1; i < nw && ok; ++i)
                ok = (lds_window(tw, off + 4 * i) & p.pmask[i]) == p.pw[i];
            if (ok && m > 32) ok = tail_check(1u, s, t.base, p.pattern, m, 32) != 0;
            if (ok) {
                atomicAdd(&s_cnt[j], 1u);
                const uint32_t q = atomicAdd(s_npark, 1u);
                if (q < kParkMax) s_park[q] = ((member0 + j) << 16) | (unit_off + k);
            }
        }
    }
}

// Copy n 16-byte elements from global memory to LDS through the LDS DMA
// path (buffer loads with the lds bit): each lane's element goes from memory
// straight into LDS, wave w of round r writing elements r * THREADS + w * 64
// + lane at its own base (lane i at base + 16 i).  The copy holds no data in
// registers and all of the workgroup's loads are in flight at once; the
// next __syncthreads() waits for them (vmcnt).
typedef __attribute__((address_space(3))) void lds_void;
template <int THREADS>
__device__ __forceinline__ void stage_lds(void *dst, const void *src, uint32_t n, int tid) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(static_cast<const uint8_t *>(src), n * 16);
    // the wave index in a scalar register: the loop and the LDS bases are scalar
    const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid / kWave);
    const uint32_t lane = (uint32_t)tid & (kWave - 1);
#pragma unroll 1
    for (uint32_t base = wave * kWave; base < n; base += THREADS) {
        if (base + lane < n)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void *)(static_cast<uint4 *>(dst) + base), 16,
                                                     (int)(lane * 16), (int)(base * 16), 0, 0);
    }
}

// Count pass over the groups of the unit's text (after its solo pairs): the
// piece goes to LDS once (windows at run-time offsets), then each group's
// table and member descriptors are staged in turn (the members into s_gd,
// the solo pairs' staging array, free by now).
// The hits are also parked: listed in LDS as they are found, then sorted by
// (member, offset) and stored as the unit's park list, whose length (or
// kParkOverflow) goes to park_n.
template <int WAVES>
__device__ __forceinline__ void batch_groups(const BatchArgs &a, const BatchUnit &unit, const BatchTextDesc &t,
                                             const uint32_t (&w)[kBatchNL * 4 + 1], uint64_t s0,
                                             BatchPairDesc *s_gd) {
    constexpr int kThreads = WAVES * kWave;
    constexpr uint32_t kDescU128 = sizeof(BatchPairDesc) / 16;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (t.group_begin == t.group_end) {
        if (tid == 0) a.park_n[blockIdx.x] = 0;
        return;
    }
    __shared__ uint32_t s_text[WAVES][kTextWords];
    __shared__ __attribute__((aligned(16))) uint32_t s_tab[kGroupTableWords];
    __shared__ uint32_t s_cnt[kGroupMax];
    __shared__ uint32_t s_park[kParkMax];
    __shared__ uint32_t s_npark;
    if (tid == 0) s_npark = 0;  // ordered before the first hit by the staging barrier
    uint32_t *tw = s_text[wave];
#pragma unroll
    for (int i = 0; i < 4; ++i) tw[lane * 4 + i] = w[i];
    if (lane == kWave - 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) tw[kWavePiece / 4 + i] = w[4 + i];
        tw[kTextWords - 1] = 0;
    }
#pragma unroll 1
    for (uint32_t g = t.group_begin; g < t.group_end; ++g) {
        // members: the next kGroupMax (or fewer) grouped pairs of the text of
        // the group's kind (m = 4..7, then m >= 8)
        const bool long_keys = g >= t.long_group;
        const uint32_t first = (long_keys ? t.short_end + (g - t.long_group) * kGroupMax
                                          : t.solo_end + (g - t.group_begin) * kGroupMax);
        const uint32_t count = min(kGroupMax, (long_keys ? t.pair_end : t.short_end) - first);
        const uint32_t *gt = a.group_tables + (size_t)g * kGroupTableWords;
        stage_lds<kThreads>(s_tab, gt, kGroupTableWords / 4, tid);
        stage_lds<kThreads>(s_gd, a.kpairs + first, count * kDescU128, tid);
        if ((uint32_t)tid < count) s_cnt[tid] = 0;
        __syncthreads();
        group_count(w, tw, s_tab, s_gd, s_cnt, s_park, &s_npark, first - t.solo_end, long_keys, t, s0,
                    (uint32_t)lane * kPiece, (uint32_t)wave * kWavePiece + (uint32_t)lane * kPiece);
        __syncthreads();
        if ((uint32_t)tid < count) a.pt_count[s_gd[tid].cnt_base + unit.tile] = s_cnt[tid];
        __syncthreads();  // s_cnt and the staged group are rewritten next
    }
    // park: the keys are distinct, so a key's rank is the number of smaller keys
    const uint32_t n = s_npark;
    const bool fits = n <= kParkMax && t.pair_end - t.solo_end <= 65536u;
    if (fits && (uint32_t)tid < n) {
        const uint32_t key = s_park[tid];
        uint32_t rank = 0;
        for (uint32_t i = 0; i < n; ++i) rank += s_park[i] < key ? 1u : 0u;
        a.park[(uint64_t)blockIdx.x * kParkMax + rank] = key;
    }
    if (tid == 0) a.park_n[blockIdx.x] = fits ? n : kParkOverflow;
}

// One unit of the count pass (WRITE false) or of the write pass (WRITE
// true).  The two passes are separate kernels so that each allocates only
// its own LDS: the count pass has no position stage, the write pass no group
// tables.
template <int WAVES, bool WRITE>
__device__ __forceinline__ void batch_unit(const BatchArgs &a) {
    constexpr int kThreads = WAVES * kWave;
    constexpr uint32_t kTileB = WAVES * kWavePiece;
    __shared__ uint32_t s_wcnt[WAVES];
    __shared__ uint32_t s_stage[WRITE ? WAVES : 1][WRITE ? kStage : 1];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

    const BatchUnit unit = a.units[blockIdx.x];
    const BatchTextDesc t = a.texts[unit.text];
    const uint64_t tile_start = (uint64_t)unit.tile * kTileB;
    const uint64_t avail = ((t.delta + t.n + 15) & ~15ull) - tile_start;
    const uint32_t nrec = avail > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)avail;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(t.base + tile_start, nrec);
    const uint32_t lane_off = (uint32_t)wave * kWavePiece + (uint32_t)lane * kPiece;
    const uint64_t s0 = tile_start + lane_off;

    // each lane loads its own 16 bytes; the 32 after them come from the next
    // two lanes (lanes 62 and 63: the next piece's first bytes, one
    // wave-uniform load), so the tile crosses the cache hierarchy once
    uint32_t wl[1][kBatchNL * 4 + 1];
    load_chunk<1, kBatchNL>(wl, rsrc, lane_off);
    uint32_t (&w)[kBatchNL * 4 + 1] = wl[0];

    // the count pass filters the solo pairs one by one and the groups
    // together; the write pass redoes, pair by pair, only entries with hits:
    // of the solo pairs, and of the grouped pairs only when the unit's group
    // hits did not fit in its park list (else it places the parked hits).
    // Pair descriptors are staged in LDS a chunk at a time, so the loop over
    // pairs waits on no global load.
    const uint32_t parked = WRITE ? a.park_n[blockIdx.x] : 0u;
    const uint32_t pb = t.pair_begin;
    const uint32_t pe = WRITE && parked == kParkOverflow ? t.pair_end : t.solo_end;
    // write pass: the unit's parked keys go to LDS by DMA now, with the text
    __shared__ __attribute__((aligned(16))) uint32_t s_keys[WRITE ? kParkMax : 1];
    if constexpr (WRITE) stage_lds<kThreads>(s_keys, a.park + (uint64_t)blockIdx.x * kParkMax, kParkMax / 4, tid);
    const int64_t wave_pos0 = (int64_t)(tile_start + (uint64_t)wave * kWavePiece) - (int64_t)t.delta;
    constexpr uint32_t kDescU128 = sizeof(BatchPairDesc) / 16;
    static_assert(sizeof(BatchPairDesc) % 16 == 0, "descriptors are copied as 16-byte elements");
    static_assert(kGroupTableWords % 4 == 0, "group tables are copied as 16-byte elements");
    __shared__ __attribute__((aligned(16))) BatchPairDesc s_pd[kPairChunk];
    // per staged pair: the count pass accumulates its entry's count in
    // s_pcnt; the write pass loads the entry's count and output offset into
    // s_po (one slot per pair keeps one LDS base live across the loop)
    __shared__ uint32_t s_pcnt[WRITE ? 1 : kPairChunk];
    __shared__ uint64_t s_po[WRITE ? kPairChunk : 1][2];
#pragma unroll 1
    for (uint32_t cb = pb; cb < pe; cb += kPairChunk) {
        const uint32_t nc = min(kPairChunk, pe - cb);
        stage_lds<kThreads>(s_pd, a.kpairs + cb, nc * kDescU128, tid);
        if ((uint32_t)tid < nc) {
            if constexpr (WRITE) {
                // the entry follows from the text's descriptor alone
                const uint32_t q = cb + (uint32_t)tid;
                const uint64_t entry = t.entry_begin + (uint64_t)(q - pb) * t.tiles + unit.tile;
                s_po[tid][0] = a.pt_count[entry];
                s_po[tid][1] = a.pt_offset[entry] + (uint64_t)a.shift[q];
            } else {
                s_pcnt[tid] = 0;
            }
        }
        __syncthreads();
        if (cb == pb) fill_halo<kBatchNL>(wl[0]);
#pragma unroll 1
        for (uint32_t j = 0; j < nc; ++j) {
            const BatchPairDesc &pd = s_pd[j];
            if (WRITE && s_po[j][0] == 0) continue;
            const DevPlan &p = pd.plan;
            uint32_t mk, verified;
            uint64_t m;
            if constexpr (WRITE) {
                // at its register cap, the write pass reads the fields where
                // it branches on them
                mk = any_mask<false>(w, p, PlanFields{p});
                m = p.m;
                verified = p.variant != 2 && p.nl == 3 ? 16u : 4u * p.nw;
            } else {
                // the fields the pair's path branches on, read together (one
                // LDS round trip instead of one per branch) into scalar
                // registers
                auto held = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
                const HeldFields f{held(p.variant), held(p.nl), held(p.pk), held(p.nw), held(p.pw[0])};
                m = held((uint32_t)p.m);  // m <= EPSM_MAX_M
                mk = any_mask<true>(w, p, f);
                verified = 4u * f.nw();
            }
            const uint64_t last = t.delta + t.n - m;  // m <= n here
            if (tile_start + kTileB > last || tile_start < t.delta) mk &= valid_mask(s0, t.delta, last);
            if (m > verified && wave_any(mk != 0))
                mk = tail_check(mk, s0, t.base, p.pattern, m, verified);
            const uint32_t c = __popc(mk);
            const uint32_t incl = wave_incl_scan32(c);
            const uint32_t wtot = last_lane(incl);
            if constexpr (!WRITE) {
                // count pass: waves add their totals; no barrier per pair
                if (lane == 0 && wtot) atomicAdd(&s_pcnt[j], wtot);
            } else {
                if (lane == 0) s_wcnt[wave] = wtot;
                __syncthreads();
                if (wtot) {
                    uint64_t obase = s_po[j][1];
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
        __syncthreads();
        if (!WRITE && (uint32_t)tid < nc) a.pt_count[s_pd[tid].cnt_base + unit.tile] = s_pcnt[tid];
        __syncthreads();  // the next chunk restages s_pd, s_pcnt and s_po
    }
    if (pb == pe) fill_halo<kBatchNL>(wl[0]);
    if constexpr (!WRITE) {
        batch_groups<WAVES>(a, unit, t, w, s0, s_pd);
    } else if (parked != kParkOverflow && parked != 0) {
        // parked group hits, sorted by (member, offset): hit i of a member is
        // its entry's (i - first)-th position, first being the member's first
        // index in the list
        __syncthreads();  // the DMA into s_keys (no barrier yet without solo pairs)
        if (wave == 0) {  // the list fits one wave: lane i places hit i
            const bool live = (uint32_t)lane < parked;
            const uint32_t key = live ? s_keys[lane] : 0u, member = key >> 16;
            // a member's hits are consecutive; its first is the nearest lane
            // at or below this one that starts a member
            const bool head = live && (lane == 0 || (s_keys[lane - 1] >> 16) != member);
            const uint64_t heads = __ballot(head);
            const uint32_t first = 63u - (uint32_t)__clzll(heads & (~0ull >> (63 - lane)));
            const uint32_t q = t.solo_end + member;  // the member's pair in kernel order
            if (live && q < t.pair_end) {
                const uint64_t entry = t.entry_begin + (uint64_t)(q - t.pair_begin) * t.tiles + unit.tile;
                const uint64_t pos = a.pt_offset[entry] + (uint64_t)a.shift[q] + ((uint32_t)lane - first);
                if (pos < a.cap) a.out[pos] = (int64_t)(tile_start + (key & 0xFFFFu)) - (int64_t)t.delta;
            }
        }
    }
}

// Both passes are latency bound (dependent loads per unit, barriers per
// pair), so they ask for six waves per SIMD at 4 waves per workgroup (80
// registers) and five otherwise.
static_assert(kParkMax <= kWave, "one lane of wave 0 per parked hit");

template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(WAVES == 4 ? 6 : 5, 8)))
void batch_kernel_count(BatchArgs a) {
    batch_unit<WAVES, false>(a);
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(WAVES == 4 ? 6 : 5, 8)))
void batch_kernel_write(BatchArgs a) {
    batch_unit<WAVES, true>(a);
}

bool batch_waves_supported(int waves) { return waves == 4 || waves == 8 || waves == 16; }

hipError_t launch_batch(const BatchArgs &a, int waves, uint32_t n_units, hipStream_t s) {
    clear_launch_error();
    if (n_units == 0) return hipSuccess;
    auto launch = [&](auto waves_c) {
        constexpr int W = decltype(waves_c)::value;
        if (a.write)
            hipLaunchKernelGGL(batch_kernel_write<W>, dim3(n_units), dim3(W * kWave), 0, s, a);
        else
            hipLaunchKernelGGL(batch_kernel_count<W>, dim3(n_units), dim3(W * kWave), 0, s, a);
    };
    switch (waves) {
        case 4: launch(std::integral_constant<int, 4>()); break;
        case 8: launch(std::integral_constant<int, 8>()); break;
        case 16: launch(std::integral_constant<int, 16>()); break;
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
    clear_launch_error();
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

// Pair results in the caller's order.  Step 1: each pair's count from the
// offsets of its first and past-last entries, and the sum of each block of
// kScanBlock pairs.
__global__ __launch_bounds__(256) void pair_count_kernel(const BatchSpan *spans, uint32_t n_pairs,
                                                         const uint64_t *offsets, uint64_t *counts,
                                                         uint64_t *block_sums) {
    __shared__ uint64_t s_part[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t v = 0;
    for (uint32_t i = threadIdx.x; i < kScanBlock; i += 256) {
        const uint64_t k = base + i;
        if (k < n_pairs) {
            const BatchSpan sp = spans[k];
            const uint64_t c = sp.tiles ? offsets[sp.cnt_base + sp.tiles] - offsets[sp.cnt_base] : 0;
            counts[k] = c;
            v += c;
        }
    }
    v = wave_sum64(v);
    if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

// Step 3 (after scan_blocks_kernel over the block sums): each pair's output
// offset, the exclusive prefix of the counts in the caller's order, and the
// shift that turns its entries' offsets (a prefix in kernel order) into
// output positions.
__global__ __launch_bounds__(256) void pair_offset_kernel(const BatchSpan *spans, uint32_t n_pairs,
                                                          const uint64_t *offsets, const uint64_t *counts,
                                                          const uint64_t *block_sums, uint64_t *pair_offsets,
                                                          int64_t *shift, uint64_t entries, uint64_t *total) {
    __shared__ uint64_t s_wave[4];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)tid * 16;
    uint64_t v[16];
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < n_pairs ? counts[base + i] : 0ull;
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
        const uint64_t k = base + i;
        if (k < n_pairs) {
            pair_offsets[k] = run;
            const BatchSpan sp = spans[k];
            if (sp.kq != kNoKq) shift[sp.kq] = (int64_t)(run - offsets[sp.cnt_base]);
        }
        run += v[i];
    }
    if (blockIdx.x == 0 && tid == 0 && total) *total = offsets[entries];
}

hipError_t launch_batch_finalize(const BatchSpan *spans, uint32_t n_pairs,
                                 const uint64_t *offsets, uint64_t entries, uint64_t *counts,
                                 uint64_t *pair_offsets, uint64_t *total, int64_t *shift,
                                 uint64_t *block_sums, hipStream_t s) {
    clear_launch_error();
    const uint32_t blocks = (uint32_t)(((uint64_t)n_pairs + kScanBlock - 1) / kScanBlock);
    if (blocks)
        hipLaunchKernelGGL(pair_count_kernel, dim3(blocks), dim3(256), 0, s, spans, n_pairs, offsets, counts,
                           block_sums);
    // exclusive scan of the block sums; its grand total goes to the spare
    // slot past them
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, block_sums, (uint64_t)blocks,
                       block_sums + blocks, (uint64_t)0);
    hipLaunchKernelGGL(pair_offset_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, s, spans, n_pairs, offsets,
                       counts, block_sums, pair_offsets, shift, entries, total);
    return hipGetLastError();
}

}  // namespace epsm

// Device-side building blocks of the scan, shared by the single-text and the
// batched kernels: buffer loads, packed windows, the direct and fingerprint
// filters, exact verification, wave reductions and the look-back.
#pragma once

#include "epsm_internal.h"

namespace epsm {


typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// gfx9-family raw buffer descriptor word 3 (32-bit data format, no swizzle).
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const uint8_t *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(p), (short)0, (int)bytes,
                                             kRsrcWord3);
}

__device__ __forceinline__ u32x4 load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}

// Window of 4 text bytes starting at byte k of the lane's register run w.
template <int N>
__device__ __forceinline__ uint32_t window(const uint32_t (&w)[N], int k) {
    const int q = k >> 2, r = k & 3;
    return r == 0 ? w[q] : __builtin_amdgcn_alignbyte(w[q + 1], w[q], (uint32_t)r);
}

__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool wave_any(bool c) { return ballot(c) != 0; }

// Window of 8 text bytes starting at byte k of the lane's register run.
template <int N>
__device__ __forceinline__ uint64_t window64(const uint32_t (&w)[N], int k) {
    return ((uint64_t)window(w, k + 4) << 32) | window(w, k);
}

// Pattern words j, j+1 as one 64-bit value.
__device__ __forceinline__ uint64_t pattern64(const DevPlan &p, int j) {
    return ((uint64_t)p.pw[j + 1] << 32) | p.pw[j];
}

// Narrow a wave mask of candidates at lane byte k with pattern words
// J0..nw-1, two words per compare: one 64-bit v_cmp whose result is the wave
// mask itself, so a pair costs one scalar AND.  Every pattern word but the
// last is whole, so only the last one is masked.  nw is the template
// constant NW, or the plan's runtime value when NW == 0 (then the high word
// of every pair is masked, since it may be the last).  SKIP: no compare for
// a start that no lane holds a candidate for (a scalar test and branch per
// start; without it the compares run unconditionally, which costs vector
// instructions only where candidates are rare).  LEAN: the form with fewer
// live registers (differences OR-ed into one test).  Every register index
// is a compile-time constant (a runtime one would move the run to scratch).
template <int NWMAX, int NW, int J0, bool SKIP, bool LEAN, int N>
__device__ __forceinline__ uint64_t verify_words(const uint32_t (&w)[N], int k, uint64_t b,
                                                 const DevPlan &p) {
    const int nw = NW > 0 ? NW : (int)p.nw;
#pragma unroll
    for (int j = J0; j < NWMAX; j += 2) {
        if (j < nw && (!SKIP || b != 0)) {
            if (j + 1 < nw) {
                const bool whole = NW > 0 && j + 2 < NW;  // the high word is not the last
                const uint32_t lo = window(w, k + 4 * j), hi = window(w, k + 4 * j + 4);
                if (LEAN) {
                    const uint32_t d0 = lo ^ p.pw[j];
                    const uint32_t d1 = whole ? (hi ^ p.pw[j + 1]) : ((hi ^ p.pw[j + 1]) & p.pmask[j + 1]);
                    b &= ballot((((uint64_t)d1 << 32) | d0) == 0);
                } else if (whole && (k & 3) == 0) {
                    // two adjacent words of the run as they are: joined into
                    // one 64-bit value they would become one 64-bit access to
                    // the run, which then no longer fits in registers
                    b &= ballot(lo == p.pw[j] && hi == p.pw[j + 1]);
                } else {
                    const uint32_t h = whole ? hi : (hi & p.pmask[j + 1]);
                    b &= ballot((((uint64_t)h << 32) | lo) == pattern64(p, j));
                }
            } else {
                b &= ballot((window(w, k + 4 * j) & p.pmask[j]) == p.pw[j]);
            }
        }
    }
    return b;
}

// Occurrences marked in 16 wave masks (wave-uniform: scalar popcounts).
__device__ __forceinline__ uint32_t masks_count(const uint64_t (&b)[16]) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) c += (uint32_t)__builtin_popcountll(b[k]);
    return c;
}

// Per-lane 16-bit mask from the 16 wave masks: bit k of lane L is bit L of b[k].
__device__ __forceinline__ uint32_t lanes_from_masks(const uint64_t (&b)[16]) {
    uint32_t lm = 0;
#pragma unroll
    for (int k = 15; k >= 0; --k)
        lm = lm + lm + (__builtin_amdgcn_inverse_ballot_w64(b[k]) ? 1u : 0u);
    return lm;
}

// m = 1: per-lane byte equality without wave masks.  For x = word ^ c*0x01010101
// a byte is zero iff the byte matches; ((x & 0x7F..) + 0x7F..) sets the high
// bit of every byte whose low seven bits are not all zero, without carries
// between bytes, so ~(that | x | 0x7F..) keeps exactly the high bits of the
// zero bytes.  One multiply gathers those four bits (byte i's bit lands on
// bit 28 + i; no partial product reaches bits 24..27 or carries into 28..31).
__device__ __forceinline__ uint32_t byte_mask(const uint32_t *w, uint32_t c) {
    const uint32_t rep = c * 0x01010101u;
    uint32_t mk = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t x = w[q] ^ rep;
        const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
        mk |= ((((z >> 7) & 0x01010101u) * 0x10204080u) >> 28) << (4 * q);
    }
    return mk;
}

// m = 2 or 3, the same per-lane test on byte runs: start 4q + i matches iff
// bytes 4q + i .. 4q + i + M - 1 equal p[0..M-1].  The word, and its copies
// advanced by one (and two) bytes, are xor-ed with the repeated pattern
// bytes and or-ed together, so a byte is zero iff its start matches; the
// zero-byte test of byte_mask then gathers the four bits.  Reads w[0..4].
template <int M>
__device__ __forceinline__ uint32_t short_mask(const uint32_t *w, uint32_t pw0) {
    static_assert(M == 2 || M == 3, "byte runs of 2 or 3");
    const uint32_t r0 = (pw0 & 0xFFu) * 0x01010101u;
    const uint32_t r1 = ((pw0 >> 8) & 0xFFu) * 0x01010101u;
    const uint32_t r2 = ((pw0 >> 16) & 0xFFu) * 0x01010101u;
    uint32_t mk = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t x = (w[q] ^ r0) | (__builtin_amdgcn_alignbyte(w[q + 1], w[q], 1) ^ r1);
        if constexpr (M == 3) x |= __builtin_amdgcn_alignbyte(w[q + 1], w[q], 2) ^ r2;
        const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
        mk |= ((((z >> 7) & 0x01010101u) * 0x10204080u) >> 28) << (4 * q);
    }
    return mk;
}

// Wave masks of the direct variant (PK >= 2): bit L of b[k] is set iff
// lane L's start k matches the prefix and the remaining register words.
// Returns false, with b undefined, when no lane has a hit.
template <int NL, int PK, int NW, bool SKIP, bool LEAN>
__device__ __forceinline__ bool direct_wave_masks(const uint32_t (&w)[NL * 4 + 1], const DevPlan &p,
                                                  uint64_t (&b)[16]) {
    static_assert(PK >= 2, "m = 1 uses byte_mask");
    constexpr int NWMAX = 4 * NL - 4;
    uint64_t any = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int q = k >> 2, r = k & 3;
        bool c;
        if constexpr (PK == 2) {
            c = (window(w, k) & 0xFFFFu) == p.pw[0];
        } else if constexpr (PK == 8) {
            c = window64(w, k) == pattern64(p, 0);  // m >= 8: no mask
        } else if constexpr (PK == 7) {
            // m = 5..7: bytes 0..7 with the high word masked to the pattern
            c = ((((uint64_t)(window(w, k + 4) & p.pmask[1])) << 32) | window(w, k)) == pattern64(p, 0);
        } else if constexpr (PK == 3) {
            // bytes k..k+2 of the run and a zero top byte in one v_perm
            const uint32_t sel = (uint32_t)r | ((uint32_t)(r + 1) << 8) |
                                 ((uint32_t)(r + 2) << 16) | (0x0Cu << 24);
            c = __builtin_amdgcn_perm(w[q + 1], w[q], sel) == p.pw[0];
        } else {
            c = window(w, k) == p.pw[0];
        }
        b[k] = ballot(c);
        any |= b[k];
    }
    if (any == 0) return false;
    constexpr int J0 = PK >= 7 ? 2 : 1;  // words the prefix compare covers
    if constexpr (PK >= 4 && (NW == 0 || NW > J0)) {
        any = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            b[k] = verify_words<NWMAX, NW, J0, SKIP, LEAN>(w, k, b[k], p);
            any |= b[k];
        }
        if (any == 0) return false;
    }
    return true;
}

// Direct variant: 16-bit hit mask of one lane piece (positions 0..15).
// All 16 prefix compares come first and their wave masks are OR-ed once;
// only a wave with some candidate narrows them with the remaining pattern
// words and transposes them into per-lane masks.  Keeping the common path
// free of per-position branches matters: the scalar unit issues one
// instruction per SIMD every four cycles and was the bottleneck.
template <int NL, int PK, int NW, bool SKIP = true, bool LEAN = true>
__device__ __forceinline__ uint32_t direct_mask(const uint32_t (&w)[NL * 4 + 1], const DevPlan &p) {
    if constexpr (PK == 1) {
        return byte_mask(w, p.pw[0]);
    } else {
        uint64_t b[16];
        return direct_wave_masks<NL, PK, NW, SKIP, LEAN>(w, p, b) ? lanes_from_masks(b) : 0u;
    }
}

// Fingerprint variant: the lane hashes the blocks at its byte 0, 8 and 16
// (the last one is the next lane's first block).  Table entry bit (8-j)
// marks offset j, so the candidates relative to the lane start are
// block0: bit 8 -> start 0; block8: bits 1..8 -> starts 1..8;
// block16: bits 1..7 -> starts 9..15 (bit 8 = start 16 belongs to the next lane).
// The candidates are verified as wave masks; returns false when no lane has
// a hit.
template <int NL, bool SKIP, bool LEAN>
__device__ __forceinline__ bool fingerprint_wave_masks(const uint32_t (&w)[NL * 4 + 1], const DevPlan &p,
                                                       const uint16_t *tab, uint64_t (&b)[16]) {
    constexpr int NWMAX = 4 * NL - 4;
    uint32_t v0 = 0, v1 = 0, v2 = 0;
    if (!p.collide) {
        v0 = fp_hash(w[0], w[1], p.hash_bits);
        v1 = fp_hash(w[2], w[3], p.hash_bits);
        v2 = fp_hash(w[4], w[5], p.hash_bits);
    }
    const uint32_t cm = ((uint32_t)tab[v0] >> 8) | (uint32_t)tab[v1] |
                        (((uint32_t)tab[v2] << 8) & 0xFFFFu);
    if (!wave_any(cm != 0)) return false;
    uint64_t any = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        // a fingerprint plan has m >= 15, so a two-load run (NL = 2) holds
        // exactly its first four words (only the fourth can be partial)
        b[k] = verify_words<NWMAX, NL == 2 ? 4 : 0, 0, SKIP, LEAN>(w, k, ballot((cm >> k) & 1u), p);
        any |= b[k];
    }
    return any != 0;
}

template <int NL, bool SKIP = true, bool LEAN = true>
__device__ __forceinline__ uint32_t fingerprint_mask(const uint32_t (&w)[NL * 4 + 1],
                                                     const DevPlan &p, const uint16_t *tab) {
    uint64_t b[16];
    return fingerprint_wave_masks<NL, SKIP, LEAN>(w, p, tab, b) ? lanes_from_masks(b) : 0u;
}

// Packed DNA (variant 3): coordinates are 2-bit symbols, 16 to a 32-bit
// word, symbol t of a word at bits 2t.  A lane holds 64 symbols (its 16 and
// the 48 after them) in w[0..3].  The window of 16 symbols at symbol k of
// word j is a funnel shift of words j and j+1 by 2k bits.
__device__ __forceinline__ uint32_t dna_window(const uint32_t (&w)[5], int j, int k) {
    return k == 0 ? w[j] : __builtin_amdgcn_alignbit(w[j + 1], w[j], (uint32_t)(2 * k));
}

// DNA hit mask of one lane piece: the first 16 symbols of the pattern
// (masked below m unless FULL, i.e. m >= 16) against each of the 16 windows,
// then the next one or two pattern words where some lane of the wave still
// has a candidate.
// Packed DNA, m >= 16: the 8-symbol block filter (Section 3.4 over 2-bit
// symbols).  An occurrence at start s holds the aligned block at the first
// multiple of 8 at or after s, at pattern offset j = q - s in [0, 7].  The
// lane's starts 0..15 are covered by its blocks at symbols 0, 8 and 16 (the
// low and high halves of w[0], the low half of w[1]): bit j of the block at
// 8i marks start 8i - j, kept when it lies in 0..15.  Each lane then checks
// its own candidates against up to three pattern words, with the window
// shift a per-lane register (every window lies within w[j], w[j + 1]).
__device__ __forceinline__ uint32_t dna_block_mask(const uint32_t (&w)[5], const DevPlan &p,
                                                   const uint16_t *tab) {
    const uint32_t t0 = tab[fp_hash(w[0] & 0xFFFFu, 0, p.hash_bits)];
    const uint32_t t1 = tab[fp_hash(w[0] >> 16, 0, p.hash_bits)];
    const uint32_t t2 = tab[fp_hash(w[1] & 0xFFFFu, 0, p.hash_bits)];
    // bit j -> start 8 - j (t1) or 16 - j (t2, j >= 1): reverse, then shift
    uint32_t cand = (t0 & 1u) | ((__builtin_bitreverse32(t1) >> 23) & 0x1FEu) |
                    ((__builtin_bitreverse32(t2) >> 15) & 0xFE00u);
    uint32_t mk = 0;
    while (cand) {
        const uint32_t k = __builtin_ctz(cand);
        cand &= cand - 1;
        bool ok = true;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j < (int)p.nw)
                ok = ok && (__builtin_amdgcn_alignbit(w[j + 1], w[j], 2 * k) & p.pmask[j]) == p.pw[j];
        mk |= ok ? 1u << k : 0u;
    }
    return mk;
}

template <bool FULL>
__device__ __forceinline__ uint32_t dna_mask(const uint32_t (&w)[5], const DevPlan &p) {
    uint64_t b[16];
    uint64_t any = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = dna_window(w, 0, k);
        b[k] = ballot((FULL ? x : (x & p.pmask[0])) == p.pw[0]);
        any |= b[k];
    }
    if (any == 0) return 0u;
    if (p.nw > 1) {
        any = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int j = 1; j < 3; ++j)
                if (j < (int)p.nw && b[k] != 0)
                    b[k] &= ballot((dna_window(w, j, k) & p.pmask[j]) == p.pw[j]);
            any |= b[k];
        }
        if (any == 0) return 0u;
    }
    return lanes_from_masks(b);
}

// Exact check of DNA pattern symbols [from, m) for each candidate, reading
// the packed text and the pattern codes from global memory.
static inline __device__ __noinline__ uint32_t tail_check_dna(uint32_t mk, uint64_t s0, const uint8_t *base,
                                                              const uint8_t *pattern, uint64_t m,
                                                              uint32_t from) {
    uint32_t keep = 0;
    while (mk) {
        const uint32_t k = __builtin_ctz(mk);
        mk &= mk - 1;
        const uint64_t s = s0 + k;
        bool ok = true;
        for (uint64_t j = from; j < m; ++j) {
            const uint64_t q = s + j;
            if (((base[q >> 2] >> (2 * (q & 3))) & 3u) != pattern[j]) { ok = false; break; }
        }
        if (ok) keep |= 1u << k;
    }
    return keep;
}

// Start positions of the lane piece at base coordinate s0 that are valid
// (delta <= s <= last), as a 16-bit mask.
__device__ __forceinline__ uint32_t valid_mask(uint64_t s0, uint64_t delta, uint64_t last) {
    uint32_t lo = 0, hi = 16;
    if (delta > s0) lo = (delta - s0) > 16 ? 16u : (uint32_t)(delta - s0);
    if (last < s0) hi = 0;
    else if (last - s0 < 15) hi = (uint32_t)(last - s0) + 1;
    return ((1u << hi) - 1u) & ~((1u << lo) - 1u);
}

// Exact check of pattern bytes [4*nw, m) for each candidate (patterns longer
// than the register run); reads the text and pattern from global memory.
static inline __device__ __noinline__ uint32_t tail_check(uint32_t mk, uint64_t s0, const uint8_t *base,
                                                   const uint8_t *pattern, uint64_t m, uint32_t from) {
    uint32_t keep = 0;
    while (mk) {
        const uint32_t k = __builtin_ctz(mk);
        mk &= mk - 1;
        const uint8_t *t = base + s0 + k;
        bool ok = true;
        for (uint64_t j = from; j < m; ++j) {
            if (t[j] != pattern[j]) { ok = false; break; }
        }
        if (ok) keep |= 1u << k;
    }
    return keep;
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts (Hillis-Steele
// inside each row of 16 lanes) and the two row broadcasts of the last lane
// of rows 0 and 1: six full-rate VALU adds, no LDS permutes.
__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Value of lane 63 (the wave total after an inclusive scan).
__device__ __forceinline__ uint32_t last_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) { return last_lane(wave_incl_scan32(v)); }

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}


__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single-pass look-back, run by one full wave.  Publishes the tile's count,
// then reads kLookWindow predecessor status words per step (kLookLoads per
// lane, issued together, so one memory round trip per step) until an
// inclusive prefix is found; publishes the tile's inclusive prefix and
// returns the exclusive one.  The window bounds how fast the inclusive
// frontier can advance (kLookWindow * tile bytes per round trip); measured,
// a 256-entry window was no faster than 64 on 128 KiB tiles, so one load
// per lane is used.
// Every wait ends: a tile's aggregate is published before its own look-back,
// and a tile only waits on lower-indexed workgroups, which in-order dispatch
// has already started.  The poll bound only guarantees termination.
constexpr int kLookLoads = 1;
constexpr int kLookWindow = kLookLoads * kWave;

__device__ __forceinline__ uint64_t poll_status(uint64_t *status, int64_t idx, uint32_t *fault,
                                                uint32_t limit = kSpinLimit) {
    if (idx < 0) return kFlagInclusive;  // before tile 0: an inclusive zero
    uint64_t st = status_load(&status[idx]);
    uint32_t polls = 0;
    while ((st >> 62) == 0) {
        if (++polls >= limit) {
            __hip_atomic_store(fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return kFlagInclusive;
        }
        __builtin_amdgcn_s_sleep(1);
        st = status_load(&status[idx]);
    }
    return st;
}

static __device__ inline uint64_t look_back(uint64_t *status, uint32_t tile, uint64_t cnt, int lane,
                              uint32_t *fault) {
    if (tile == 0) {
        if (lane == 0) status_store(&status[0], kFlagInclusive | cnt);
        return 0;
    }
    if (lane == 0) status_store(&status[tile], kFlagAggregate | cnt);
    uint64_t excl = 0;
    int64_t top = (int64_t)tile - 1;
    for (;;) {
        // entry j*64 + lane of the window is tile top - (j*64 + lane)
        uint64_t st[kLookLoads];
#pragma unroll
        for (int j = 0; j < kLookLoads; ++j) {
            const int64_t idx = top - (j * kWave + lane);
            st[j] = idx >= 0 ? status_load(&status[idx]) : kFlagInclusive;
        }
        bool found = false;
#pragma unroll
        for (int j = 0; j < kLookLoads; ++j) {
            if (!found) {
                if ((st[j] >> 62) == 0) st[j] = poll_status(status, top - (j * kWave + lane), fault);
                const uint64_t incl = __ballot((st[j] >> 62) == 2);
                const int first = incl ? __ffsll((unsigned long long)incl) - 1 : kWave;
                excl += wave_sum64(lane <= first ? (st[j] & kValueMask) : 0);
                found = incl != 0;
            }
        }
        if (found) break;
        top -= kLookWindow;
    }
    if (lane == 0) status_store(&status[tile], kFlagInclusive | (excl + cnt));
    return excl;
}

// Positions staged per wave before they are written out (wave-relative
// offsets; one piece adds at most 1024).
constexpr uint32_t kStage = 1024;

typedef int64_t i64x2 __attribute__((ext_vector_type(2)));

// Write stage[0..fill) as positions wave_pos0 + stage[j] to out[obase + j]
// (entries at or past cap are dropped).  Lanes write consecutive pairs of
// entries as one 16-byte store (a wave instruction covers 1 KiB); an entry
// before the first 16-byte boundary of the range, and an odd last one, are
// written alone.
__device__ __forceinline__ void flush_stage(const uint32_t *stage, uint32_t fill, int64_t *out,
                                            uint64_t cap, uint64_t obase, int64_t wave_pos0,
                                            int lane) {
    // the stage was filled by other lanes of this wave: order the LDS accesses
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint64_t end = min((uint64_t)fill, cap > obase ? cap - obase : 0ull);  // entries written
    if ((uintptr_t)out & 7u) {
        // an output that is not 8-byte aligned: one entry per store
        for (uint32_t j = lane; j < end; j += kWave) out[obase + j] = wave_pos0 + stage[j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        return;
    }
    // entry `head` (0 or 1) is the first on a 16-byte boundary
    const uint32_t head = (((uintptr_t)(out + obase)) & 15u) ? 1u : 0u;
    if (head && end > 0 && lane == 0) out[obase] = wave_pos0 + stage[0];
    const uint64_t pairs = end > head ? (end - head) / 2 : 0;
    for (uint64_t q = lane; q < pairs; q += kWave) {
        const uint32_t j = head + 2 * (uint32_t)q;
        i64x2 v;
        v.x = wave_pos0 + stage[j];
        v.y = wave_pos0 + stage[j + 1];
        *reinterpret_cast<i64x2 *>(out + obase + j) = v;
    }
    if (end > head && ((end - head) & 1) && lane == 0) out[obase + end - 1] = wave_pos0 + stage[end - 1];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Write stage[0..fill) as dst[j] = add + stage[j] (tile-relative offsets of
// a two-phase slot list), dropping entries at or past `room`.  Lanes write
// consecutive entries.
__device__ __forceinline__ void flush_list(const uint32_t *stage, uint32_t fill, uint32_t *dst,
                                           uint32_t room, uint32_t add, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t j = lane; j < fill && j < room; j += kWave) dst[j] = add + stage[j];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A lane's run of byte texts is loaded in the streaming form: each lane loads
// only its own 16 bytes with the non-temporal hint (a grid-stride read
// reaches 7.0 TB/s with it, 6.5 without; a second read of a neighbour's bytes
// would miss once the hint has let them go), and takes the blocks after them
// from its right neighbour (fill_halo); lane 63's are the next piece's first
// bytes, the same address for the whole wave, which every lane loads (one
// memory request).
constexpr int kStreamLoad = 2;  // cache-policy operand of the buffer load: nt

template <int U, int NL>
__device__ __forceinline__ void load_chunk(uint32_t (&w)[U][NL * 4 + 1], __amdgpu_buffer_rsrc_t r,
                                           uint32_t off) {
    const uint32_t halo = off - (uint32_t)__lane_id() * kPiece + (kWave - 1) * kPiece;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(
                r, (int)(l == 0 ? off + u * kWavePiece : halo + u * kWavePiece + l * kPiece), 0, kStreamLoad);
            w[u][4 * l + 0] = v.x;
            w[u][4 * l + 1] = v.y;
            w[u][4 * l + 2] = v.z;
            w[u][4 * l + 3] = v.w;
        }
        w[u][NL * 4] = 0;
    }
}

// Complete a streaming run: block l of lane L is block l - 1 of lane L + 1
// (DPP wave_shl:1); lane 63 has no right neighbour and keeps what it loaded
// (the DPP result there is the old value).  Called right before the piece is
// used, once its loads have landed, so the prefetch overlap is kept.  Needs
// the whole wave active.
template <int NL>
__device__ __forceinline__ void fill_halo(uint32_t (&w)[NL * 4 + 1]) {
#pragma unroll
    for (int l = 1; l < NL; ++l)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[4 * l + j] = (uint32_t)__builtin_amdgcn_update_dpp((int)w[4 * l + j], (int)w[4 * (l - 1) + j],
                                                                 0x130, 0xF, 0xF, false);
}

// DNA: one dwordx4 per lane and piece (64 symbols) at byte offset off.
template <int U>
__device__ __forceinline__ void load_chunk_dna(uint32_t (&w)[U][5], __amdgpu_buffer_rsrc_t r,
                                               uint32_t off) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const u32x4 v = load16(r, off + u * (kWavePiece / 4));
        w[u][0] = v.x;
        w[u][1] = v.y;
        w[u][2] = v.z;
        w[u][3] = v.w;
        w[u][4] = 0;
    }
}

// Hit masks of the U pieces of one chunk, parked in LDS (two 16-bit masks per
// word); returns the lane's hit count.  CNT (count mode, patterns held in
// registers, no tail check): the wave masks are counted as they are (scalar
// popcounts, into wave_cnt) instead of being turned into per-lane masks.
// The direct filter verifies without a branch per start (SKIP false; its
// 8-byte prefix leaves few waves with candidates unless the text is dense)
// except in the three-load kernels, which keep the lean form for their
// registers; the fingerprint filter's candidates are sparse within a wave
// even on binary text (8/256 of the blocks), so it verifies only the starts
// that have some, in the lean form (measured faster there).
template <int U, int NL, int VAR, int PK, int NW, bool CNT, int PAIRS, int THREADS>
__device__ __forceinline__ uint32_t process_chunk(uint32_t (&w)[U][NL * 4 + 1], int c,
                                                  const ScanArgs &a, const uint16_t *tab,
                                                  uint64_t lane_start, bool edge, bool tail,
                                                  uint32_t (*s_mask)[THREADS], int tid,
                                                  uint32_t &wave_cnt) {
    constexpr bool kLean = NL > 2;
    uint32_t cnt = 0, lo = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if constexpr (VAR != 3) fill_halo<NL>(w[u]);
        const int piece = c * U + u;
        const uint64_t s0 = lane_start + (uint64_t)piece * kWavePiece;
        if constexpr (CNT) {
            uint64_t b[16];
            bool any;
            if constexpr (VAR == 1) any = direct_wave_masks<NL, PK, NW, kLean, kLean>(w[u], a.plan, b);
            else any = fingerprint_wave_masks<NL, true, true>(w[u], a.plan, tab, b);
            if (any) {
                if (edge) {
                    // only the first tile holds starts below delta and only
                    // the last one holds starts past `last`
                    const uint32_t vm = valid_mask(s0, a.delta, a.last);
#pragma unroll
                    for (int k = 0; k < 16; ++k) b[k] &= ballot((vm >> k) & 1u);
                }
                wave_cnt += masks_count(b);
            }
            continue;
        }
        uint32_t mk;
        if constexpr (VAR == 1) mk = direct_mask<NL, PK, NW, kLean, kLean>(w[u], a.plan);
        else if constexpr (VAR == 2) mk = fingerprint_mask<NL, true, true>(w[u], a.plan, tab);
        else if constexpr (PK == 16) mk = dna_block_mask(w[u], a.plan, tab);
        else mk = dna_mask<false>(w[u], a.plan);
        if (edge) mk &= valid_mask(s0, a.delta, a.last);
        if (tail && wave_any(mk != 0)) {
            if constexpr (VAR == 3)
                mk = tail_check_dna(mk, s0, a.base, a.plan.pattern, a.plan.m, 16u * a.plan.nw);
            else
                mk = tail_check(mk, s0, a.base, a.plan.pattern, a.plan.m, 4u * a.plan.nw);
        }
        cnt += __popc(mk);
        if (a.write == 0) continue;  // count only: the masks are not needed
        if (u & 1) s_mask[piece >> 1][tid] = lo | (mk << 16);
        else lo = mk;
    }
    return cnt;
}

}  // namespace epsm

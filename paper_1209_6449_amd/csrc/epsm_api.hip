// C ABI of the exact packed string matching library (see include/epsm.h).
//
// Host side: pattern preprocessing (Sections 3.2-3.4: packed pattern words
// for the direct compare, the fingerprint table for EPSMc), argument checks,
// a per-stream device workspace for the look-back status words, and kernel
// launches.  Nothing here touches text bytes: all matching runs on the GPU.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "epsm_host.h"

using namespace epsm;

namespace epsm {
namespace host {

thread_local std::string g_last_error;

epsm_status fail(epsm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

epsm_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? EPSM_ENOMEM : EPSM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

constexpr uint32_t kKnownPlanFlags = EPSM_PLAN_HOST_ONLY | EPSM_PLAN_FORCE_DIRECT |
                                     EPSM_PLAN_FORCE_FINGERPRINT | EPSM_PLAN_COLLIDE |
                                     EPSM_PLAN_HASH_BITS(0xF) | EPSM_PLAN_DNA |
                                     EPSM_PLAN_NO_STRIDE | EPSM_PLAN_PREFIX4 |
                                     EPSM_PLAN_SHORT_RUN | EPSM_PLAN_SIGMA(0x1FF);
// flags a variant-table row may add to a plan's own
constexpr uint32_t kVariantRowFlags = EPSM_PLAN_SHORT_RUN | EPSM_PLAN_PREFIX4 | EPSM_PLAN_HASH_BITS(0xF);
constexpr uint32_t kDefaultHashBits = 11;  // k = 11 in Section 3.4

// Default tile: 8 waves x 16 KiB per wave = 128 KiB per workgroup tile.
// The tune table (first matching entry wins) overrides it per kernel class,
// mode and text length.
std::mutex g_tune_mutex;
TileConfig g_tile = {8, 16};
std::vector<epsm_tune_entry> g_tune;
uint32_t g_default_hash_bits = kDefaultHashBits;
std::atomic<bool> g_debug_giveup{false};  // epsm_debug_force_giveup
constexpr uint32_t kMaxTuneEntries = 256;
std::vector<epsm_variant_entry> g_variants;  // epsm_set_variant_table (under g_tune_mutex)
constexpr uint32_t kMaxVariantEntries = 256;

uint32_t kernel_class(const DevPlan &d) {
    if (d.variant == EPSM_VARIANT_DNA) return EPSM_CLASS_DNA;
    if (d.variant == EPSM_VARIANT_FINGERPRINT || d.variant == EPSM_VARIANT_STRIDE)
        return EPSM_CLASS_FINGERPRINT;
    return (d.nl == 2 && d.pk < 4) ? EPSM_CLASS_BYTES : EPSM_CLASS_WORDS;
}

// EPSM_WRITE_AUTO: two phases (no tile waits on another) for searches of at
// least kTwoPhaseMinTiles tiles whose output capacity is at most one
// position per 128 text bytes; otherwise a single pass: short texts save the
// later kernels, and denser outputs are written while other tiles are still
// reading.  Measured on 1 GiB texts the two strategies tie at one position
// per 128 bytes; at one per 64 the single pass is 12% faster (parking a
// list and copying it moves 16 bytes per position, the single pass 8), at
// one per 256 the two-phase write is 12% faster (no look-back waits).
constexpr uint64_t kTwoPhaseMinTiles = 32;
constexpr uint64_t kTwoPhaseMaxDensity = 128;  // text bytes per output position

struct SearchChoice {
    TileConfig tile;
    uint32_t strategy;  // EPSM_WRITE_*: AUTO resolved by the caller
};

SearchChoice choice_for(const DevPlan &d, bool count_only, uint64_t n) {
    const uint32_t cls = kernel_class(d), mode = count_only ? 1u : 0u;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const epsm_tune_entry &e : g_tune)
        if (e.kernel_class == cls && e.count_only == mode && n <= e.n_max)
            return {{(int)e.waves, (int)e.pieces}, e.strategy};
    return {g_tile, EPSM_WRITE_AUTO};
}

// Device workspace of one search: [tile counts] (count only), [look-back
// status words] (single pass, cleared before the scan), or [tile counts][tile
// offsets][wave counts][slots] (two phase).  Only the status words are
// cleared; every other entry is written before it is read.
struct SearchWorkspace {
    size_t tcnt = 0, status = 0, toff = 0, wcnt = 0, slots = 0, total = 0, zeroed = 0;
};

SearchWorkspace search_workspace(uint64_t tiles, TileConfig tile, uint32_t write) {
    SearchWorkspace w;
    size_t at = 0;
    if (write == kWriteLookBack) {
        // one status word per tile, plus one that no tile publishes (the
        // target of the forced wait of epsm_debug_force_giveup)
        w.status = at;
        at += (tiles + 1) * sizeof(uint64_t);
        w.zeroed = at;
    } else if (write == kWriteTwoPhase) {
        w.tcnt = at;
        at += ((tiles * sizeof(uint32_t)) + 255) & ~size_t(255);
        w.toff = at;
        at += (((tiles + 1) * sizeof(uint64_t)) + 255) & ~size_t(255);
        w.wcnt = at;
        at += ((tiles * (uint64_t)tile.waves * sizeof(uint32_t)) + 255) & ~size_t(255);
        w.slots = at;
        at += tiles * (uint64_t)tile.bytes() / 32 * sizeof(uint32_t);
    } else {
        w.tcnt = at;
        at += tiles * sizeof(uint32_t);
    }
    w.total = std::max<size_t>(at, 256);
    return w;
}


// ---- workspace: one device buffer per (device, stream), grown on demand ----
// Growth is stream ordered (hipFreeAsync of the old buffer, hipMallocAsync of
// the new one, both on the stream), so it never waits for the device.  While
// the stream is being captured into a graph nothing may be allocated: a call
// that needs more than the stream holds fails, and the caller reserves first.
struct Workspace {
    uint8_t *ptr = nullptr;
    size_t bytes = 0;
    int device = -1;
};
std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

epsm_status workspace_for(hipStream_t stream, size_t bytes, uint8_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    Workspace &ws = g_ws[{dev, stream}];
    if (ws.bytes < bytes) {
        if (capturing(stream))
            return fail(EPSM_EUNSUPPORTED, "the stream is being captured and its workspace holds " +
                                               std::to_string(ws.bytes) + " bytes, this call needs " +
                                               std::to_string(bytes) + ": call epsm_reserve before capturing");
        if (ws.ptr) {
            e = hipFreeAsync(ws.ptr, stream);  // after the stream's earlier work
            ws.ptr = nullptr;
            ws.bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFreeAsync(workspace)");
        }
        size_t want = std::max<size_t>(bytes, 1 << 16);
        want = (want + 4095) & ~size_t(4095);
        e = hipMallocAsync((void **)&ws.ptr, want, stream);
        if (e != hipSuccess) {
            ws.ptr = nullptr;
            return hip_fail(e, "hipMallocAsync(workspace)");
        }
        ws.bytes = want;
        ws.device = dev;
    }
    *out = ws.ptr;
    return EPSM_OK;
}

// One device word per (device, stream) that kernels set when a bounded wait
// gives up; read back by epsm_stream_check.  Created (and cleared by a kernel
// on the stream, in stream order) by epsm_reserve or by the first search on
// the stream; never while the stream is being captured.
std::map<std::pair<int, hipStream_t>, uint32_t *> g_fault;

epsm_status fault_word(hipStream_t stream, bool create, uint32_t **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    auto it = g_fault.find({dev, stream});
    if (it != g_fault.end()) {
        *out = it->second;
        return EPSM_OK;
    }
    if (!create) return EPSM_OK;
    if (capturing(stream))
        return fail(EPSM_EUNSUPPORTED, "the stream is being captured and has no fault word yet: "
                                       "call epsm_reserve on it before capturing");
    uint32_t *f = nullptr;
    e = hipMallocAsync((void **)&f, 256, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(fault word)");
    e = launch_zero_u64((uint64_t *)f, 256 / 8, stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(f, stream);
        return hip_fail(e, "launch(zero fault word)");
    }
    g_fault[{dev, stream}] = f;
    *out = f;
    return EPSM_OK;
}

// ---- pinned staging of batch descriptors -----------------------------------
// A one-shot batch builds its descriptors on the host; they reach the device
// by one stream-ordered copy from pinned host memory, so the call returns
// without waiting for the device.  A block is reused once the event recorded
// after its copy has completed; a block copied under graph capture is read by
// every replay of the graph, so it is kept until epsm_release.
struct StagingBlock {
    uint8_t *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;  // recorded after the copy (not under capture)
    bool in_use = false;        // a copy may still read it (check `done`)
    bool filling = false;       // being filled by a caller: not available
    bool captured = false;      // read by a graph: never reused
    int device = -1;
};
std::mutex g_staging_mutex;
std::vector<StagingBlock *> g_staging;

// A free block of at least `bytes` (the smallest), else a new one.  Under
// graph capture nothing may be allocated or queried, so only blocks already
// known to be free qualify (epsm_reserve sets one aside).
epsm_status staging_acquire(size_t bytes, int dev, bool capture, StagingBlock **out) {
    std::lock_guard<std::mutex> lock(g_staging_mutex);
    StagingBlock *best = nullptr;
    for (StagingBlock *b : g_staging) {
        if (b->captured || b->filling || b->device != dev) continue;
        if (b->in_use && !capture && hipEventQuery(b->done) != hipErrorNotReady) b->in_use = false;
        if (b->in_use || b->bytes < bytes) continue;
        if (!best || b->bytes < best->bytes) best = b;
    }
    if (!best) {
        if (capture)
            return fail(EPSM_EUNSUPPORTED, "the stream is being captured and no free staging block of " +
                                               std::to_string(bytes) + " bytes exists: call epsm_reserve "
                                               "with batch_bytes >= epsm_batch_workspace before capturing");
        std::unique_ptr<StagingBlock> b(new (std::nothrow) StagingBlock());
        if (!b) return fail(EPSM_ENOMEM, "staging block");
        size_t want = 1 << 16;
        while (want < bytes) want *= 2;
        hipError_t e = hipHostMalloc((void **)&b->host, want, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(batch staging)");
        e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(b->host);
            return hip_fail(e, "hipEventCreate(batch staging)");
        }
        b->bytes = want;
        b->device = dev;
        best = b.release();
        g_staging.push_back(best);
    }
    best->in_use = true;
    best->filling = true;  // until staging_commit
    *out = best;
    return EPSM_OK;
}

// The copy out of blk is queued (queued = false: it was not): record its
// event, or keep the block for good when a graph captured the copy.
epsm_status staging_commit(StagingBlock *blk, hipStream_t s, bool queued) {
    hipError_t e = hipSuccess;
    const bool cap = queued && capturing(s);
    if (queued && !cap) e = hipEventRecord(blk->done, s);
    std::lock_guard<std::mutex> lock(g_staging_mutex);
    blk->filling = false;
    if (!queued) blk->in_use = false;
    if (cap || e != hipSuccess) blk->captured = true;  // no event to wait on: never reuse
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "hipEventRecord(batch staging)");
}

// ---- static scratch of epsm_search_noalloc ----------------------------------
// One array per device, in this code object's global memory, held from the
// library's load until the process ends.  Host code never uses the array's
// name as an address: hipGetSymbolAddress gives each device's copy once, with
// that device current, and the kernels take that pointer as their workspace.
// Bytes [0, 256) hold the fault word of its bounded waits, the rest is the
// search workspace.  Every call on a device shares its copy.
constexpr size_t kStaticFaultBytes = 256;
static __device__ __align__(256) uint8_t scratch[EPSM_NOALLOC_SCRATCH_BYTES];
static_assert(EPSM_NOALLOC_SCRATCH_BYTES > kStaticFaultBytes, "scratch too small");

constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mutex;
uint8_t *g_static_ptr[kMaxStaticDevices] = {};  // device address of `scratch`, per device

// The current device's copy of `scratch` (looked up on the first call on the
// device); create = false only reports one already looked up (else NULL).
epsm_status static_scratch(bool create, uint8_t **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxStaticDevices)
        return fail(EPSM_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_static_mutex);
    if (!g_static_ptr[dev] && create) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_static_ptr[dev] = (uint8_t *)ptr;
    }
    *out = g_static_ptr[dev];
    return EPSM_OK;
}

// A caller-fixed workspace (the static scratch) used instead of the stream's:
// a search whose layout does not fit fails instead of growing it.
struct FixedScratch {
    uint8_t *ws = nullptr;      // workspace
    size_t bytes = 0;           // its size
    uint32_t *fault = nullptr;  // fault word of bounded waits
};

epsm_status scratch_too_small(size_t need, size_t have) {
    return fail(EPSM_EUNSUPPORTED, "this search needs " + std::to_string(need) +
                                       " bytes of scratch; the static scratch holds " +
                                       std::to_string(have) + " (use epsm_search)");
}

uint32_t load_le32(const uint8_t *p, uint64_t m, uint64_t at) {
    uint32_t v = 0;
    for (int b = 0; b < 4; ++b)
        if (at + b < m) v |= (uint32_t)p[at + b] << (8 * b);
    return v;
}

epsm_status check_plan(epsm_plan_t plan) {
    if (!plan) return fail(EPSM_EINVAL, "plan is NULL");
    if (plan->device < 0) return fail(EPSM_EINVAL, "plan was built host-only (EPSM_PLAN_HOST_ONLY)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != plan->device) return fail(EPSM_EINVAL, "plan belongs to another device");
    return EPSM_OK;
}

// Count (write = false) or positions (write = true) for one text.
// Long patterns (strided filter): a count pass per workgroup, an exclusive
// scan of the counts, then (positions) the write pass; the total is the
// scan's last entry.  Workspace: [counts u32][offsets u64][scan block sums].
epsm_status run_stride(epsm_plan_t plan, const uint8_t *d_text, uint64_t n, int64_t *d_out,
                       uint64_t cap, uint64_t *d_n_hits, hipStream_t stream, bool write,
                       const FixedScratch *fx) {
    const DevPlan &d = plan->dev;
    StrideArgs a{};
    const uintptr_t addr = (uintptr_t)d_text;
    a.base = (const uint8_t *)(addr & ~uintptr_t(15));
    a.delta = addr & 15;
    a.last = a.delta + n - d.m;
    a.load_end = (a.delta + n + 15) & ~uint64_t(15);
    a.stride = d.stride;
    a.hash_bits = kStrideHashBits;
    a.table = d.stride_table;
    a.blocks = d.stride_blocks;
    a.pattern = d.pattern;
    a.m = d.m;
    a.first_block = (a.delta + a.stride - 1) / a.stride;
    const uint64_t last_block = (a.last + a.stride - 1) / a.stride;
    a.num_blocks = last_block >= a.first_block ? last_block - a.first_block + 1 : 0;
    const uint64_t tiles = (a.num_blocks + kStrideBlocksPerTile - 1) / kStrideBlocksPerTile;
    if (tiles > 0x7FFFFFFFull) return fail(EPSM_EUNSUPPORTED, "text too long for the tile grid");
    const size_t cnt_bytes = (tiles * sizeof(uint32_t) + 255) & ~size_t(255);
    const size_t off_bytes = ((tiles + 1) * sizeof(uint64_t) + 255) & ~size_t(255);
    const size_t bsum_bytes = ((tiles + kScanBlock - 1) / kScanBlock + 1) * sizeof(uint64_t);
    uint8_t *ws = nullptr;
    const size_t need = cnt_bytes + off_bytes + bsum_bytes;
    if (fx) {
        if (need > fx->bytes) return scratch_too_small(need, fx->bytes);
        ws = fx->ws;
    } else {
        epsm_status st = workspace_for(stream, need, &ws);
        if (st != EPSM_OK) return st;
    }
    a.tile_count = (uint32_t *)ws;
    uint64_t *offsets = (uint64_t *)(ws + cnt_bytes);
    a.tile_offset = offsets;
    hipError_t e = launch_stride(a, (uint32_t)tiles, stream);
    if (e == hipSuccess)
        e = launch_scan_counts(a.tile_count, tiles, offsets, (uint64_t *)(ws + cnt_bytes + off_bytes), stream);
    if (e == hipSuccess && write && cap > 0) {
        a.write = 1;
        a.out = d_out;
        a.cap = cap;
        e = launch_stride(a, (uint32_t)tiles, stream);
    }
    if (e == hipSuccess) e = launch_copy_u64(offsets + tiles, d_n_hits, stream);
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "launch(stride)");
}

epsm_status run_search(epsm_plan_t plan, const uint8_t *d_text, uint64_t n, int64_t *d_out,
                       uint64_t cap, uint64_t *d_n_hits, hipStream_t stream, bool write,
                       bool dna = false, const FixedScratch *fx = nullptr) {
    epsm_status st = check_plan(plan);
    if (st != EPSM_OK) return st;
    if (dna != (plan->dev.variant == EPSM_VARIANT_DNA))
        return fail(EPSM_EINVAL, dna ? "a packed DNA search needs a plan made with EPSM_PLAN_DNA"
                                     : "a plan made with EPSM_PLAN_DNA needs a packed DNA search");
    if (!d_n_hits) return fail(EPSM_EINVAL, "d_n_hits is NULL");
    if (n > 0 && !d_text) return fail(EPSM_EINVAL, "d_text is NULL");
    if (write && cap > 0 && !d_out) return fail(EPSM_EINVAL, "d_out is NULL with out_capacity > 0");
    const uint64_t m = plan->dev.m;
    if (n == 0 || m > n) {
        hipError_t e = launch_set_u64(d_n_hits, 0, stream);
        return e == hipSuccess ? EPSM_OK : hip_fail(e, "launch(set)");
    }
    if (plan->dev.variant == EPSM_VARIANT_STRIDE)
        return run_stride(plan, d_text, n, d_out, cap, d_n_hits, stream, write, fx);
    // coordinates are bytes, or 2-bit symbols (four per byte) for packed DNA
    ScanArgs a{};
    const uint32_t sh = dna ? 2u : 0u;
    const uintptr_t addr = (uintptr_t)d_text;
    a.base = (const uint8_t *)(addr & ~uintptr_t(15));
    a.delta = (uint64_t)(addr & 15) << sh;
    a.last = a.delta + n - m;
    a.load_end = ((((a.delta + n) + (1u << sh) - 1) >> sh) + 15) & ~uint64_t(15);  // bytes
    a.shift = sh;
    a.out = d_out;
    a.cap = write ? cap : 0;
    a.n_hits = d_n_hits;
    a.plan = plan->dev;
    const uint64_t wsym = dna_wide_tile_symbols();
    const uint64_t wtiles = (a.last + 1 + wsym - 1) / wsym;
    if (dna && fx) return fail(EPSM_EINVAL, "packed DNA searches use the stream workspace");
    if (dna && (!write || cap <= wtiles * kDnaWideMaxPerTile)) {
        // packed: the wide-lane kernel (block filter for m >= 8, direct
        // compare below); positions by a count pass (tile and wave counts,
        // and up to 64 hits of each wave parked), the tile offsets, and a
        // write pass over the tiles with hits that copies the parked hits
        // and re-reads only the spans of waves with more.  Denser outputs
        // (capacity above kDnaWideMaxPerTile per tile) take the scan below.
        if (wtiles > 0x7FFFFFFFull) return fail(EPSM_EUNSUPPORTED, "text too long for the tile grid");
        a.num_tiles = (uint32_t)wtiles;
        a.write = write ? kWriteTwoPhase : kWriteNone;
        const size_t cnt_bytes = (wtiles * sizeof(uint32_t) + 255) & ~size_t(255);
        const size_t off_bytes = ((wtiles + 1) * sizeof(uint64_t) + 255) & ~size_t(255);
        const size_t wave_bytes = (wtiles * dna_wide_waves() * sizeof(uint32_t) + 255) & ~size_t(255);
        const size_t slot_bytes = wtiles * dna_wide_waves() * dna_wide_slot() * sizeof(uint32_t);
        uint8_t *ws = nullptr;
        st = workspace_for(stream, cnt_bytes + (write ? off_bytes + wave_bytes + slot_bytes : 0), &ws);
        if (st != EPSM_OK) return st;
        a.tcnt = (uint32_t *)ws;
        a.toff = (uint64_t *)(ws + cnt_bytes);
        a.wcnt = (uint32_t *)(ws + cnt_bytes + off_bytes);
        a.slots = (uint32_t *)(ws + cnt_bytes + off_bytes + wave_bytes);
        hipError_t e = launch_dna_wide(a, write ? 1 : 0, stream);
        if (e == hipSuccess)
            e = write ? launch_tile_offsets(a.tcnt, a.num_tiles, a.toff, d_n_hits, stream)
                      : launch_sum_tiles(a.tcnt, a.num_tiles, d_n_hits, stream);
        if (e == hipSuccess && write) e = launch_dna_wide(a, 2, stream);
        return e == hipSuccess ? EPSM_OK : hip_fail(e, "launch(dna wide)");
    }
    const SearchChoice ch = choice_for(plan->dev, !write, n);
    const TileConfig tile = ch.tile;
    const uint64_t tile_bytes = (uint64_t)tile.bytes();
    const uint64_t tiles = (a.last + 1 + tile_bytes - 1) / tile_bytes;
    if (tiles > 0x7FFFFFFFull) return fail(EPSM_EUNSUPPORTED, "text too long for the tile grid");
    a.num_tiles = (uint32_t)tiles;
    if (!write)
        a.write = kWriteNone;
    else if (ch.strategy == EPSM_WRITE_AUTO)
        a.write = tiles >= kTwoPhaseMinTiles && cap <= n / kTwoPhaseMaxDensity ? kWriteTwoPhase
                                                                             : kWriteLookBack;
    else
        a.write = ch.strategy == EPSM_WRITE_TWO_PHASE ? kWriteTwoPhase : kWriteLookBack;

    SearchWorkspace L = search_workspace(tiles, tile, a.write);
    uint8_t *ws = nullptr;
    if (fx) {
        // a fixed scratch: a two-phase layout (about n/8 bytes) that does not
        // fit falls back to the single pass (8 bytes per tile)
        if (L.total > fx->bytes && a.write == kWriteTwoPhase) {
            a.write = kWriteLookBack;
            L = search_workspace(tiles, tile, a.write);
        }
        if (L.total > fx->bytes) return scratch_too_small(L.total, fx->bytes);
        ws = fx->ws;
    } else {
        st = workspace_for(stream, L.total, &ws);
        if (st != EPSM_OK) return st;
    }
    a.tcnt = (uint32_t *)(ws + L.tcnt);
    a.status = (uint64_t *)(ws + L.status);
    a.toff = (uint64_t *)(ws + L.toff);
    a.wcnt = (uint32_t *)(ws + L.wcnt);
    a.slots = (uint32_t *)(ws + L.slots);
    if (a.write == kWriteLookBack) {
        if (fx)
            a.fault = fx->fault;
        else
            st = fault_word(stream, true, &a.fault);
        if (st != EPSM_OK) return st;
        a.debug_giveup = g_debug_giveup.load() ? 1u : 0u;
    }
    hipError_t e = hipSuccess;
    if (L.zeroed) {
        e = launch_zero_u64((uint64_t *)ws, L.zeroed / 8, stream);
        if (e != hipSuccess) return hip_fail(e, "launch(zero)");
    }

    e = launch_scan(a, tile, (int)tiles, stream);
    if (e != hipSuccess) return hip_fail(e, "launch(scan)");
    if (a.write == kWriteNone)
        e = launch_sum_tiles(a.tcnt, a.num_tiles, d_n_hits, stream);
    else if (a.write == kWriteTwoPhase) {
        e = launch_tile_offsets(a.tcnt, a.num_tiles, a.toff, d_n_hits, stream);
        if (e == hipSuccess) e = launch_expand(a, tile, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "launch(sum_tiles/expand)");
    return EPSM_OK;
}


// ---- batched search: host side ----------------------------------------------

int g_batch_waves = 8;  // batch tile = g_batch_waves KiB

BatchPtrs batch_ptrs(uint8_t *base, const BatchLayout &L) {
    return {(BatchTextDesc *)(base + L.texts), (BatchPairDesc *)(base + L.kpairs),
            (BatchSpan *)(base + L.spans), (uint32_t *)(base + L.gtables), (BatchUnit *)(base + L.units),
            (uint32_t *)(base + L.park), (uint32_t *)(base + L.parkn), (uint32_t *)(base + L.ptc),
            (uint64_t *)(base + L.pto), (uint64_t *)(base + L.bsum), (int64_t *)(base + L.shift),
            (uint64_t *)(base + L.pbsum)};
}

epsm_status build_batch(const epsm_batch *b, int waves, HostBatch &hb, bool check_outputs,
                        bool group) {
    if (!b) return fail(EPSM_EINVAL, "batch is NULL");
    if (b->flags & ~(EPSM_BATCH_COUNT_ONLY | EPSM_BATCH_NO_GROUPS))
        return fail(EPSM_EINVAL, "unknown batch flags");
    if (b->flags & EPSM_BATCH_NO_GROUPS) group = false;
    if (b->n_texts && !b->texts) return fail(EPSM_EINVAL, "texts is NULL");
    if (b->n_pairs && !b->pairs) return fail(EPSM_EINVAL, "pairs is NULL");
    if (check_outputs) {
        if (b->n_pairs && (!b->d_counts || !b->d_offsets))
            return fail(EPSM_EINVAL, "d_counts and d_offsets are required");
        const bool write = !(b->flags & EPSM_BATCH_COUNT_ONLY);
        if (write && b->out_capacity && !b->d_out)
            return fail(EPSM_EINVAL, "d_out is NULL with out_capacity > 0");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const uint64_t tile_bytes = (uint64_t)waves * kWavePiece;
    hb = HostBatch();  // callers may reuse a HostBatch: start from empty vectors
    hb.waves = waves;
    hb.texts.assign(b->n_texts, BatchTextDesc{});
    std::vector<uint32_t> text_tiles(b->n_texts, 0), text_pairs(b->n_texts, 0);
    for (uint32_t i = 0; i < b->n_texts; ++i) {
        const epsm_text_ref &t = b->texts[i];
        if (t.n && !t.d_text) return fail(EPSM_EINVAL, "a text with n > 0 has a NULL pointer");
        const uintptr_t addr = (uintptr_t)t.d_text;
        BatchTextDesc &d = hb.texts[i];
        d.base = (const uint8_t *)(addr & ~uintptr_t(15));
        d.delta = (uint32_t)(addr & 15);
        d.n = t.n;
        const uint64_t tiles = t.n ? (d.delta + t.n + tile_bytes - 1) / tile_bytes : 0;
        if (tiles > 0xFFFFFFFFull) return fail(EPSM_EUNSUPPORTED, "text too long for a batch");
        text_tiles[i] = (uint32_t)tiles;
        d.tiles = (uint32_t)tiles;
    }
    hb.pairs.assign(b->n_pairs, BatchPairDesc{});
    uint64_t entries = 0;
    // per pair, read once from its plan: m (the passes below read it from
    // this compact array, not from descriptors 160 bytes apart), whether it
    // is a pair with entries of a plan that lives on the host, and whether
    // that plan has a table
    std::vector<uint32_t> pm(b->n_pairs, 0);
    std::vector<uint8_t> host_only(b->n_pairs, 0), has_table(b->n_pairs, 0);
    for (uint32_t k = 0; k < b->n_pairs; ++k) {
        const epsm_pair_ref &pr = b->pairs[k];
        if (pr.text >= b->n_texts) return fail(EPSM_EINVAL, "pair refers to a text out of range");
        if (!pr.plan) return fail(EPSM_EINVAL, "pair has a NULL plan");
        if (pr.plan->dev.variant == EPSM_VARIANT_DNA)
            return fail(EPSM_EINVAL, "batches search byte texts; EPSM_PLAN_DNA plans are not accepted");
        if (pr.plan->device >= 0 && pr.plan->device != dev)
            return fail(EPSM_EINVAL, "plan belongs to another device");
        BatchPairDesc &d = hb.pairs[k];
        d.plan = pr.plan->dev;
        if (d.plan.variant == EPSM_VARIANT_STRIDE) d.plan.variant = EPSM_VARIANT_FINGERPRINT;  // tile filter
        d.text = pr.text;
        d.tiles = pr.plan->dev.m <= b->texts[pr.text].n ? text_tiles[pr.text] : 0;
        pm[k] = (uint32_t)std::min<uint64_t>(d.plan.m, 0xFFFFFFFFull);
        host_only[k] = pr.plan->device < 0 && d.tiles;
        has_table[k] = !pr.plan->table.empty();
        entries += d.tiles;  // cnt_base is given in kernel order below
        if (d.tiles) text_pairs[pr.text]++;
    }
    hb.entries = entries;
    std::vector<uint8_t> in_group(b->n_pairs, 0);  // filtered in a group by the count pass
    // pairs grouped by text (the caller's order kept within a text)
    std::vector<uint32_t> start(b->n_texts + 1, 0);
    for (uint32_t i = 0; i < b->n_texts; ++i) start[i + 1] = start[i] + text_pairs[i];
    std::vector<uint32_t> order(start[b->n_texts], 0);
    std::vector<uint32_t> fillp(start.begin(), start.end() - 1);
    for (uint32_t k = 0; k < b->n_pairs; ++k)
        if (hb.pairs[k].tiles) order[fillp[hb.pairs[k].text]++] = k;
    uint64_t units = 0;
    for (uint32_t i = 0; i < b->n_texts; ++i)
        if (text_pairs[i]) units += text_tiles[i];
    // kernel order: a text with at least kGroupMin patterns of m >= 4 filters
    // them in the count pass in groups of up to kGroupMax, each through one
    // bucket table of their first four (m = 4..7) or eight (m >= 8) bytes;
    // its other pairs, filtered one by one, come first
    hb.korder.reserve(order.size());
    {
        uint64_t groups = 0;  // reserved up front: the tables come to 5 KiB a group
        for (uint32_t i = 0; i < b->n_texts; ++i) {
            uint32_t short_ = 0, long_ = 0;
            for (uint32_t q = start[i]; q < start[i + 1]; ++q) {
                short_ += pm[order[q]] >= 4 && pm[order[q]] < 8;
                long_ += pm[order[q]] >= 8;
            }
            if (group && short_ + long_ >= kGroupMin)
                groups += (short_ + kGroupMax - 1) / kGroupMax + (long_ + kGroupMax - 1) / kGroupMax;
        }
        hb.group_tables.reserve(groups * kGroupTableWords);
    }
    for (uint32_t i = 0; i < b->n_texts; ++i) {
        BatchTextDesc &d = hb.texts[i];
        uint32_t words = 0;
        for (uint32_t q = start[i]; q < start[i + 1]; ++q) words += pm[order[q]] >= 4;
        const bool grouped = group && words >= kGroupMin;
        d.pair_begin = (uint32_t)hb.korder.size();
        for (uint32_t q = start[i]; q < start[i + 1]; ++q)
            if (!grouped || pm[order[q]] < 4) hb.korder.push_back(order[q]);
        d.solo_end = (uint32_t)hb.korder.size();
        d.group_begin = (uint32_t)(hb.group_tables.size() / kGroupTableWords);
        // groups of the patterns of m = 4..7 (4-byte keys), then of m >= 8
        // (8-byte keys); each kind starts a new group
        for (int kind = 0; kind < 2; ++kind) {
            if (kind == 1) {
                d.short_end = (uint32_t)hb.korder.size();
                d.long_group = (uint32_t)(hb.group_tables.size() / kGroupTableWords);
            }
            if (!grouped) continue;
            const uint32_t kind_begin = (uint32_t)hb.korder.size();
            for (uint32_t q = start[i]; q < start[i + 1]; ++q) {
                const uint32_t k = order[q];
                if (pm[k] < 4 || (pm[k] >= 8) != (kind == 1)) continue;
                const DevPlan &pl = hb.pairs[k].plan;
                const uint32_t member = (uint32_t)(hb.korder.size() - kind_begin) % kGroupMax;
                if (member == 0) hb.group_tables.resize(hb.group_tables.size() + kGroupTableWords, 0);
                const uint32_t bucket = kind == 0 ? group_bucket(pl.pw[0]) : group_bucket8(pl.pw[0], pl.pw[1]);
                uint32_t *table = hb.group_tables.data() + hb.group_tables.size() - kGroupTableWords;
                table[bucket] |= 1u << member;
                reinterpret_cast<uint8_t *>(table + kGroupBuckets)[bucket] = 1;
                hb.korder.push_back(k);
                in_group[k] = 1;
            }
        }
        d.pair_end = (uint32_t)hb.korder.size();
        d.group_end = (uint32_t)(hb.group_tables.size() / kGroupTableWords);
    }
    // host-only plans: their table (for pairs filtered alone) and, for the
    // tail check, their pattern travel in the batch's own device buffer.
    // Grouped pairs need no table: the group filter compares pattern words, and a
    // write-pass recompute of a grouped fingerprint pair compares its first
    // 16 bytes directly (its batch descriptor is made a direct one) and
    // checks the rest with the tail check
    hb.blob_table.assign(b->n_pairs, kNoBlob);
    hb.blob_pattern.assign(b->n_pairs, kNoBlob);
    for (uint32_t k = 0; k < b->n_pairs; ++k) {
        if (!in_group[k]) continue;
        DevPlan &pl = hb.pairs[k].plan;
        if (pl.variant == EPSM_VARIANT_FINGERPRINT) {
            pl.variant = EPSM_VARIANT_DIRECT;
            pl.hash_bits = 0;
            pl.table = nullptr;
        }
    }
    // one copy of a table per distinct plan; patterns (at most 48 bytes
    // padded) are copied per pair
    std::unordered_map<epsm_plan_t, uint64_t> table_at;
    auto append = [&](const uint8_t *src, size_t n) {
        const uint64_t at = hb.blob.size();
        hb.blob.insert(hb.blob.end(), src, src + n);
        hb.blob.resize((hb.blob.size() + 15) & ~size_t(15), 0);
        return at;
    };
    for (uint32_t k = 0; k < b->n_pairs; ++k) {
        if (!host_only[k]) continue;
        epsm_plan_t pl = b->pairs[k].plan;
        if (!in_group[k] && has_table[k]) {
            auto it = table_at.find(pl);
            if (it == table_at.end())
                it = table_at.emplace(pl, append((const uint8_t *)pl->table.data(),
                                                 pl->table.size() * sizeof(uint16_t))).first;
            hb.blob_table[k] = it->second;
        }
        // the pattern goes along whenever a kernel may read it: for m > 16,
        // the tail check past the register words and the write pass, which
        // compares only 16 bytes from registers (up to 16 bytes, every
        // variant holds the whole pattern in its register words)
        if (pm[k] > 16) hb.blob_pattern[k] = append(pl->pattern.data(), pl->pattern.size());
    }
    // entries in kernel order: a text's pairs, each with one entry per tile
    uint64_t next = 0;
    for (uint32_t i = 0; i < b->n_texts; ++i) {
        BatchTextDesc &d = hb.texts[i];
        d.entry_begin = next;
        for (uint32_t q = d.pair_begin; q < d.pair_end; ++q) {
            hb.pairs[hb.korder[q]].cnt_base = next;
            next += text_tiles[i];
        }
    }
    if (next != entries) return fail(EPSM_EINVAL, "internal: batch entries do not add up");
    if (units > 0x7FFFFFFFull) return fail(EPSM_EUNSUPPORTED, "batch has too many tiles");
    hb.units.reserve(units);
    for (uint32_t i = 0; i < b->n_texts; ++i)
        if (text_pairs[i])
            for (uint32_t t = 0; t < text_tiles[i]; ++t) hb.units.push_back({i, t});
    return EPSM_OK;
}

epsm_status upload_batch(HostBatch &hb, const BatchLayout &L, uint8_t *dev, hipStream_t s, bool sync) {
    for (size_t k = 0; k < hb.pairs.size(); ++k) {  // point host-only plans at the blob copy
        if (hb.blob_table[k] != kNoBlob)
            hb.pairs[k].plan.table = (const uint16_t *)(dev + L.blob + hb.blob_table[k]);
        if (hb.blob_pattern[k] != kNoBlob)
            hb.pairs[k].plan.pattern = dev + L.blob + hb.blob_pattern[k];
    }
    const size_t bytes = L.ptc;  // the descriptors end where the count arrays begin
    if (bytes == 0) return EPSM_OK;
    int devid = 0;
    hipError_t e = hipGetDevice(&devid);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    StagingBlock *blk = nullptr;
    epsm_status st = staging_acquire(bytes, devid, capturing(s), &blk);
    if (st != EPSM_OK) return st;
    uint8_t *h = blk->host;
    auto put = [&](size_t at, const void *src, size_t n) {
        if (n) std::memcpy(h + at, src, n);
    };
    put(L.blob, hb.blob.data(), hb.blob.size());
    put(L.texts, hb.texts.data(), hb.texts.size() * sizeof(BatchTextDesc));
    for (size_t i = 0; i < hb.korder.size(); ++i)
        put(L.kpairs + i * sizeof(BatchPairDesc), &hb.pairs[hb.korder[i]], sizeof(BatchPairDesc));
    std::vector<uint32_t> kq(hb.pairs.size(), kNoKq);
    for (size_t q = 0; q < hb.korder.size(); ++q) kq[hb.korder[q]] = (uint32_t)q;
    for (size_t k = 0; k < hb.pairs.size(); ++k) {
        const BatchSpan sp{hb.pairs[k].cnt_base, hb.pairs[k].tiles, kq[k]};
        put(L.spans + k * sizeof(BatchSpan), &sp, sizeof(sp));
    }
    put(L.gtables, hb.group_tables.data(), hb.group_tables.size() * sizeof(uint32_t));
    put(L.units, hb.units.data(), hb.units.size() * sizeof(BatchUnit));
    e = hipMemcpyAsync(dev, h, bytes, hipMemcpyHostToDevice, s);
    st = staging_commit(blk, s, e == hipSuccess);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    if (st != EPSM_OK) return st;
    if (sync) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    }
    return EPSM_OK;
}

// The kernel sequence of one batch (stream ordered, no host round trip):
// count pass, scan, per-pair counts/offsets, then the write pass.
epsm_status run_batch_count(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                            hipStream_t s) {
    BatchArgs a{};
    a.texts = P.texts;
    a.kpairs = P.kpairs;
    a.group_tables = P.gtables;
    a.units = P.units;
    a.park = P.park;
    a.park_n = P.parkn;
    a.pt_count = P.ptc;
    a.pt_offset = P.pto;
    a.write = 0;
    hipError_t e = launch_batch(a, hb.waves, (uint32_t)hb.units.size(), s);
    if (e == hipSuccess) e = launch_scan_counts(P.ptc, hb.entries, P.pto, P.bsum, s);
    if (e == hipSuccess)
        e = launch_batch_finalize(P.spans, (uint32_t)hb.pairs.size(), P.pto, hb.entries, o.d_counts,
                                  o.d_offsets, o.d_total, P.shift, P.pbsum, s);
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "batch launch (count)");
}

epsm_status run_batch_write(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                            hipStream_t s) {
    if (!o.write || !o.cap) return EPSM_OK;
    BatchArgs a{};
    a.texts = P.texts;
    a.kpairs = P.kpairs;
    a.units = P.units;
    a.park = P.park;
    a.park_n = P.parkn;
    a.pt_count = P.ptc;
    a.pt_offset = P.pto;
    a.shift = P.shift;
    a.entries = hb.entries;
    a.out = o.d_out;
    a.cap = o.cap;
    a.write = 1;
    hipError_t e = launch_batch(a, hb.waves, (uint32_t)hb.units.size(), s);
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "batch launch (write)");
}

epsm_status run_batch(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                      hipStream_t s) {
    epsm_status st = run_batch_count(P, hb, o, s);
    return st == EPSM_OK ? run_batch_write(P, hb, o, s) : st;
}

int batch_waves() { return g_batch_waves; }

}  // namespace host
}  // namespace epsm

using namespace epsm::host;

struct epsm_batch_plan_s {
    HostBatch hb;               // sizes; units kept only for their count
    BatchPtrs ptrs{};
    epsm_batch_outputs out{};
    uint8_t *mem = nullptr;
    int device = -1;
    std::mutex mutex;
    std::map<hipStream_t, hipGraphExec_t> graphs;
};

extern "C" {

uint32_t epsm_fingerprint(uint32_t lo, uint32_t hi, uint32_t k, int collide) {
    if (collide) return 0;
    return fp_hash(lo, hi, k);
}

epsm_status epsm_plan(const uint8_t *pattern, uint64_t m, uint32_t flags, epsm_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(EPSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pattern) return fail(EPSM_EINVAL, "pattern is NULL");
    if (m == 0) return fail(EPSM_EINVAL, "m must be > 0");
    if (m > EPSM_MAX_M) return fail(EPSM_EUNSUPPORTED, "m exceeds EPSM_MAX_M");
    if (flags & ~kKnownPlanFlags) return fail(EPSM_EINVAL, "unknown plan flags");
    if ((flags & EPSM_PLAN_FORCE_DIRECT) && (flags & EPSM_PLAN_FORCE_FINGERPRINT))
        return fail(EPSM_EINVAL, "FORCE_DIRECT and FORCE_FINGERPRINT are exclusive");
    const uint32_t sigma = (flags >> 16) & 0x1FFu;  // alphabet hint, 0 = unknown
    if (sigma > 256) return fail(EPSM_EINVAL, "EPSM_PLAN_SIGMA takes 1..256 (0: unknown)");
    const bool dna = (flags & EPSM_PLAN_DNA) != 0;
    const bool forced = flags & (EPSM_PLAN_FORCE_DIRECT | EPSM_PLAN_FORCE_FINGERPRINT | EPSM_PLAN_COLLIDE);
    // the variant table's row for (m, sigma), if any
    uint32_t row_variant = 0, row_flags = 0, table_row = 0;
    uint32_t k = (flags >> 8) & 0xF;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        if (!dna && !forced) {
            for (size_t i = 0; i < g_variants.size(); ++i) {
                const epsm_variant_entry &e = g_variants[i];
                if (m >= e.m_min && m <= e.m_max && sigma >= e.sigma_min && sigma <= e.sigma_max) {
                    row_variant = e.variant;
                    row_flags = e.flags;
                    table_row = (uint32_t)i + 1;
                    break;
                }
            }
        }
        if (k == 0) k = (row_flags >> 8) & 0xF;
        if (k == 0) k = g_default_hash_bits;
    }
    if (k < 8 || k > 14) return fail(EPSM_EINVAL, "hash bits must be in [8, 14]");
    const uint32_t eff = flags | (row_flags & (EPSM_PLAN_SHORT_RUN | EPSM_PLAN_PREFIX4));

    if (dna) {
        if (flags & (EPSM_PLAN_FORCE_DIRECT | EPSM_PLAN_FORCE_FINGERPRINT | EPSM_PLAN_COLLIDE |
                     EPSM_PLAN_HASH_BITS(0xF)))
            return fail(EPSM_EINVAL, "EPSM_PLAN_DNA takes no variant or fingerprint flags");
        for (uint64_t i = 0; i < m; ++i)
            if (pattern[i] > 3) return fail(EPSM_EINVAL, "DNA pattern codes must be 0..3");
    }
    bool fingerprint = !dna && m >= 16;
    if (row_variant == EPSM_VARIANT_DIRECT) fingerprint = false;
    if (row_variant == EPSM_VARIANT_FINGERPRINT || row_variant == EPSM_VARIANT_STRIDE) fingerprint = true;
    if (flags & EPSM_PLAN_FORCE_DIRECT) fingerprint = false;
    if (flags & EPSM_PLAN_FORCE_FINGERPRINT) {
        if (m < 15) return fail(EPSM_EINVAL, "the fingerprint variant needs m >= 15");
        fingerprint = true;
    }

    epsm_plan_s *p = new (std::nothrow) epsm_plan_s();
    if (!p) return fail(EPSM_ENOMEM, "plan allocation");
    p->pattern.assign(pattern, pattern + m);
    p->flags = flags;
    p->table_row = table_row;
    DevPlan &d = p->dev;
    d.m = m;
    for (int j = 0; j < 8; ++j) {
        d.pw[j] = load_le32(pattern, m, 4ull * j);
        uint32_t mask = 0;
        for (int b = 0; b < 4; ++b)
            if (4ull * j + b < m) mask |= 0xFFu << (8 * b);
        d.pmask[j] = mask;
    }
    d.variant = fingerprint ? EPSM_VARIANT_FINGERPRINT : EPSM_VARIANT_DIRECT;
    // a lane's register run spans three 16-byte blocks only where it must
    // hold 8 pattern words (direct compare of m > 16); the fingerprint
    // filter needs bytes 0..23 of the run, verifies 16 bytes from registers
    // and the rest with the tail check, which keeps it at two blocks and
    // fewer VGPRs
    d.nl = (!fingerprint && m > 16 && !(eff & EPSM_PLAN_SHORT_RUN)) ? 3 : 2;
    const uint32_t nwmax = 4 * d.nl - 4;
    const uint64_t words = (m + 3) / 4;
    d.nw = (uint32_t)std::min<uint64_t>(words, nwmax);
    // prefix bytes of the direct filter: for m >= 5 one 64-bit compare of
    // the first min(m, 8) bytes (a register run of two blocks holds every
    // window it needs), so m <= 8 needs no verify at all
    d.pk = (uint32_t)std::min<uint64_t>(m, 4);
    if (!fingerprint && d.nl == 2 && m >= 5 && !(eff & EPSM_PLAN_PREFIX4))
        d.pk = (uint32_t)std::min<uint64_t>(m, 8);
    d.collide = (flags & EPSM_PLAN_COLLIDE) ? 1 : 0;
    d.hash_bits = fingerprint ? k : 0;
    if (dna) {
        // 16 symbols per word, symbol t of word j at bits 2t; the first three
        // words are compared from registers, the rest by the tail check
        d.variant = EPSM_VARIANT_DNA;
        d.nl = 1;
        d.pk = m >= 16 ? 16 : 4;  // 16: the first word needs no mask
        d.nw = (uint32_t)std::min<uint64_t>((m + 15) / 16, 3);
        for (int j = 0; j < 8; ++j) {
            uint32_t wv = 0, mv = 0;
            for (int t = 0; t < 16; ++t) {
                const uint64_t i = 16ull * j + t;
                if (i < m) {
                    wv |= (uint32_t)pattern[i] << (2 * t);
                    mv |= 3u << (2 * t);
                }
            }
            d.pw[j] = wv;
            d.pmask[j] = mv;
        }
        if (m >= 16) {
            // Section 3.4's filter over packed symbols: every occurrence holds
            // an aligned 8-symbol block at pattern offset j in [0, 7]; bit j of
            // entry v is set iff the block of symbols j..j+7 (16 bits, symbol t
            // at bits 2t) hashes to v
            d.hash_bits = kDnaHashBits;
            p->table.assign((size_t)1 << kDnaHashBits, 0);
            for (uint32_t j = 0; j < 8; ++j) {
                uint32_t block = 0;
                for (uint32_t t = 0; t < 8; ++t) block |= (uint32_t)pattern[j + t] << (2 * t);
                p->table[fp_hash(block, 0, kDnaHashBits)] |= (uint16_t)(1u << j);
            }
        } else if (m >= 8) {
            // the same with 4-symbol blocks at offsets j in [0, 3] (every
            // occurrence of m >= 7 holds one); an 8-bit block indexes the
            // 256-entry table directly
            d.pk = 8;
            d.hash_bits = 8;
            p->table.assign((size_t)1 << 8, 0);
            for (uint32_t j = 0; j < 4; ++j) {
                uint32_t block = 0;
                for (uint32_t t = 0; t < 4; ++t) block |= (uint32_t)pattern[j + t] << (2 * t);
                p->table[block] |= (uint16_t)(1u << j);
            }
        }
    }
    if (fingerprint) {
        // Section 3.4: L[v] = { j : h(p[j..j+7]) = v }, offsets j in [0, 7].
        p->table.assign((size_t)1 << k, 0);
        for (uint32_t j = 0; j < 8 && j + 8 <= m; ++j) {
            const uint32_t lo = load_le32(pattern, m, j), hi = load_le32(pattern, m, j + 4);
            const uint32_t v = epsm_fingerprint(lo, hi, k, d.collide);
            p->table[v] |= (uint16_t)(1u << (8 - j));
        }
    }
    // Long patterns: EPSMc with stride S (Section 3.4 inspects one block per
    // stride), S the largest power of two <= min(m - 7, kStrideMax), at least
    // kStrideMin (kStrideMinRow when a variant-table row asks for the strided
    // filter); the table lists, per hash value, the offsets j in [0, S) of
    // the pattern blocks p[j..j+7] with that hash, in ascending j.  A table
    // row of the per-block fingerprint filter keeps the stride off.
    const uint32_t s_min = row_variant == EPSM_VARIANT_STRIDE ? kStrideMinRow : kStrideMin;
    if (fingerprint && !forced && !(flags & EPSM_PLAN_NO_STRIDE) && row_variant != EPSM_VARIANT_FINGERPRINT &&
        m >= s_min + 7) {
        uint32_t S = s_min;
        while (S * 2 <= kStrideMax && S * 2 + 7 <= m) S *= 2;
        const uint32_t buckets = 1u << kStrideHashBits;
        std::vector<uint32_t> hv(S);
        std::vector<uint16_t> &t = p->stride_table;
        t.assign(buckets + 1 + S, 0);
        for (uint32_t j = 0; j < S; ++j) {
            hv[j] = fp_hash(load_le32(pattern, m, j), load_le32(pattern, m, j + 4), kStrideHashBits);
            t[hv[j] + 1]++;
        }
        for (uint32_t v = 0; v < buckets; ++v) t[v + 1] += t[v];
        std::vector<uint16_t> fillp(t.begin(), t.begin() + buckets);
        for (uint32_t j = 0; j < S; ++j) t[buckets + 1 + fillp[hv[j]]++] = (uint16_t)j;
        // the pattern block of each listed offset, in the same order
        p->stride_blocks.resize(2 * (size_t)S);
        for (uint32_t i = 0; i < S; ++i) {
            const uint32_t j = t[buckets + 1 + i];
            p->stride_blocks[2 * i] = load_le32(pattern, m, j);
            p->stride_blocks[2 * i + 1] = load_le32(pattern, m, j + 4);
        }
        d.stride = S;
        d.variant = EPSM_VARIANT_STRIDE;
    }

    if (!(flags & EPSM_PLAN_HOST_ONLY)) {
        hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "hipGetDevice");
        }
        // one device block: [pattern, zero padded to 16 bytes][table]
        const size_t pat_bytes = (m + 15) & ~uint64_t(15);
        const size_t tab_bytes = p->table.size() * sizeof(uint16_t);
        const size_t sblk_bytes = p->stride_blocks.size() * sizeof(uint32_t);  // first: 8-byte aligned
        const size_t stab_bytes = p->stride_table.size() * sizeof(uint16_t);
        std::vector<uint8_t> staging(pat_bytes + tab_bytes + sblk_bytes + stab_bytes, 0);
        if (sblk_bytes)
            std::memcpy(staging.data() + pat_bytes + tab_bytes, p->stride_blocks.data(), sblk_bytes);
        if (stab_bytes)
            std::memcpy(staging.data() + pat_bytes + tab_bytes + sblk_bytes, p->stride_table.data(),
                        stab_bytes);
        std::memcpy(staging.data(), pattern, m);
        if (tab_bytes) std::memcpy(staging.data() + pat_bytes, p->table.data(), tab_bytes);
        e = hipMalloc(&p->d_pattern, staging.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_pattern, staging.data(), staging.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            epsm_status st = hip_fail(e, "plan device copy");
            epsm_plan_destroy(p);
            return st;
        }
        d.pattern = p->d_pattern;
        d.table = tab_bytes ? (const uint16_t *)(p->d_pattern + pat_bytes) : nullptr;
        d.stride_blocks = sblk_bytes ? (const uint2 *)(p->d_pattern + pat_bytes + tab_bytes) : nullptr;
        d.stride_table =
            stab_bytes ? (const uint16_t *)(p->d_pattern + pat_bytes + tab_bytes + sblk_bytes) : nullptr;
    }
    *out = p;
    return EPSM_OK;
}

void epsm_plan_destroy(epsm_plan_t plan) {
    if (!plan) return;
    if (plan->d_pattern) (void)hipFree(plan->d_pattern);
    delete plan;
}

epsm_status epsm_plan_get_info(epsm_plan_t plan, epsm_plan_info *info) {
    if (!plan || !info) return fail(EPSM_EINVAL, "NULL argument");
    const DevPlan &d = plan->dev;
    info->m = d.m;
    info->variant = d.variant;
    info->flags = plan->flags;
    info->hash_bits = d.hash_bits;
    info->prefix_words = d.nw;
    for (int j = 0; j < 8; ++j) {
        info->words[j] = d.pw[j];
        info->masks[j] = d.pmask[j];
    }
    info->table = plan->table.empty() ? nullptr : plan->table.data();
    info->device = plan->device;
    info->kernel_class = kernel_class(d);
    info->stride = d.stride;
    info->prefix_bytes = d.variant == EPSM_VARIANT_DIRECT ? d.pk : 0;
    info->run_blocks = d.nl;
    info->table_row = plan->table_row;
    return EPSM_OK;
}

epsm_status epsm_search(epsm_plan_t plan, const uint8_t *d_text, uint64_t n, int64_t *d_out,
                        uint64_t out_capacity, uint64_t *d_n_hits, void *stream) {
    g_last_error.clear();
    return run_search(plan, d_text, n, d_out, out_capacity, d_n_hits, (hipStream_t)stream, true);
}

epsm_status epsm_count(epsm_plan_t plan, const uint8_t *d_text, uint64_t n, uint64_t *d_n_hits,
                       void *stream) {
    g_last_error.clear();
    return run_search(plan, d_text, n, nullptr, 0, d_n_hits, (hipStream_t)stream, false);
}

epsm_status epsm_search_noalloc(epsm_plan_t plan, const uint8_t *d_text, uint64_t n, int64_t *d_out,
                                uint64_t out_capacity, uint64_t *d_n_hits, void *stream) {
    g_last_error.clear();
    uint8_t *base = nullptr;
    epsm_status st = static_scratch(true, &base);
    if (st != EPSM_OK) return st;
    FixedScratch fx;
    fx.fault = (uint32_t *)base;
    fx.ws = base + kStaticFaultBytes;
    fx.bytes = EPSM_NOALLOC_SCRATCH_BYTES - kStaticFaultBytes;
    return run_search(plan, d_text, n, d_out, out_capacity, d_n_hits, (hipStream_t)stream, true,
                      false, &fx);
}

epsm_status epsm_search_dna(epsm_plan_t plan, const uint8_t *d_packed, uint64_t n, int64_t *d_out,
                            uint64_t out_capacity, uint64_t *d_n_hits, void *stream) {
    g_last_error.clear();
    return run_search(plan, d_packed, n, d_out, out_capacity, d_n_hits, (hipStream_t)stream, true,
                      true);
}

epsm_status epsm_count_dna(epsm_plan_t plan, const uint8_t *d_packed, uint64_t n,
                           uint64_t *d_n_hits, void *stream) {
    g_last_error.clear();
    return run_search(plan, d_packed, n, nullptr, 0, d_n_hits, (hipStream_t)stream, false, true);
}

epsm_status epsm_pack_dna(const uint8_t *d_codes, uint64_t n, uint8_t *d_packed, void *stream) {
    g_last_error.clear();
    if (n && (!d_codes || !d_packed)) return fail(EPSM_EINVAL, "NULL buffer");
    hipError_t e = launch_pack_dna(d_codes, n, d_packed, (hipStream_t)stream);
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "launch(pack_dna)");
}


epsm_status epsm_search_batch(const epsm_batch *batch, void *stream) {
    g_last_error.clear();
    HostBatch hb;
    epsm_status st = build_batch(batch, g_batch_waves, hb, true);
    if (st != EPSM_OK) return st;
    const BatchLayout L(hb);
    uint8_t *ws = nullptr;
    st = workspace_for((hipStream_t)stream, L.total, &ws);
    if (st != EPSM_OK) return st;
    st = upload_batch(hb, L, ws, (hipStream_t)stream, false);
    if (st != EPSM_OK) return st;
    const epsm_batch_outputs o{batch->d_out, batch->out_capacity, batch->d_counts, batch->d_offsets,
                               batch->d_total, !(batch->flags & EPSM_BATCH_COUNT_ONLY)};
    return run_batch(batch_ptrs(ws, L), hb, o, (hipStream_t)stream);
}

epsm_status epsm_batch_prepare(const epsm_batch *batch, epsm_batch_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(EPSM_EINVAL, "out is NULL");
    *out = nullptr;
    epsm_batch_plan_s *bp = new (std::nothrow) epsm_batch_plan_s();
    if (!bp) return fail(EPSM_ENOMEM, "batch plan allocation");
    epsm_status st = build_batch(batch, g_batch_waves, bp->hb, true);
    if (st != EPSM_OK) {
        delete bp;
        return st;
    }
    const BatchLayout L(bp->hb);
    hipError_t e = hipGetDevice(&bp->device);
    if (e == hipSuccess) e = hipMalloc(&bp->mem, std::max<size_t>(L.total, 256));
    if (e != hipSuccess) {
        bp->mem = nullptr;
        epsm_batch_destroy(bp);
        return hip_fail(e, "batch plan device memory");
    }
    st = upload_batch(bp->hb, L, bp->mem, nullptr, true);
    if (st != EPSM_OK) {
        epsm_batch_destroy(bp);
        return st;
    }
    bp->ptrs = batch_ptrs(bp->mem, L);
    bp->out = {batch->d_out, batch->out_capacity, batch->d_counts, batch->d_offsets, batch->d_total,
               !(batch->flags & EPSM_BATCH_COUNT_ONLY)};
    // descriptors stay on the device; the host copies are no longer needed
    bp->hb.texts.clear();
    bp->hb.texts.shrink_to_fit();
    bp->hb.korder = std::vector<uint32_t>();
    bp->hb.blob.clear();
    bp->hb.blob.shrink_to_fit();
    bp->hb.group_tables = std::vector<uint32_t>();
    bp->hb.units.shrink_to_fit();
    *out = bp;
    return EPSM_OK;
}

epsm_status epsm_batch_launch(epsm_batch_plan_t bp, void *stream) {
    g_last_error.clear();
    if (!bp) return fail(EPSM_EINVAL, "batch plan is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != bp->device) return fail(EPSM_EINVAL, "batch plan belongs to another device");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return run_batch(bp->ptrs, bp->hb, bp->out, s);  // the null stream cannot be captured
    std::lock_guard<std::mutex> lock(bp->mutex);
    auto it = bp->graphs.find(s);
    if (it == bp->graphs.end()) {
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        epsm_status st = run_batch(bp->ptrs, bp->hb, bp->out, s);
        e = hipStreamEndCapture(s, &g);
        if (st != EPSM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = bp->graphs.emplace(s, ge).first;
    }
    e = hipGraphLaunch(it->second, s);
    return e == hipSuccess ? EPSM_OK : hip_fail(e, "hipGraphLaunch");
}

void epsm_batch_destroy(epsm_batch_plan_t bp) {
    if (!bp) return;
    for (auto &kv : bp->graphs) (void)hipGraphExecDestroy(kv.second);
    if (bp->mem) (void)hipFree(bp->mem);
    delete bp;
}

epsm_status epsm_batch_get_info(epsm_batch_plan_t bp, uint64_t *units, uint64_t *entries,
                                uint32_t *tile_bytes) {
    if (!bp) return fail(EPSM_EINVAL, "batch plan is NULL");
    if (units) *units = bp->hb.units.size();
    if (entries) *entries = bp->hb.entries;
    if (tile_bytes) *tile_bytes = (uint32_t)(bp->hb.waves * kWavePiece);
    return EPSM_OK;
}

epsm_status epsm_set_batch_config(uint32_t waves) {
    g_last_error.clear();
    if (!batch_waves_supported((int)waves)) return fail(EPSM_EUNSUPPORTED, "batch tile not built");
    g_batch_waves = (int)waves;
    return EPSM_OK;
}

epsm_status epsm_set_tile_config(uint32_t waves, uint32_t pieces) {
    g_last_error.clear();
    TileConfig c{(int)waves, (int)pieces};
    if (!tile_config_supported(c)) return fail(EPSM_EUNSUPPORTED, "tile configuration not built");
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tile = c;
    return EPSM_OK;
}

uint32_t epsm_tile_configs(uint32_t *waves, uint32_t *pieces, uint32_t capacity) {
    TileConfig cfg[16];
    const int n = std::min(built_tile_configs(cfg, 16), 16);
    for (int i = 0; i < n && (uint32_t)i < capacity; ++i) {
        if (waves) waves[i] = (uint32_t)cfg[i].waves;
        if (pieces) pieces[i] = (uint32_t)cfg[i].pieces;
    }
    return (uint32_t)n;
}

epsm_status epsm_set_tune_table(const epsm_tune_entry *entries, uint32_t count) {
    g_last_error.clear();
    if (count && !entries) return fail(EPSM_EINVAL, "entries is NULL");
    if (count > kMaxTuneEntries) return fail(EPSM_EINVAL, "too many tune entries");
    for (uint32_t i = 0; i < count; ++i) {
        const epsm_tune_entry &e = entries[i];
        if (e.kernel_class >= EPSM_N_CLASSES) return fail(EPSM_EINVAL, "unknown kernel class");
        if (e.count_only > 1) return fail(EPSM_EINVAL, "count_only must be 0 or 1");
        if (e.strategy > EPSM_WRITE_TWO_PHASE) return fail(EPSM_EINVAL, "unknown write strategy");
        if (!tile_config_supported({(int)e.waves, (int)e.pieces}))
            return fail(EPSM_EUNSUPPORTED, "tile configuration not built");
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune.assign(entries, entries + count);
    return EPSM_OK;
}

epsm_status epsm_set_variant_table(const epsm_variant_entry *entries, uint32_t count) {
    g_last_error.clear();
    if (count > kMaxVariantEntries) return fail(EPSM_EINVAL, "at most 256 variant rows");
    if (count && !entries) return fail(EPSM_EINVAL, "entries is NULL");
    std::vector<epsm_variant_entry> rows(entries, entries + count);
    for (uint32_t i = 0; i < count; ++i) {
        const epsm_variant_entry &e = rows[i];
        const std::string at = "variant row " + std::to_string(i) + ": ";
        if (e.m_min == 0 || e.m_min > e.m_max) return fail(EPSM_EINVAL, at + "empty or zero m range");
        if (e.sigma_min > e.sigma_max || e.sigma_max > 256) return fail(EPSM_EINVAL, at + "bad sigma range");
        if (e.variant != EPSM_VARIANT_DIRECT && e.variant != EPSM_VARIANT_FINGERPRINT &&
            e.variant != EPSM_VARIANT_STRIDE)
            return fail(EPSM_EINVAL, at + "variant must be direct, fingerprint or strided");
        if (e.variant == EPSM_VARIANT_FINGERPRINT && e.m_min < 15)
            return fail(EPSM_EINVAL, at + "the fingerprint filter needs m >= 15");
        if (e.variant == EPSM_VARIANT_STRIDE && e.m_min < kStrideMinRow + 7)
            return fail(EPSM_EINVAL, at + "the strided filter needs m >= " + std::to_string(kStrideMinRow + 7));
        if (e.flags & ~kVariantRowFlags) return fail(EPSM_EINVAL, at + "unknown flags");
        const uint32_t k = (e.flags >> 8) & 0xF;
        if (k && (k < 8 || k > 14)) return fail(EPSM_EINVAL, at + "hash bits must be in [8, 14]");
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_variants.swap(rows);
    return EPSM_OK;
}

epsm_status epsm_estimate_alphabet(const uint8_t *d_text, uint64_t n, uint32_t *sigma, void *stream) {
    g_last_error.clear();
    if (!sigma) return fail(EPSM_EINVAL, "sigma is NULL");
    if (n > 0 && !d_text) return fail(EPSM_EINVAL, "d_text is NULL");
    *sigma = 0;
    if (n == 0) return EPSM_OK;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = nullptr;
    epsm_status st = workspace_for(s, 256, &ws);
    if (st != EPSM_OK) return st;
    hipError_t e = launch_alphabet(d_text, (uint32_t)std::min<uint64_t>(n, kAlphabetSample), (uint32_t *)ws, s);
    if (e != hipSuccess) return hip_fail(e, "launch(alphabet)");
    uint32_t v = 0;
    e = hipMemcpyAsync(&v, ws, sizeof(v), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(alphabet)");
    *sigma = v;
    return EPSM_OK;
}

epsm_status epsm_set_default_hash_bits(uint32_t k) {
    g_last_error.clear();
    if (k == 0) k = kDefaultHashBits;
    if (k < 8 || k > 14) return fail(EPSM_EINVAL, "hash bits must be in [8, 14]");
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_default_hash_bits = k;
    return EPSM_OK;
}

epsm_status epsm_reserve(void *stream, uint64_t max_n, uint64_t batch_bytes) {
    g_last_error.clear();
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return fail(EPSM_EUNSUPPORTED, "epsm_reserve on a stream that is being captured");
    // the largest workspace any built tile and write strategy needs for max_n
    TileConfig cfg[16];
    const int nc = std::min(built_tile_configs(cfg, 16), 16);
    size_t need = batch_bytes;
    for (int i = 0; i < nc; ++i) {
        const uint64_t tiles = max_n / (uint64_t)cfg[i].bytes() + 2;
        need = std::max(need, search_workspace(tiles, cfg[i], kWriteLookBack).total);
        need = std::max(need, search_workspace(tiles, cfg[i], kWriteTwoPhase).total);
    }
    // packed DNA texts of max_n symbols through the wide-lane kernel
    const uint64_t wtiles = max_n / dna_wide_tile_symbols() + 2;
    need = std::max<size_t>(need, wtiles * (4 + 8 + dna_wide_waves() * (4 + 4 * dna_wide_slot())) + 1024);
    // strided long-pattern filter: counts, offsets and scan block sums per tile
    const uint64_t stiles = max_n / (kStrideMinRow * kStrideBlocksPerTile) + 2;
    need = std::max<size_t>(need, stiles * 12 + (stiles / kScanBlock + 2) * 8 + 1024);
    uint8_t *ws = nullptr;
    epsm_status st = workspace_for(s, need, &ws);
    if (st != EPSM_OK) return st;
    uint32_t *f = nullptr;
    st = fault_word(s, true, &f);
    if (st != EPSM_OK || batch_bytes == 0) return st;
    // one free staging block for a batch call captured later on any stream
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    StagingBlock *blk = nullptr;
    st = staging_acquire(batch_bytes, dev, false, &blk);
    if (st != EPSM_OK) return st;
    std::lock_guard<std::mutex> lock(g_staging_mutex);
    blk->filling = false;
    blk->in_use = false;
    return EPSM_OK;
}

epsm_status epsm_batch_workspace(const epsm_batch *batch, uint64_t *bytes) {
    g_last_error.clear();
    if (!bytes) return fail(EPSM_EINVAL, "bytes is NULL");
    HostBatch hb;
    epsm_status st = build_batch(batch, g_batch_waves, hb, false);
    if (st != EPSM_OK) return st;
    *bytes = BatchLayout(hb).total;
    return EPSM_OK;
}

void epsm_release(void) {
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lock(g_ws_mutex);
        for (auto &kv : g_ws)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        g_ws.clear();
        for (auto &kv : g_fault)
            if (kv.second) (void)hipFree(kv.second);
        g_fault.clear();
    }
    std::lock_guard<std::mutex> lock(g_staging_mutex);
    for (StagingBlock *b : g_staging) {
        (void)hipEventDestroy(b->done);
        (void)hipHostFree(b->host);
        delete b;
    }
    g_staging.clear();
}

void epsm_debug_force_giveup(int enable) { g_debug_giveup.store(enable != 0); }

epsm_status epsm_stream_check(void *stream) {
    g_last_error.clear();
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // the stream's own fault word, then the device's static one (waits of
    // epsm_search_noalloc calls on any stream of this device)
    uint32_t *words[2] = {nullptr, nullptr};
    epsm_status st = fault_word(s, false, &words[0]);
    if (st != EPSM_OK) return st;
    uint8_t *base = nullptr;
    st = static_scratch(false, &base);
    if (st != EPSM_OK) return st;
    words[1] = (uint32_t *)base;
    for (uint32_t *f : words) {
        if (!f) continue;  // no waiting kernel ever used this word
        uint32_t v = 0;
        e = hipMemcpy(&v, f, sizeof(v), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(fault word)");
        if (!v) continue;
        const uint32_t zero = 0;  // report each give-up once
        e = hipMemcpy(f, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(fault word)");
        return fail(EPSM_EDEVICE, f == words[0]
                                      ? "a kernel on this stream gave up a bounded wait: its output is not trustworthy"
                                      : "an epsm_search_noalloc kernel on this device gave up a bounded wait: "
                                        "its output is not trustworthy");
    }
    return EPSM_OK;
}

const char *epsm_last_error(void) { return g_last_error.c_str(); }

const char *epsm_status_string(epsm_status s) {
    switch (s) {
        case EPSM_OK: return "EPSM_OK";
        case EPSM_EINVAL: return "EPSM_EINVAL";
        case EPSM_ENOMEM: return "EPSM_ENOMEM";
        case EPSM_EDEVICE: return "EPSM_EDEVICE";
        case EPSM_EUNSUPPORTED: return "EPSM_EUNSUPPORTED";
    }
    return "EPSM_UNKNOWN";
}

int epsm_version(void) { return 110; }

}  // extern "C"

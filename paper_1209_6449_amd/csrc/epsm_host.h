// Host-side internals of the library shared by its translation units (the
// C ABI in epsm_api.hip and the serving engine in epsm_serve.hip).
#pragma once

#include <map>
#include <string>
#include <vector>

#include "../../include/epsm.h"
#include "epsm_internal.h"

struct epsm_plan_s {
    std::vector<uint8_t> pattern;
    std::vector<uint16_t> table;  // host copy, fingerprint only
    std::vector<uint16_t> stride_table;  // strided filter: bucket starts, then offsets
    std::vector<uint32_t> stride_blocks; // strided filter: pattern blocks (lo, hi) per offset
    epsm::DevPlan dev{};          // pointers filled for device plans
    uint32_t flags = 0;
    uint32_t table_row = 0;       // 1 + the variant-table row that chose the variant, or 0
    int device = -1;
    uint8_t *d_pattern = nullptr;  // device block: pattern, then table
};

// Where a batch writes its results.
struct epsm_batch_outputs {
    int64_t *d_out;
    uint64_t cap;
    uint64_t *d_counts;
    uint64_t *d_offsets;
    uint64_t *d_total;
    bool write;
};


namespace epsm {
namespace host {

epsm_status fail(epsm_status s, const std::string &msg);
epsm_status hip_fail(hipError_t e, const char *what);
epsm_status check_plan(epsm_plan_t plan);

struct HostBatch {
    std::vector<BatchTextDesc> texts;
    std::vector<BatchPairDesc> pairs;      // the caller's order
    // kernel order (indices into pairs, pairs with entries only): per text,
    // its pairs filtered alone, then its grouped pairs, kGroupMax a group
    std::vector<uint32_t> korder;
    std::vector<uint32_t> group_tables;    // kGroupTableWords per group (masks, then bitmap)
    std::vector<BatchUnit> units;
    // device data of host-only plans (fingerprint tables, long patterns),
    // uploaded with the descriptors; per pair the blob offsets (or kNoBlob)
    std::vector<uint8_t> blob;
    std::vector<uint64_t> blob_table, blob_pattern;
    uint64_t entries = 0;
    int waves = 8;
};
constexpr uint64_t kNoBlob = ~uint64_t(0);

// Byte layout of the device copy of a batch: descriptors, then the
// (pair, tile) counts, their offsets, the scan's block sums, the parked
// group hits and the per-pair shifts and block sums of the pair scan (the
// device-only part, not uploaded).
struct BatchLayout {
    size_t blob, texts, kpairs, spans, gtables, units, park, parkn, ptc, pto, bsum, shift, pbsum, total;
    explicit BatchLayout(const HostBatch &hb) {
        auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
        size_t at = 0;
        blob = at; at += up(hb.blob.size());
        texts = at; at += up(hb.texts.size() * sizeof(BatchTextDesc));
        kpairs = at; at += up(hb.korder.size() * sizeof(BatchPairDesc));
        spans = at; at += up(hb.pairs.size() * sizeof(BatchSpan));
        gtables = at; at += up(hb.group_tables.size() * sizeof(uint32_t));
        units = at; at += up(hb.units.size() * sizeof(BatchUnit));
        ptc = at; at += up(hb.entries * sizeof(uint32_t));
        pto = at; at += up((hb.entries + 1) * sizeof(uint64_t));
        bsum = at; at += up(((hb.entries + kScanBlock - 1) / kScanBlock + 1) * sizeof(uint64_t));
        park = at; at += up(hb.units.size() * kParkMax * sizeof(uint32_t));
        parkn = at; at += up(hb.units.size() * sizeof(uint32_t));
        shift = at; at += up(hb.korder.size() * sizeof(int64_t));
        pbsum = at; at += up(((hb.pairs.size() + kScanBlock - 1) / kScanBlock + 1) * sizeof(uint64_t));
        total = at;
    }
};

struct BatchPtrs {
    BatchTextDesc *texts;
    BatchPairDesc *kpairs;
    BatchSpan *spans;
    uint32_t *gtables;
    BatchUnit *units;
    uint32_t *park;
    uint32_t *parkn;
    uint32_t *ptc;
    uint64_t *pto;
    uint64_t *bsum;
    int64_t *shift;
    uint64_t *pbsum;
};

BatchPtrs batch_ptrs(uint8_t *base, const BatchLayout &L);
// Validate a batch and build its work descriptors (check_outputs: require
// the output pointers of the epsm_batch).  group: gather the patterns of a
// text into multi-pattern groups for the count pass.
epsm_status build_batch(const epsm_batch *b, int waves, HostBatch &hb, bool check_outputs,
                        bool group = true);
// Copy descriptors (and host-only plan data) to `dev` in stream order, from a
// pinned staging block of the library (the host vectors may be released when
// it returns); sync: also wait for the copy.
epsm_status upload_batch(HostBatch &hb, const BatchLayout &L, uint8_t *dev, hipStream_t s, bool sync);
epsm_status run_batch_count(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                            hipStream_t s);
epsm_status run_batch_write(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                            hipStream_t s);
epsm_status run_batch(const BatchPtrs &P, const HostBatch &hb, const epsm_batch_outputs &o,
                      hipStream_t s);
int batch_waves();

}  // namespace host
}  // namespace epsm

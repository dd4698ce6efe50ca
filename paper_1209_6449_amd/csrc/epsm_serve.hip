// Serving engine: continuous batching of pattern queries over texts that stay
// resident in HBM.
//
// Clients submit queries (a resident text id and a set of patterns) from any
// thread.  A scheduler thread keeps up to `slots` micro-batches in flight, one
// per HIP stream, so work that arrives while others run is admitted as soon as
// a slot and device memory are free and overlaps with them on the device.  A
// micro-batch is a batched search (epsm_batch) over all patterns of the
// queries it took, in two stages: the count stage (count pass, scan, counts to
// pinned host memory), then -- once the output size is known and admitted
// against the HBM budget -- the write stage (write pass, positions to pinned
// host memory).  Admission never fails a query: work waits for memory, and a
// micro-batch larger than the whole budget runs when nothing else holds
// device memory.  Results are bit-identical to searching each pattern alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "epsm_host.h"

using namespace epsm;
using namespace epsm::host;

namespace {

struct Query {
    uint64_t id = 0;
    uint32_t text = 0;
    std::vector<epsm_plan_t> plans;  // host-only plans, owned
    uint64_t entries = 0;             // (pattern, tile) entries: work estimate
    uint64_t est_bytes = 0;           // device work estimate for admission
    double submit = 0, start = 0, done = 0;
    int32_t status = EPSM_OK;
    uint32_t batch_queries = 0;
    bool polled = false;              // handed out by epsm_server_poll
    std::vector<uint64_t> counts, offsets;
    std::vector<int64_t> positions;
    uint64_t total = 0;
    epsm_query_result view{};
    ~Query() {
        for (epsm_plan_t p : plans) epsm_plan_destroy(p);
    }
};

struct Text {
    const uint8_t *ptr;
    uint64_t n;
};

enum class SlotState { Idle, Counting, WaitMem, Writing };

template <typename T>
struct Pinned {  // growable pinned host buffer
    T *ptr = nullptr;
    size_t cap = 0;
    hipError_t reserve(size_t n) {
        if (n <= cap) return hipSuccess;
        size_t want = std::max<size_t>(n, 2 * cap);
        want = std::max<size_t>(want, 1024);
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc((void **)&ptr, want * sizeof(T), hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        else ptr = nullptr;
        return e;
    }
    ~Pinned() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    SlotState state = SlotState::Idle;
    std::vector<Query *> queries;
    std::vector<uint32_t> first_pair;  // per query, its first pair index
    HostBatch hb;
    std::unique_ptr<BatchLayout> layout;
    uint8_t *d_work = nullptr;
    uint64_t *d_meta = nullptr;  // [counts n_pairs][offsets n_pairs][total]
    int64_t *d_out = nullptr;
    uint64_t work_bytes = 0, out_bytes = 0;
    uint64_t total = 0;
    Pinned<uint64_t> h_meta;
    Pinned<int64_t> h_pos;
};

}  // namespace

struct epsm_server_s {
    epsm_server_config cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;  // scheduler wake-up
    std::condition_variable cv_done;  // poll wake-up
    std::vector<Text> texts;
    std::deque<Query *> pending;
    std::deque<Query *> completed;
    std::unordered_map<uint64_t, std::unique_ptr<Query>> queries;
    std::vector<Slot> slots;
    uint64_t next_id = 1;
    uint64_t reserved = 0, peak = 0;  // device bytes held by micro-batches
    uint64_t submitted = 0, done = 0, batches = 0;
    bool stop = false;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    uint64_t tile_bytes() const { return (uint64_t)batch_waves() * kWavePiece; }
    uint64_t text_tiles(uint32_t t) const {
        const uint64_t n = texts[t].n, delta = (uintptr_t)texts[t].ptr & 15;
        return n ? (delta + n + tile_bytes() - 1) / tile_bytes() : 0;
    }
    bool writing_slots() const {
        for (const Slot &s : slots)
            if (s.state == SlotState::Writing) return true;
        return false;
    }
    void reserve(uint64_t b) {
        reserved += b;
        peak = std::max(peak, reserved);
    }

    void fail_batch(Slot &s, int32_t status);
    void start_batch(Slot &s, std::unique_lock<std::mutex> &lk);
    void counted(Slot &s);
    void start_write(Slot &s);
    void finished(Slot &s);
    void run();
};

// Complete every query of a micro-batch with an error status.
void epsm_server_s::fail_batch(Slot &s, int32_t status) {
    const double t = now();
    for (Query *q : s.queries) {
        q->status = status;
        q->done = t;
        completed.push_back(q);
        ++done;
    }
    if (s.d_out) (void)hipFreeAsync(s.d_out, s.stream);
    if (s.d_work) (void)hipFreeAsync(s.d_work, s.stream);
    s.d_out = nullptr;
    s.d_work = nullptr;
    reserved -= s.work_bytes + s.out_bytes;
    s.work_bytes = s.out_bytes = 0;
    s.queries.clear();
    s.state = SlotState::Idle;
    cv_done.notify_all();
}

// Form a micro-batch from the head of the queue and launch its count stage.
// Called with the lock held; the lock is released while descriptors upload.
void epsm_server_s::start_batch(Slot &s, std::unique_lock<std::mutex> &lk) {
    const uint64_t budget = cfg.hbm_budget;
    uint64_t est = 0, entries = 0;
    while (!pending.empty() && s.queries.size() < cfg.max_batch_queries) {
        Query *q = pending.front();
        const bool first = s.queries.empty();
        if (!first && entries + q->entries > cfg.max_batch_entries) break;
        // memory admission: fits the budget, or nothing else holds memory
        if (reserved + est + q->est_bytes > budget && !(first && reserved == 0)) break;
        est += q->est_bytes;
        entries += q->entries;
        s.queries.push_back(q);
        pending.pop_front();
    }
    if (s.queries.empty()) return;
    reserve(est);
    s.work_bytes = est;
    ++batches;
    const double t_start = now();
    for (Query *q : s.queries) {
        q->start = t_start;
        q->batch_queries = (uint32_t)s.queries.size();
    }
    // batch description: the distinct texts of the queries, then every pattern
    std::vector<epsm_text_ref> trefs;
    std::unordered_map<uint32_t, uint32_t> local;
    std::vector<epsm_pair_ref> prefs;
    s.first_pair.clear();
    for (Query *q : s.queries) {
        auto it = local.find(q->text);
        if (it == local.end()) {
            it = local.emplace(q->text, (uint32_t)trefs.size()).first;
            trefs.push_back({texts[q->text].ptr, texts[q->text].n});
        }
        s.first_pair.push_back((uint32_t)prefs.size());
        for (epsm_plan_t p : q->plans) prefs.push_back({it->second, p});
    }
    lk.unlock();
    epsm_batch b{};
    b.texts = trefs.data();
    b.n_texts = (uint32_t)trefs.size();
    b.pairs = prefs.data();
    b.n_pairs = (uint32_t)prefs.size();
    epsm_status st = build_batch(&b, batch_waves(), s.hb, false);
    hipError_t e = hipSuccess;
    if (st == EPSM_OK) {
        s.layout.reset(new BatchLayout(s.hb));
        const size_t meta = (2 * (size_t)b.n_pairs + 1) * sizeof(uint64_t);
        e = hipMallocAsync((void **)&s.d_work, s.layout->total + meta + 256, s.stream);
        if (e == hipSuccess) {
            s.d_meta = (uint64_t *)(s.d_work + ((s.layout->total + 255) & ~size_t(255)));
            e = s.h_meta.reserve(2 * (size_t)b.n_pairs + 1);
        }
        if (e == hipSuccess) st = upload_batch(s.hb, *s.layout, s.d_work, s.stream, false);
        else st = hip_fail(e, "serve: work buffer");
    }
    if (st == EPSM_OK) {
        const BatchPtrs P = batch_ptrs(s.d_work, *s.layout);
        const epsm_batch_outputs o{nullptr, 0, s.d_meta, s.d_meta + b.n_pairs,
                                   s.d_meta + 2 * (size_t)b.n_pairs, true};
        st = run_batch_count(P, s.hb, o, s.stream);
        if (st == EPSM_OK) {
            e = hipMemcpyAsync(s.h_meta.ptr, s.d_meta, (2 * (size_t)b.n_pairs + 1) * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.event, s.stream);
            if (e != hipSuccess) st = hip_fail(e, "serve: count stage");
        }
    }
    lk.lock();
    if (st != EPSM_OK) {
        fail_batch(s, st);
        return;
    }
    s.state = SlotState::Counting;
}

// Count stage done: sizes are known.
void epsm_server_s::counted(Slot &s) {
    const size_t n_pairs = s.hb.pairs.size();
    s.total = s.h_meta.ptr[2 * n_pairs];
    s.state = SlotState::WaitMem;
    start_write(s);
}

// Admit the output against the budget and launch the write stage.  On an
// error the micro-batch fails and fail_batch releases whatever device memory
// the slot still holds.
void epsm_server_s::start_write(Slot &s) {
    const uint64_t need = s.total * sizeof(int64_t);
    if (need && reserved + need > cfg.hbm_budget && writing_slots()) return;  // wait for memory
    reserve(need);
    s.out_bytes = need;
    hipError_t e = hipSuccess;
    if (s.total) {
        if (cfg.flags & EPSM_SERVER_FAIL_OUTPUT_ALLOC) e = hipErrorOutOfMemory;  // test hook
        else e = hipMallocAsync((void **)&s.d_out, need, s.stream);
        if (e != hipSuccess) s.d_out = nullptr;
        if (e == hipSuccess) e = s.h_pos.reserve(s.total);
        if (e == hipSuccess) {
            const BatchPtrs P = batch_ptrs(s.d_work, *s.layout);
            const epsm_batch_outputs o{s.d_out, s.total, s.d_meta, s.d_meta + s.hb.pairs.size(),
                                       s.d_meta + 2 * s.hb.pairs.size(), true};
            epsm_status st = run_batch_write(P, s.hb, o, s.stream);
            if (st != EPSM_OK) e = hipErrorLaunchFailure;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.h_pos.ptr, s.d_out, need, hipMemcpyDeviceToHost, s.stream);
    }
    if (e == hipSuccess && s.d_out) {
        e = hipFreeAsync(s.d_out, s.stream);
        if (e == hipSuccess) s.d_out = nullptr;
    }
    if (e == hipSuccess) {
        e = hipFreeAsync(s.d_work, s.stream);
        if (e == hipSuccess) s.d_work = nullptr;
    }
    if (e == hipSuccess) e = hipEventRecord(s.event, s.stream);
    if (e != hipSuccess) {
        fail_batch(s, e == hipErrorOutOfMemory ? EPSM_ENOMEM : EPSM_EDEVICE);
        return;
    }
    s.state = SlotState::Writing;
}

// Write stage done: hand the results to the queries.
void epsm_server_s::finished(Slot &s) {
    const size_t n_pairs = s.hb.pairs.size();
    const uint64_t *cnt = s.h_meta.ptr, *off = s.h_meta.ptr + n_pairs;
    const double t = now();
    for (size_t i = 0; i < s.queries.size(); ++i) {
        Query *q = s.queries[i];
        const uint32_t p0 = s.first_pair[i];
        const size_t np = q->plans.size();
        q->counts.assign(cnt + p0, cnt + p0 + np);
        q->total = 0;
        for (uint64_t c : q->counts) q->total += c;
        q->offsets.resize(np);
        const uint64_t base = np ? off[p0] : 0;
        for (size_t k = 0; k < np; ++k) q->offsets[k] = off[p0 + k] - base;
        // a query's pairs are consecutive, so its positions are one run
        q->positions.assign(s.h_pos.ptr + base, s.h_pos.ptr + base + q->total);
        q->done = t;
        q->status = EPSM_OK;
        completed.push_back(q);
        ++done;
    }
    reserved -= s.work_bytes + s.out_bytes;
    s.work_bytes = s.out_bytes = 0;
    s.queries.clear();
    s.state = SlotState::Idle;
    cv_done.notify_all();
}

void epsm_server_s::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        bool progress = false;
        for (Slot &s : slots) {
            if (s.state == SlotState::Counting || s.state == SlotState::Writing) {
                const hipError_t q = hipEventQuery(s.event);
                if (q == hipErrorNotReady) continue;
                progress = true;
                if (q != hipSuccess) fail_batch(s, EPSM_EDEVICE);
                else if (s.state == SlotState::Counting) counted(s);
                else finished(s);
            } else if (s.state == SlotState::WaitMem) {
                start_write(s);
                if (s.state != SlotState::WaitMem) progress = true;
            }
        }
        for (Slot &s : slots) {
            if (s.state == SlotState::Idle && !pending.empty()) {
                start_batch(s, lk);
                if (s.state != SlotState::Idle) progress = true;
            }
        }
        if (!progress) {
            bool busy = false;
            for (const Slot &s : slots) busy |= s.state != SlotState::Idle;
            // poll in-flight events every 20 us; sleep until a submit otherwise
            if (busy) cv_work.wait_for(lk, std::chrono::microseconds(20));
            else cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
    // drain: wait for the device, then fail whatever is still queued
    lk.unlock();
    for (Slot &s : slots) (void)hipStreamSynchronize(s.stream);
    lk.lock();
    for (Slot &s : slots)
        if (s.state != SlotState::Idle) fail_batch(s, EPSM_EDEVICE);
    while (!pending.empty()) {
        Query *q = pending.front();
        pending.pop_front();
        q->status = EPSM_EDEVICE;
        q->done = now();
        completed.push_back(q);
        ++done;
    }
    cv_done.notify_all();
}

extern "C" {

epsm_status epsm_server_create(const epsm_server_config *cfg, epsm_server_t *out) {
    if (!out) return fail(EPSM_EINVAL, "out is NULL");
    *out = nullptr;
    epsm_server_s *s = new (std::nothrow) epsm_server_s();
    if (!s) return fail(EPSM_ENOMEM, "server allocation");
    if (cfg) s->cfg = *cfg;
    if (s->cfg.flags & ~EPSM_SERVER_FAIL_OUTPUT_ALLOC) {
        delete s;
        return fail(EPSM_EINVAL, "unknown server flags");
    }
    if (!s->cfg.slots) s->cfg.slots = 4;
    if (s->cfg.slots > 16) {
        delete s;
        return fail(EPSM_EINVAL, "at most 16 slots");
    }
    if (!s->cfg.max_batch_queries) s->cfg.max_batch_queries = 64;
    if (!s->cfg.max_batch_entries) s->cfg.max_batch_entries = 1ull << 25;
    if (!s->cfg.hbm_budget) s->cfg.hbm_budget = 16ull << 30;
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&s->device);
    s->slots.resize(s->cfg.slots);
    for (Slot &sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.event, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        epsm_status st = hip_fail(e, "server streams");
        epsm_server_destroy(s);
        return st;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return EPSM_OK;
}

epsm_status epsm_server_add_text(epsm_server_t s, const uint8_t *d_text, uint64_t n,
                                 uint32_t *text_id) {
    if (!s || !text_id) return fail(EPSM_EINVAL, "NULL argument");
    if (n && !d_text) return fail(EPSM_EINVAL, "d_text is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *text_id = (uint32_t)s->texts.size();
    s->texts.push_back({d_text, n});
    return EPSM_OK;
}

epsm_status epsm_server_submit(epsm_server_t s, uint32_t text_id, const uint8_t *patterns,
                               const uint64_t *lengths, uint32_t n_patterns, uint64_t *query_id) {
    if (!s || !query_id) return fail(EPSM_EINVAL, "NULL argument");
    if (n_patterns && (!patterns || !lengths)) return fail(EPSM_EINVAL, "patterns or lengths is NULL");
    std::unique_ptr<Query> q(new (std::nothrow) Query());
    if (!q) return fail(EPSM_ENOMEM, "query allocation");
    uint64_t at = 0;
    for (uint32_t k = 0; k < n_patterns; ++k) {
        epsm_plan_t p = nullptr;
        epsm_status st = epsm_plan(patterns + at, lengths[k], EPSM_PLAN_HOST_ONLY, &p);
        if (st != EPSM_OK) return st;
        q->plans.push_back(p);
        at += lengths[k];
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (text_id >= s->texts.size()) return fail(EPSM_EINVAL, "unknown text id");
    if (s->stop) return fail(EPSM_EINVAL, "server is shutting down");
    q->text = text_id;
    q->entries = (uint64_t)n_patterns * s->text_tiles(text_id);
    // device work: 12 bytes per (pattern, tile) entry, descriptors, tables,
    // and the parked hits of each tile of the text
    uint64_t table_bytes = 0;
    for (epsm_plan_t p : q->plans) table_bytes += p->table.size() * sizeof(uint16_t) + p->pattern.size();
    q->est_bytes = q->entries * 12 + (uint64_t)n_patterns * (sizeof(BatchPairDesc) + 64) +
                   table_bytes + s->text_tiles(text_id) * (kParkMax + 1) * sizeof(uint32_t) + (64u << 10);
    q->id = s->next_id++;
    q->submit = s->now();
    *query_id = q->id;
    s->pending.push_back(q.get());
    s->queries.emplace(q->id, std::move(q));
    ++s->submitted;
    s->cv_work.notify_one();
    return EPSM_OK;
}

epsm_status epsm_server_poll(epsm_server_t s, epsm_query_result *out, uint32_t max, uint32_t *n_out,
                             uint32_t wait_us) {
    if (!s || !n_out || (max && !out)) return fail(EPSM_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && wait_us)
        s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                            [s] { return !s->completed.empty(); });
    uint32_t n = 0;
    while (n < max && !s->completed.empty()) {
        Query *q = s->completed.front();
        s->completed.pop_front();
        epsm_query_result &r = q->view;
        r.query_id = q->id;
        r.text_id = q->text;
        r.n_patterns = (uint32_t)q->plans.size();
        r.status = q->status;
        r.batch_queries = q->batch_queries;
        r.total = q->total;
        r.counts = q->counts.data();
        r.offsets = q->offsets.data();
        r.positions = q->positions.data();
        r.submit_time = q->submit;
        r.start_time = q->start;
        r.done_time = q->done;
        q->polled = true;
        out[n++] = r;
    }
    *n_out = n;
    return EPSM_OK;
}

epsm_status epsm_server_release(epsm_server_t s, uint64_t query_id) {
    if (!s) return fail(EPSM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(query_id);
    if (it == s->queries.end()) return fail(EPSM_EINVAL, "unknown query id");
    // only a query already returned by epsm_server_poll: the completion queue
    // still points at one that has completed but not been polled
    if (!it->second->polled) return fail(EPSM_EINVAL, "query has not been returned by epsm_server_poll");
    s->queries.erase(it);
    return EPSM_OK;
}

double epsm_server_now(epsm_server_t s) { return s ? s->now() : 0.0; }

epsm_status epsm_server_get_stats(epsm_server_t s, epsm_server_stats *st) {
    if (!s || !st) return fail(EPSM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->completed = s->done;
    st->queued = s->pending.size();
    st->in_flight = s->submitted - s->done - s->pending.size();
    st->batches = s->batches;
    st->bytes_reserved = s->reserved;
    st->bytes_peak = s->peak;
    return EPSM_OK;
}

void epsm_server_destroy(epsm_server_t s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot &sl : s->slots) {
        if (sl.event) (void)hipEventDestroy(sl.event);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}

}  // extern "C"

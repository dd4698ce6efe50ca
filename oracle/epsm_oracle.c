/*
 * Brute-force oracle for exact string matching.  TEST INFRASTRUCTURE ONLY:
 * the test suite, the smoke check and the benchmark's CPU-baseline leg are the
 * only callers.  It shares no code, header or table with the GPU library.
 *
 * What it computes is the problem statement of the paper (Introduction and
 * Section 2, "Notions and Terminology"): for a text t[0..n-1] and a pattern
 * p[0..m-1] with m > 0, report every position s, 0 <= s <= n-m, such that
 * t[s+j] == p[j] for all 0 <= j < m.  Occurrences may overlap (all of them are
 * reported); positions are 0-based start indices, emitted in ascending order.
 * This is the same predicate the paper uses to define wsmatch (Section 3.1:
 * r_i = 1 iff a_{i+j} = b_j for j = 0..k-1).  Every EPSM variant finishes with
 * an exact "naive check", so the method's output is exactly this set.
 *
 * Plain loops, no SIMD intrinsics, no memmem/memcmp: a reader can check it
 * against the definition by eye.  Bytes are arbitrary values 0..255 (0 is an
 * ordinary symbol; the text is length-counted, never NUL terminated).
 *
 * Build: gcc -O2 -shared -fPIC -pthread -o liboracle.so epsm_oracle.c
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

/* 1 iff p occurs in t at s (caller guarantees s + m <= n). */
static int occurs_at(const uint8_t *t, uint64_t s, const uint8_t *p, uint64_t m)
{
    for (uint64_t j = 0; j < m; j++)
        if (t[s + j] != p[j])
            return 0;
    return 1;
}

/*
 * Occurrences whose start lies in [s_begin, s_end) (clamped to [0, n-m]).
 * Writes the first `cap` of them, in ascending order, to out (out may be NULL
 * when cap == 0) and returns how many there are in the range.
 */
uint64_t oracle_range(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m,
                      uint64_t s_begin, uint64_t s_end, int64_t *out, uint64_t cap)
{
    uint64_t count = 0;
    if (m == 0 || m > n)
        return 0;
    uint64_t last = n - m; /* largest valid start */
    if (s_end > last + 1)
        s_end = last + 1;
    for (uint64_t s = s_begin; s < s_end; s++) {
        if (occurs_at(t, s, p, m)) {
            if (count < cap)
                out[count] = (int64_t)s;
            count++;
        }
    }
    return count;
}

/* All occurrences: first `cap` positions to out, full count returned. */
uint64_t oracle_search(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m,
                       int64_t *out, uint64_t cap)
{
    return oracle_range(t, n, p, m, 0, n, out, cap);
}

uint64_t oracle_count(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m)
{
    return oracle_range(t, n, p, m, 0, n, NULL, 0);
}

/* ---- multi-threaded count: contiguous start ranges, one per thread ------ */

struct count_job {
    const uint8_t *t;
    uint64_t n;
    const uint8_t *p;
    uint64_t m;
    uint64_t s_begin, s_end;
    uint64_t result;
};

static void *count_worker(void *arg)
{
    struct count_job *job = (struct count_job *)arg;
    job->result = oracle_range(job->t, job->n, job->p, job->m, job->s_begin,
                               job->s_end, NULL, 0);
    return NULL;
}

/*
 * Same count as oracle_count, split over `threads` POSIX threads by
 * contiguous start-position ranges (a partition, so the per-range counts add
 * up to the total).  Returns (uint64_t)-1 if a thread cannot be created.
 */
uint64_t oracle_count_mt(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m,
                         int threads)
{
    if (m == 0 || m > n)
        return 0;
    if (threads < 1)
        threads = 1;
    uint64_t starts = n - m + 1;
    struct count_job *jobs = calloc((size_t)threads, sizeof(*jobs));
    pthread_t *tids = calloc((size_t)threads, sizeof(*tids));
    char *started = calloc((size_t)threads, 1);
    if (!jobs || !tids || !started) {
        free(jobs);
        free(tids);
        free(started);
        return (uint64_t)-1;
    }
    uint64_t failed = 0;
    for (int i = 0; i < threads; i++) {
        jobs[i].t = t;
        jobs[i].n = n;
        jobs[i].p = p;
        jobs[i].m = m;
        jobs[i].s_begin = starts * (uint64_t)i / (uint64_t)threads;
        jobs[i].s_end = starts * (uint64_t)(i + 1) / (uint64_t)threads;
        if (pthread_create(&tids[i], NULL, count_worker, &jobs[i]) == 0)
            started[i] = 1;
        else
            failed = 1;
    }
    uint64_t total = 0;
    for (int i = 0; i < threads; i++) {
        if (started[i]) {
            pthread_join(tids[i], NULL);
            total += jobs[i].result;
        }
    }
    free(jobs);
    free(tids);
    free(started);
    return failed ? (uint64_t)-1 : total;
}

/* ---- multi-threaded positions: contiguous start ranges, one per thread -- */

struct range_job {
    const uint8_t *t;
    uint64_t n;
    const uint8_t *p;
    uint64_t m;
    uint64_t s_begin, s_end;
    int64_t *out;       /* room for s_end - s_begin positions */
    uint64_t result;
};

static void *range_worker(void *arg)
{
    struct range_job *job = (struct range_job *)arg;
    job->result = oracle_range(job->t, job->n, job->p, job->m, job->s_begin, job->s_end,
                               job->out, job->s_end - job->s_begin);
    return NULL;
}

/*
 * The occurrences whose start lies in [s_begin, s_end), all of them, in
 * ascending order, found by `threads` POSIX threads over contiguous start
 * ranges.  out must hold s_end - s_begin entries (every start could match):
 * thread i writes the occurrences of its range at out + (its first start -
 * s_begin), then the ranges' results are moved down, in range order, to be
 * contiguous.  Returns the number of occurrences, or (uint64_t)-1 if a thread
 * cannot be created.
 */
uint64_t oracle_range_mt(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m,
                         uint64_t s_begin, uint64_t s_end, int64_t *out, int threads)
{
    if (m == 0 || m > n)
        return 0;
    if (s_end > n - m + 1)
        s_end = n - m + 1;
    if (s_begin >= s_end)
        return 0;
    if (threads < 1)
        threads = 1;
    uint64_t starts = s_end - s_begin;
    struct range_job *jobs = calloc((size_t)threads, sizeof(*jobs));
    pthread_t *tids = calloc((size_t)threads, sizeof(*tids));
    char *started = calloc((size_t)threads, 1);
    if (!jobs || !tids || !started) {
        free(jobs);
        free(tids);
        free(started);
        return (uint64_t)-1;
    }
    uint64_t failed = 0;
    for (int i = 0; i < threads; i++) {
        jobs[i].t = t;
        jobs[i].n = n;
        jobs[i].p = p;
        jobs[i].m = m;
        jobs[i].s_begin = s_begin + starts * (uint64_t)i / (uint64_t)threads;
        jobs[i].s_end = s_begin + starts * (uint64_t)(i + 1) / (uint64_t)threads;
        jobs[i].out = out + (jobs[i].s_begin - s_begin);
        if (pthread_create(&tids[i], NULL, range_worker, &jobs[i]) == 0)
            started[i] = 1;
        else
            failed = 1;
    }
    uint64_t total = 0;
    for (int i = 0; i < threads; i++) {
        if (!started[i])
            continue;
        pthread_join(tids[i], NULL);
        /* Range i's results start at or after where the previous ranges end,
         * so moving them down one element at a time never overwrites an
         * element not yet moved. */
        for (uint64_t k = 0; k < jobs[i].result; k++)
            out[total + k] = jobs[i].out[k];
        total += jobs[i].result;
    }
    free(jobs);
    free(tids);
    free(started);
    return failed ? (uint64_t)-1 : total;
}

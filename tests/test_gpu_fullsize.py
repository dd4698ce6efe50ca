"""Full-size parity: the benchmark configurations at their real shapes.

Every position the GPU writes is compared, element by element, with the CPU
oracle on the same seeded input; the oracle's answer is produced range by
range by its threaded form (contiguous start ranges, concatenated in order)
and compared with the matching slice of the GPU output, so no output is
ever held whole on the host twice.  The library runs in the launch
configuration the benchmark times: the packaged tune table of this device
(tiles, write strategies, fingerprint width, batch tile) is applied.

  * 1 GiB texts over 2, 4, 20, 64, 128 codes: all 16 patterns of each
    (positions and count modes)
  * 4 GiB Zipf text: the 16 cut patterns m = 1..16 (positions and count)
  * 4 GiB a^n with a^m, m = 1..16: the closed form (positions 0..n-m, count
    n-m+1), checked on the device
  * the 10,000-text batch at full shape: every pair of a seeded subset of
    500 texts plus the 8 longest (16 MiB), as one prepared batch launched
    twice from its captured graph
  * serving: the 256 resident texts (about 11 GiB) with a seeded sample of 10
    queries of the Poisson stream, submitted together
  * the expand kernel's multi-tile list copy (9 list tiles per workgroup):
    400 MiB sparse text at 64 KiB tiles, two-phase write
"""
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
CHUNK = 1 << 26  # starts per oracle range
NO_LIMIT = (1 << 64) - 1


def say(msg: str) -> None:
    print(msg, flush=True)


@pytest.fixture(scope="module")
def epsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as mod
    from paper_1209_6449_amd import autotune
    mod.lib()
    applied = autotune.apply_default()
    say(f"tune table: {applied}")
    yield mod
    mod.set_tune_table([])
    mod.set_default_hash_bits(0)
    mod.set_batch_config(8)


def host_copy(spec: W.TextSpec, t: torch.Tensor) -> np.ndarray:
    """Host copy of a GPU-generated text, spot-checked against the CPU generator."""
    text = t.cpu().numpy()
    for start in (0, spec.n // 3, max(0, spec.n - 4096)):
        length = min(4096, spec.n - start)
        assert np.array_equal(text[start:start + length], W.gen_numpy(spec, start, length))
    return text


def compare_positions(got: torch.Tensor, total: int, text: np.ndarray, pattern: bytes, label: str) -> int:
    """got[0:total] (device) must equal the oracle's occurrences of pattern in text."""
    n, m = text.size, len(pattern)
    k = 0
    for lo in range(0, max(n - m + 1, 0), CHUNK):
        exp = oracle.search_range_mt(text, pattern, lo, lo + CHUNK, THREADS)
        if exp.size:
            assert k + exp.size <= total, f"{label}: the GPU reports {total} positions, the oracle more"
            g = got[k:k + exp.size].cpu().numpy()
            if not np.array_equal(g, exp):
                bad = int(np.flatnonzero(g != exp)[0])
                raise AssertionError(f"{label}: entry {k + bad}: GPU {g[bad]}, oracle {exp[bad]}")
        k += exp.size
    assert k == total, f"{label}: GPU count {total}, oracle {k}"
    return k


def search_and_compare(epsm, t: torch.Tensor, text: np.ndarray, pattern: bytes, label: str,
                       out: torch.Tensor | None = None) -> int:
    plan = epsm.Plan(pattern)
    say(f"{label}: m={len(pattern)} variant={plan.info()['variant']}")
    cnt = epsm.count(t, plan)
    buf = out if out is not None and out.numel() >= cnt else torch.empty(max(cnt, 1), dtype=torch.int64,
                                                                         device="cuda")
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    epsm.search_into(plan, t, buf[:cnt], hits)
    epsm.stream_check()
    assert int(hits.item()) == cnt, f"{label}: count {cnt}, search {int(hits.item())}"
    return compare_positions(buf, cnt, text, pattern, label)


# ---- 1 GiB texts, five alphabets ----------------------------------------------


@pytest.mark.parametrize("sigma", W.CONFIG2_SIGMAS)
def test_config2_full(epsm, sigma):
    spec, cases = W.config2(sigma)
    say(f"config2 sigma={sigma}: generating {spec.n} bytes")
    t = W.gen_bytes(spec, device="cuda")
    text = host_copy(spec, t)
    out = None
    for c in cases:
        total = search_and_compare(epsm, t, text, c.pattern, f"config2 sigma={sigma} {c.origin}", out)
        if c.origin == "cut":
            assert total >= 1
    del t


# ---- 4 GiB Zipf text and 4 GiB a^n ------------------------------------------


@pytest.fixture(scope="module")
def zipf4g(epsm):
    spec, cases, _, _ = W.config3()
    say(f"config3: generating the {spec.n}-byte Zipf text")
    t = W.gen_bytes(spec, device="cuda")
    text = host_copy(spec, t)
    yield t, text, cases
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("ms", [(1, 8), (9, 16)], ids=["m1-8", "m9-16"])
def test_config3_zipf_full(epsm, zipf4g, ms):
    t, text, cases = zipf4g
    for c in cases:
        if ms[0] <= len(c.pattern) <= ms[1]:
            total = search_and_compare(epsm, t, text, c.pattern, "config3 zipf")
            assert total >= 1


def test_config3_periodic_closed_form(epsm):
    """a^n with a^m: exactly n-m+1 hits at 0..n-m (the closed form), on the device."""
    _, _, per, per_cases = W.config3()
    n = per.n
    t = torch.full((n,), per.fill, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    step = 1 << 28
    for c in per_cases:
        m = len(c.pattern)
        say(f"config3 a^n: m={m}")
        plan = epsm.Plan(c.pattern)
        assert epsm.count(t, plan) == n - m + 1
        out[-1] = -7
        epsm.search_into(plan, t, out[:n - m + 1], hits)
        epsm.stream_check()
        assert int(hits.item()) == n - m + 1
        for s in range(0, n - m + 1, step):
            e = min(s + step, n - m + 1)
            assert torch.equal(out[s:e], torch.arange(s, e, dtype=torch.int64, device="cuda")), (m, s)
        if m > 1:
            assert int(out[-1].item()) == -7  # nothing written past the capacity
    del t, out
    torch.cuda.empty_cache()


# ---- the batch at full shape ------------------------------------------------


def test_config4_subset_full_shape(epsm):
    bts = W.config4()
    g = W.rng(4, 77)
    idx = set(g.choice(len(bts), 500, replace=False).tolist())
    idx |= set(np.argsort([bt.spec.n for bt in bts])[-8:].tolist())
    idx = sorted(idx)
    say(f"config4 subset: {len(idx)} texts, {sum(bts[i].spec.n for i in idx)} bytes")
    texts = [W.gen_bytes(bts[i].spec, device="cuda") for i in idx]
    pairs = [(j, epsm.Plan(p, epsm.PLAN_HOST_ONLY)) for j, i in enumerate(idx) for p in bts[i].patterns]
    pats = [bts[i].patterns[k] for i in idx for k in range(len(bts[i].patterns))]
    b0 = epsm.Batch(texts, pairs, count_only=True)
    b0.run()
    total = int(b0.total.item())
    say(f"config4 subset: {len(pairs)} pairs, {total} positions")
    out = torch.full((max(total, 1),), -1, dtype=torch.int64, device="cuda")
    batch = epsm.Batch(texts, pairs, out=out[:total] if total else None)
    bp = epsm.BatchPlan(batch)
    stream = torch.cuda.current_stream()
    bp.launch(stream)  # captured on first use
    epsm.stream_check()
    first = out[:total].clone()
    out.fill_(-1)
    bp.launch(stream)  # a replay of the captured graph
    epsm.stream_check()
    assert torch.equal(out[:total], first)
    n = len(pairs)
    counts = batch.counts[:n].cpu().numpy()
    offsets = batch.offsets[:n].cpu().numpy()
    assert np.array_equal(counts, b0.counts[:n].cpu().numpy())
    got = first.cpu().numpy()
    hosts = [t.cpu().numpy() for t in texts]
    for j, i in enumerate(idx[:4]):
        assert np.array_equal(hosts[j][:256], W.gen_numpy(bts[i].spec, 0, min(256, bts[i].spec.n)))

    oracle.count(b"a", b"a")  # load the oracle before the worker threads use it

    def expected(k):
        ti = pairs[k][0]
        return oracle.search_range_mt(hosts[ti], pats[k], 0, hosts[ti].size, 1)

    say("config4 subset: oracle over every pair")
    with ThreadPoolExecutor(THREADS) as ex:
        for k, exp in enumerate(ex.map(expected, range(n), chunksize=64)):
            o, c = int(offsets[k]), int(counts[k])
            assert c == exp.size, (k, c, exp.size)
            assert np.array_equal(got[o:o + c], exp), k
    assert int(offsets[-1]) + int(counts[-1]) == total


# ---- serving over the full resident set --------------------------------------


def test_config5_sampled_queries_full_set(epsm):
    from paper_1209_6449_amd import serve
    specs = W.config5_texts()
    say(f"config5: generating {len(specs)} resident texts ({sum(s.n for s in specs)} bytes)")
    texts = [W.gen_bytes(sp, device="cuda") for sp in specs]
    torch.cuda.synchronize()
    qs = W.config5_queries(specs, 1000, qps=100.0)
    pick = sorted(W.rng(5, 77).choice(len(qs), 10, replace=False).tolist())
    srv = serve.Server(slots=4, max_batch_queries=32)
    try:
        for t in texts:
            srv.add_text(t)
        ids = {srv.submit(qs[i].text, qs[i].patterns): i for i in pick}
        results = {}
        deadline = time.time() + 120
        while len(results) < len(ids) and time.time() < deadline:
            for r in srv.poll(64, 20_000):
                results[r.query_id] = r
        assert len(results) == len(ids), "queries did not complete"
    finally:
        srv.close()
    hosts = {}
    for qid, i in sorted(ids.items(), key=lambda kv: kv[1]):
        q, r = qs[i], results[qid]
        assert r.status == 0
        if q.text not in hosts:
            hosts.clear()
            hosts[q.text] = host_copy(specs[q.text], texts[q.text])
        text = hosts[q.text]
        say(f"config5 query {i}: text {q.text} ({text.size} B), {len(q.patterns)} patterns, "
            f"micro-batch of {r.batch_queries}")
        for k, p in enumerate(q.patterns):
            exp = oracle.search_range_mt(text, p, 0, text.size, THREADS)
            assert np.array_equal(r.pattern_positions(k), exp), (i, k)


# ---- expand kernel: several list tiles per workgroup -------------------------


def test_expand_multi_tile_lists(epsm):
    """6400 tiles of 64 KiB: each expand workgroup copies the lists of 9 tiles."""
    spec = W.TextSpec(n=400 * (1 << 20), kind="uniform", key=W.text_key(92, 1), sigma=64)
    t = W.gen_bytes(spec, device="cuda")
    text = host_copy(spec, t)
    epsm.set_tune_table([(cls, 0, NO_LIMIT, 8, 8, epsm.WRITE_TWO_PHASE) for cls in (0, 1, 2)])
    try:
        for lo, m in ((1_234_567, 2), (77_000_000, 3), (300_000_001, 6), (5, 20)):
            search_and_compare(epsm, t, text, text[lo:lo + m].tobytes(), "expand lists")
    finally:
        from paper_1209_6449_amd import autotune
        epsm.set_tune_table([])
        autotune.apply_default()

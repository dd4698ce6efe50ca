"""Serving: continuous batching returns, for every query, exactly what the
query returns when run alone (and what the oracle returns)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as epsm
    from paper_1209_6449_amd import serve
    epsm.lib()
    specs = W.config5_texts(n_texts=12, min_len=1 << 16, max_len=1 << 22)
    texts = [W.gen_bytes(sp, device="cuda") for sp in specs]
    host = [t.cpu().numpy() for t in texts]
    queries = W.config5_queries(specs, n_queries=40, qps=400.0, max_patterns=48)
    return epsm, serve, texts, host, queries


def say(msg):
    print(msg, flush=True)


def check_against_oracle(outcome, query, host):
    for k, p in enumerate(query.patterns):
        exp = oracle.positions(host[query.text], p)
        assert np.array_equal(outcome.pattern_positions(k), exp), (query.text, k, p)


def test_mix_equals_alone_and_oracle(env):
    epsm, serve, texts, host, queries = env
    with serve.Server(slots=4, max_batch_queries=16) as srv:
        for t in texts:
            srv.add_text(t)
        say(f"mixed stream of {len(queries)} queries")
        # arrivals 20x faster than the recorded stream (8000 queries/s) so that
        # queries queue up behind each other and share micro-batches
        mixed, lat, wall = serve.run_queries(srv, queries, rate_scale=20.0)
        assert all(o.status == 0 for o in mixed)
        st = srv.stats()
        assert st["completed"] == len(queries)
        # queries were batched together (continuous batching, not one by one)
        assert max(o.batch_queries for o in mixed) > 1
        say("each query alone")
        for i, q in enumerate(queries):
            qid = srv.submit(q.text, q.patterns)
            got = []
            while not got:
                got = srv.poll(1, 100_000)
            alone = got[0]
            assert alone.query_id == qid and alone.status == 0 and alone.batch_queries == 1
            assert np.array_equal(alone.counts, mixed[i].counts), i
            assert np.array_equal(alone.offsets, mixed[i].offsets), i
            assert np.array_equal(alone.positions, mixed[i].positions), i
            if i % 4 == 0:
                check_against_oracle(alone, q, host)


def test_tiny_budget_queues_but_never_fails(env):
    epsm, serve, texts, host, queries = env
    with serve.Server(slots=3, max_batch_queries=8, hbm_budget=1 << 20) as srv:
        for t in texts:
            srv.add_text(t)
        say("tiny HBM budget")
        outs, lat, wall = serve.run_queries(srv, queries[:20], rate_scale=10.0)
        assert all(o.status == 0 for o in outs)
        for i in range(0, 20, 5):
            check_against_oracle(outs[i], queries[i], host)
        st = srv.stats()
        assert st["completed"] == 20 and st["bytes_reserved"] == 0


def test_burst_is_batched_and_overlapped(env):
    epsm, serve, texts, host, queries = env
    burst = [W.Query(0.0, q.text, q.patterns) for q in queries]
    with serve.Server(slots=4, max_batch_queries=8) as srv:
        for t in texts:
            srv.add_text(t)
        say("burst")
        outs, lat, wall = serve.run_queries(srv, burst)
        st = srv.stats()
        assert st["batches"] < len(burst)
        assert all(o.status == 0 for o in outs)
        # micro-batches overlap on the device: some batch started before
        # another one finished
        spans = sorted({(o.start_time, o.done_time) for o in outs})
        assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
        for i in range(0, len(burst), 7):
            check_against_oracle(outs[i], burst[i], host)


def test_empty_query_and_bad_text_id(env):
    epsm, serve, texts, host, queries = env
    with serve.Server(slots=1) as srv:
        srv.add_text(texts[0])
        qid = srv.submit(0, [])
        got = []
        while not got:
            got = srv.poll(1, 100_000)
        assert got[0].query_id == qid and got[0].status == 0 and got[0].positions.size == 0
        with pytest.raises(epsm.EpsmError):
            srv.submit(5, [b"ab"])
        with pytest.raises(epsm.EpsmError):
            srv.submit(0, [b""])  # m = 0


def test_release_only_after_poll(env):
    epsm, serve, texts, host, queries = env
    import time
    with serve.Server(slots=1) as srv:
        srv.add_text(texts[0])
        qid = srv.submit(0, [b"ab", b"abc"])
        L = epsm.lib()
        deadline = time.time() + 60
        while srv.stats()["completed"] < 1 and time.time() < deadline:
            time.sleep(0.001)
        # completed but not yet polled: its results are still queued
        assert L.epsm_server_release(srv._h, qid) != 0
        got = []
        while not got:
            got = srv.poll(1, 100_000)  # poll() releases what it returns
        assert got[0].query_id == qid and got[0].status == 0
        assert L.epsm_server_release(srv._h, qid) != 0  # already released

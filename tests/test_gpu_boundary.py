"""The boundary's stream contract on the GPU.

* epsm_search, epsm_count and epsm_search_batch captured into one graph on a
  fresh stream (after epsm_reserve) and replayed: every replay equals the
  oracle, with eager work and synchronisations between the replays.
* The Python helpers run on the stream they are given.
* A bounded wait that gives up surfaces as an error (forced from the host
  with the library's test hook; every kernel still exits normally).
* A serving write stage whose output allocation fails completes its queries
  with EPSM_ENOMEM and releases the memory it was admitted for.
* A failed runtime call elsewhere on the thread (its error left for
  hipGetLastError) does not make the library's next launches fail.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TILE = 128 * 1024


@pytest.fixture(scope="module")
def epsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as mod
    mod.lib()
    return mod


def say(msg: str) -> None:
    print(msg, flush=True)


def uniform_text(n, sigma, seed):
    spec = W.TextSpec(n=n, kind="uniform", key=W.text_key(90, seed), sigma=sigma)
    return W.gen_numpy(spec)


def test_capture_search_count_and_batch_in_one_graph(epsm):
    # a single-pass text (fewer than 32 tiles) and a two-phase one (sparse
    # output of a long text), plus a batch of device and host-only plans
    small = uniform_text(3 * TILE + 5, 4, 1)
    big = uniform_text(64 * TILE + 123, 64, 2)
    p_small = small[1000:1006].tobytes()             # dense-ish: single pass
    p_big = big[77_777:77_779].tobytes()             # m = 2 on sigma 64: sparse, two phase
    p_count = big[5_000_000:5_000_017].tobytes()     # fingerprint variant
    exp_small = oracle.positions(small, p_small)
    exp_big = oracle.positions(big, p_big)
    exp_count = oracle.count(big, p_count)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t_small = torch.from_numpy(small).cuda()
        t_big = torch.from_numpy(big).cuda()
        out_small = torch.full((exp_small.size,), -1, dtype=torch.int64, device="cuda")
        out_big = torch.full((exp_big.size,), -1, dtype=torch.int64, device="cuda")
        hits = torch.zeros(3, dtype=torch.int64, device="cuda")
    plans = [epsm.Plan(p_small), epsm.Plan(p_big), epsm.Plan(p_count)]
    bpairs = [(0, epsm.Plan(small[:3].tobytes(), epsm.PLAN_HOST_ONLY)), (1, plans[1]),
              (1, epsm.Plan(big[99:120].tobytes(), epsm.PLAN_HOST_ONLY)), (0, plans[0])]
    bexp = [oracle.positions(small if ti == 0 else big, p.pattern) for ti, p in bpairs]
    btotal = sum(e.size for e in bexp)
    with torch.cuda.stream(s):
        bout = torch.full((btotal,), -1, dtype=torch.int64, device="cuda")
    batch = epsm.Batch([t_small, t_big], bpairs, out=bout)
    s.synchronize()
    epsm.reserve(big.size, batch.workspace_bytes(), stream=s)
    s.synchronize()
    say(f"capture: search n={small.size}, search n={big.size}, count m=17, batch of {len(bpairs)} pairs")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        epsm.search_into(plans[0], t_small, out_small, hits[0:1], s)
        epsm.search_into(plans[1], t_big, out_big, hits[1:2], s)
        epsm.count_into(plans[2], t_big, hits[2:3], s)
        batch.run(s)
    for rep in range(4):
        with torch.cuda.stream(s):  # eager work between replays
            out_small.fill_(-1)
            out_big.fill_(-1)
            hits.fill_(-7)
            bout.fill_(-1)
            batch.counts.fill_(-1)
            batch.offsets.fill_(-1)
        s.synchronize()
        say(f"replay {rep}")
        g.replay()
        epsm.stream_check(s)
        assert np.array_equal(out_small.cpu().numpy(), exp_small)
        assert np.array_equal(out_big.cpu().numpy(), exp_big)
        assert hits.cpu().tolist() == [exp_small.size, exp_big.size, exp_count]
        counts = batch.counts[:len(bpairs)].cpu().numpy()
        offs = batch.offsets[:len(bpairs)].cpu().numpy()
        got = bout.cpu().numpy()
        for k, e in enumerate(bexp):
            assert counts[k] == e.size
            assert np.array_equal(got[offs[k]:offs[k] + counts[k]], e), k
    del g


def test_capture_without_reserve_fails_cleanly(epsm):
    """Under capture nothing is allocated: a stream without workspace reports
    EPSM_EUNSUPPORTED instead of allocating (the capture is then abandoned)."""
    text = torch.from_numpy(uniform_text(4 * TILE, 4, 3)).cuda()
    plan = epsm.Plan(b"\x01\x02\x03")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
        hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    s.synchronize()
    say("capture on a fresh stream without epsm_reserve")
    g = torch.cuda.CUDAGraph()
    err = None
    try:
        with torch.cuda.graph(g, stream=s):
            try:
                epsm.search_into(plan, text, out, hits, s)
            except epsm.EpsmError as e:
                err = e
    except RuntimeError:
        pass  # an empty or invalidated capture may be refused by torch; the status is what counts
    assert err is not None and err.name == "EPSM_EUNSUPPORTED", err
    # the stream still works eagerly afterwards
    s.synchronize()
    exp = oracle.positions(text.cpu().numpy(), b"\x01\x02\x03")
    got = epsm.search(text, plan, stream=s)
    assert np.array_equal(got.cpu().numpy(), exp)


def test_helpers_run_on_the_given_stream(epsm):
    text_np = uniform_text(5 * TILE + 77, 4, 4)
    codes_np = (text_np & 3).astype(np.uint8)
    text = torch.from_numpy(text_np).cuda()
    codes = torch.from_numpy(codes_np).cuda()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for m in (1, 3, 8, 12, 16, 24):
        p = text_np[9000:9000 + m].tobytes()
        say(f"fresh stream: search/count m={m}")
        exp = oracle.positions(text_np, p)
        assert np.array_equal(epsm.search(text, p, stream=s).cpu().numpy(), exp)
        assert epsm.count(text, p, stream=s) == exp.size
    with torch.cuda.stream(s):
        packed = epsm.pack_dna(codes, stream=s)
    for m in (2, 7, 9, 20):
        p = codes_np[31_000:31_000 + m].tobytes()
        say(f"fresh stream: DNA search/count m={m}")
        exp = oracle.positions(codes_np, p)
        assert np.array_equal(epsm.search_dna(packed, codes_np.size, p, stream=s).cpu().numpy(), exp)
        assert epsm.count_dna(packed, codes_np.size, p, stream=s) == exp.size
    say("fresh stream: search_batch")
    pats = [text_np[i:i + m].tobytes() for i, m in ((5, 2), (700, 9), (12345, 20))]
    pos, cnt, off = epsm.search_batch([text], [(0, p) for p in pats], stream=s)
    pos, cnt, off = pos.cpu().numpy(), cnt.cpu().numpy(), off.cpu().numpy()
    for k, p in enumerate(pats):
        assert np.array_equal(pos[off[k]:off[k] + cnt[k]], oracle.positions(text_np, p))


def test_forced_giveup_surfaces(epsm):
    text_np = uniform_text(6 * TILE + 3, 2, 5)
    text = torch.from_numpy(text_np).cuda()
    p = text_np[100:104].tobytes()
    exp = oracle.positions(text_np, p)
    plan = epsm.Plan(p)
    cls = plan.info()["kernel_class"]
    epsm.set_tune_table([(cls, 0, 1 << 40, 8, 16, epsm.WRITE_SINGLE_PASS)])
    s = torch.cuda.Stream()
    try:
        epsm.debug_force_giveup(True)
        with torch.cuda.stream(s):
            out = torch.empty(exp.size, dtype=torch.int64, device="cuda")
            hits = torch.zeros(1, dtype=torch.int64, device="cuda")
        say("single-pass search with a forced give-up")
        epsm.search_into(plan, text, out, hits, s)
        with pytest.raises(epsm.EpsmError) as ei:
            epsm.stream_check(s)
        assert ei.value.name == "EPSM_EDEVICE"
        # the forced wait is an extra one: the output itself is complete
        assert np.array_equal(out.cpu().numpy(), exp)
        epsm.stream_check(s)  # reported once, then cleared
        say("the synchronising helper raises")
        with pytest.raises(epsm.EpsmError):
            epsm.search(text, plan, stream=s)
    finally:
        epsm.debug_force_giveup(False)
        epsm.set_tune_table([])
    epsm.stream_check(s)
    assert np.array_equal(epsm.search(text, plan, stream=s).cpu().numpy(), exp)


def test_serving_output_allocation_failure_releases_memory(epsm):
    from paper_1209_6449_amd import serve
    specs = W.config5_texts(n_texts=4, min_len=1 << 16, max_len=1 << 20)
    texts = [W.gen_bytes(sp, device="cuda") for sp in specs]
    torch.cuda.synchronize()
    # cut patterns always hit, so every micro-batch has output to allocate
    g = W.rng(90, 7)
    queries = [W.Query(0.0, i % 4, [W.cut_pattern(specs[i % 4], 6, g)[0] for _ in range(3)]) for i in range(8)]
    say("server whose output allocations fail")
    with serve.Server(slots=2, max_batch_queries=2, flags=epsm._lib.SERVER_FAIL_OUTPUT_ALLOC) as srv:
        for t in texts:
            srv.add_text(t)
        outs, _, _ = serve.run_queries(srv, queries)
        assert all(o.status == epsm._lib.EPSM_ENOMEM for o in outs), [o.status for o in outs]
        st = srv.stats()
        assert st["completed"] == len(queries) and st["bytes_reserved"] == 0
    say("the same queries on a normal server")
    host = [t.cpu().numpy() for t in texts]
    with serve.Server(slots=2, max_batch_queries=2) as srv:
        for t in texts:
            srv.add_text(t)
        outs, _, _ = serve.run_queries(srv, queries)
        for o, q in zip(outs, queries):
            assert o.status == 0
            for k, p in enumerate(q.patterns):
                assert np.array_equal(o.pattern_positions(k), oracle.positions(host[q.text], p))


def _loaded_hip_runtime():
    """The HIP runtime this process has loaded (the one the library uses)."""
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1]
            if "libamdhip64.so" in path:
                return ctypes.CDLL(path)
    pytest.skip("HIP runtime not found in the process")


def test_stale_runtime_error_does_not_fail_launches(epsm):
    """Each library call runs right after the stale error, with nothing in
    between (PyTorch's own launches would report that error too)."""
    hip = _loaded_hip_runtime()
    hip.hipSetDevice.restype = ctypes.c_int
    hip.hipSetDevice.argtypes = [ctypes.c_int]
    t = uniform_text(1 << 20, 4, 7)
    text = torch.from_numpy(t).cuda()
    pat, pat2 = t[1000:1003].tobytes(), t[5:25].tobytes()
    exp, exp2 = oracle.positions(t, pat), oracle.positions(t, pat2)
    plan, plan2 = epsm.Plan(pat), epsm.Plan(pat2)
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.full((len(exp) + len(exp2),), -1, dtype=torch.int64, device="cuda")
    b = epsm.Batch([text], [(0, plan), (0, plan2)], out=out)
    torch.cuda.synchronize()
    # an ordinal no device has: the call only returns an error, and leaves it
    # as the thread's last error
    say("stale error, then a count")
    assert hip.hipSetDevice(1 << 20) != 0
    epsm.count_into(plan, text, hits)
    torch.cuda.synchronize()
    assert int(hits.item()) == len(exp)
    say("stale error, then a batch")
    assert hip.hipSetDevice(1 << 20) != 0
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.concatenate([exp, exp2]))
    epsm.stream_check()

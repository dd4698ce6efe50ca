"""Batched search: output identical to per-pair plain searches and to the oracle.

Integer work: bit-exact equality of positions, counts and offsets.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def epsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as mod
    mod.lib()
    return mod


def say(msg):
    print(msg, flush=True)


def make_batch(seed, n_texts=60, min_len=1, max_len=300_000, max_pat=40):
    """Texts of log-uniform length (some empty / shorter than m), sigma 2/4/64,
    patterns cut or random with m in [1, 40], pairs in shuffled order."""
    rng = np.random.default_rng(seed)
    texts, host, pairs = [], [], []
    for i in range(n_texts):
        if i % 17 == 0:
            n = 0
        else:
            n = int(math.exp(rng.uniform(math.log(max(min_len, 1)), math.log(max_len))))
        sigma = int(rng.choice([2, 4, 64]))
        t = rng.integers(0, sigma, n).astype(np.uint8)
        off = int(rng.integers(0, 16))  # unaligned starts
        buf = torch.zeros(n + off + 1, dtype=torch.uint8, device="cuda")
        if n:
            buf[off:off + n] = torch.from_numpy(t).cuda()
        texts.append(buf[off:off + n])
        host.append(t)
        for _ in range(int(rng.integers(1, max_pat))):
            m = int(rng.integers(1, 41))
            if n >= m and rng.random() < 0.6:
                o = int(rng.integers(0, n - m + 1))
                p = t[o:o + m].tobytes()
            else:
                p = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
            pairs.append((i, p))
    order = rng.permutation(len(pairs))
    pairs = [pairs[k] for k in order]
    return texts, host, pairs


@pytest.mark.parametrize("waves", [4, 8, 16])
def test_batch_equals_plain_and_oracle(epsm, waves):
    epsm.set_batch_config(waves)
    texts, host, pairs = make_batch(seed=waves)
    plans = [(ti, epsm.Plan(p)) for ti, p in pairs]
    say(f"batch waves={waves} texts={len(texts)} pairs={len(pairs)}")
    pos, counts, offsets = epsm.search_batch(texts, plans)
    epsm.stream_check()
    pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
    assert offsets[0] == 0
    assert np.array_equal(offsets[1:], np.cumsum(counts)[:-1])
    for k, (ti, plan) in enumerate(plans):
        got = pos[offsets[k]:offsets[k] + counts[k]]
        exp = oracle.positions(host[ti], plan.pattern)
        assert np.array_equal(got, exp), (k, ti, len(plan.pattern))
        if k % 7 == 0:
            plain = epsm.search(texts[ti], plan).cpu().numpy()
            assert np.array_equal(plain, got)
    epsm.set_batch_config(8)


def test_count_only_batch(epsm):
    texts, host, pairs = make_batch(seed=5, n_texts=30)
    plans = [(ti, epsm.Plan(p)) for ti, p in pairs]
    b = epsm.Batch(texts, plans, count_only=True)
    say("count-only batch")
    b.run()
    counts = b.counts[:len(plans)].cpu().numpy()
    for k, (ti, plan) in enumerate(plans):
        assert counts[k] == oracle.count(host[ti], plan.pattern)
    assert int(b.total.item()) == counts.sum()


def test_truncated_batch_output_is_prefix(epsm):
    texts, host, pairs = make_batch(seed=9, n_texts=20)
    plans = [(ti, epsm.Plan(p)) for ti, p in pairs]
    full, counts, offsets = epsm.search_batch(texts, plans)
    total = full.numel()
    for cap in (0, 1, total // 3, total - 1):
        say(f"truncated batch cap={cap} of {total}")
        out = torch.full((max(cap, 1),), -5, dtype=torch.int64, device="cuda")
        b = epsm.Batch(texts, plans, out=out[:cap] if cap else None)
        b.run()
        assert torch.equal(b.counts[:len(plans)], counts)
        assert torch.equal(b.offsets[:len(plans)], offsets)
        assert int(b.total.item()) == total
        if cap:
            assert torch.equal(out[:cap], full[:cap])


def test_prepared_batch_graph_replays(epsm):
    """A prepared batch replays its captured graph; every replay is identical,
    with eager work and synchronisation between replays."""
    texts, host, pairs = make_batch(seed=13, n_texts=40)
    plans = [(ti, epsm.Plan(p)) for ti, p in pairs]
    ref, counts, offsets = epsm.search_batch(texts, plans)
    total = ref.numel()
    out = torch.full((max(total, 1),), -1, dtype=torch.int64, device="cuda")
    b = epsm.Batch(texts, plans, out=out[:total] if total else None)
    bp = epsm.BatchPlan(b)
    info = bp.info()
    assert info["units"] > 0 and info["entries"] >= info["units"]
    stream = torch.cuda.Stream()
    for r in range(4):
        say(f"graph replay {r}")
        out.fill_(-1)
        b.counts.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            bp.launch(stream)
        stream.synchronize()
        assert torch.equal(out[:total], ref)
        assert torch.equal(b.counts[:len(plans)], counts)
        assert torch.equal(b.offsets[:len(plans)], offsets)
        # unrelated eager work between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
    bp.close()


def test_batch_with_config4_shapes_small(epsm):
    """A scaled-down config-4 batch (log-uniform lengths, sigma 4/64, 1-64
    patterns, m uniform in [1, 32], half cut / half random)."""
    bts = W.config4(n_texts=40, min_len=1 << 10, max_len=1 << 18)
    texts = [W.gen_bytes(bt.spec, device="cuda") for bt in bts]
    host = [t.cpu().numpy() for t in texts]
    pairs = [(i, epsm.Plan(p)) for i, bt in enumerate(bts) for p in bt.patterns]
    say(f"config4-small pairs={len(pairs)}")
    pos, counts, offsets = epsm.search_batch(texts, pairs)
    pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
    for k, (ti, plan) in enumerate(pairs):
        exp = oracle.positions(host[ti], plan.pattern)
        assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), k


def test_parked_hits_at_the_list_boundary(epsm):
    """Grouped hits are parked per 4 KiB unit up to 64: a unit with exactly
    64 (one of them crossing into the next unit), a unit with 65 (the write
    pass recomputes it), a unit with a few; and texts whose grouped patterns
    are all of m = 4..7 (4-byte keys) or all of m >= 8 (8-byte keys).
    Patterns use bytes the texts never hold, so the planted hits are all."""
    epsm.set_batch_config(4)
    try:
        rng = np.random.default_rng(77)
        U = 4096

        def pattern(m):
            return bytes(rng.integers(200, 256, m).astype(np.uint8))

        def text_with(n, plants):
            t = rng.integers(0, 64, n).astype(np.uint8)
            for off, p in plants:
                t[off:off + len(p)] = np.frombuffer(p, dtype=np.uint8)
            return t

        mixed = [pattern(m) for m in (4, 5, 6, 7, 8, 11, 16, 24)]
        plants = [(60 * i, mixed[i % 8]) for i in range(63)] + [(U - 3, mixed[4])]  # unit 0: 64
        plants += [(U + 16 + 60 * i, mixed[i % 8]) for i in range(65)]               # unit 1: 65
        plants += [(2 * U + 100 * i, mixed[i % 8]) for i in range(10)]               # unit 2: 10
        short = [pattern(m) for m in (4, 5, 6, 7, 5)]
        long_ = [pattern(m) for m in (8, 9, 12, 20, 31, 33)]
        host = [text_with(3 * U, plants),
                text_with(2 * U + 77, [(50 * i, short[i % 5]) for i in range(120)]),
                text_with(2 * U + 5, [(70 * i, long_[i % 6]) for i in range(100)])]
        texts = [torch.from_numpy(t.copy()).cuda() for t in host]
        pairs = [(0, epsm.Plan(p, epsm.PLAN_HOST_ONLY if k % 2 else 0)) for k, p in enumerate(mixed)]
        pairs += [(0, epsm.Plan(bytes([7])))]  # a solo pair beside the groups
        pairs += [(1, epsm.Plan(p)) for p in short] + [(2, epsm.Plan(p, epsm.PLAN_HOST_ONLY)) for p in long_]
        for groups in (True, False):
            say(f"parked-hit boundary: groups={groups}")
            pos, counts, offsets = epsm.search_batch(texts, pairs, groups=groups)
            epsm.stream_check()
            pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
            for k, (ti, plan) in enumerate(pairs):
                exp = oracle.positions(host[ti], plan.pattern)
                assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), (k, groups)
        assert sum(int(c) for c in counts[:8]) == 64 + 65 + 10
    finally:
        epsm.set_batch_config(8)


def test_grouped_pairs_carry_no_fingerprint_table(epsm):
    """Host-only fingerprint plans (m >= 16) filtered in a group bring no
    hash table into the batch (only ungrouped ones do), and their output
    is the same either way, including a unit whose group hits overflow
    its park list and are recomputed."""
    rng = np.random.default_rng(91)
    n = 3 * 8192
    t = rng.integers(0, 4, n).astype(np.uint8)
    pats = [t[o:o + m].tobytes() for o, m in zip(rng.integers(0, n - 40, 12), (16, 17, 20, 24, 28, 31, 32, 18,
                                                                            16, 22, 26, 30))]
    stem = bytes(rng.integers(200, 256, 20).astype(np.uint8))
    for i in range(80):  # 80 hits of one pattern inside the first 8 KiB
        t[90 * i:90 * i + 20] = np.frombuffer(stem, dtype=np.uint8)
    pats.append(stem)
    text = torch.from_numpy(t.copy()).cuda()
    plans = [(0, epsm.Plan(p, epsm.PLAN_HOST_ONLY)) for p in pats]
    assert all(pl.info()["variant"] == epsm.VARIANT_FINGERPRINT for _, pl in plans)
    grouped = epsm.Batch([text], plans).workspace_bytes()
    alone = epsm.Batch([text], plans, groups=False).workspace_bytes()
    say(f"workspace grouped={grouped} ungrouped={alone}")
    assert alone - grouped >= len(plans) * 4096 - 2 * 5120
    for groups in (True, False):
        pos, counts, offsets = [x.cpu().numpy() for x in epsm.search_batch([text], plans, groups=groups)]
        epsm.stream_check()
        for k, (_, plan) in enumerate(plans):
            exp = oracle.positions(t, plan.pattern)
            assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), (k, groups)
    assert counts[-1] == 80


def test_shared_host_plans_grouped_and_alone(epsm):
    """One host-only plan object in several pairs: grouped in a text with
    many patterns, alone in a text with few, and twice in one text; long
    fingerprint plans among them.  The table travels once, for the pairs
    filtered alone, and every pair's positions equal the oracle's."""
    rng = np.random.default_rng(93)
    host = [rng.integers(0, 4, n).astype(np.uint8) for n in (40000, 30000, 9000)]
    texts = [torch.from_numpy(t.copy()).cuda() for t in host]
    shared = [epsm.Plan(host[0][o:o + m].tobytes(), epsm.PLAN_HOST_ONLY)
              for o, m in ((100, 20), (2000, 33), (7000, 17), (5000, 9))]
    many = [epsm.Plan(host[0][o:o + m].tobytes(), epsm.PLAN_HOST_ONLY)
            for o, m in zip(rng.integers(0, 30000, 10), (4, 5, 8, 12, 16, 24, 30, 6, 10, 40))]
    pairs = [(0, p) for p in shared + many]          # text 0: all grouped (m >= 4)
    pairs += [(1, shared[0]), (1, shared[1])]        # text 1: too few to group
    pairs += [(2, shared[2]), (2, shared[2]), (2, shared[3])] + [(2, p) for p in many[:3]]
    order = rng.permutation(len(pairs))
    pairs = [pairs[k] for k in order]
    say(f"shared host plans: {len(pairs)} pairs")
    pos, counts, offsets = [x.cpu().numpy() for x in epsm.search_batch(texts, pairs)]
    epsm.stream_check()
    for k, (ti, plan) in enumerate(pairs):
        exp = oracle.positions(host[ti], plan.pattern)
        assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), (k, ti, plan.m)


def test_empty_batch(epsm):
    say("empty batch")
    b = epsm.Batch([], [], count_only=False)
    b.run()
    assert int(b.total.item()) == 0


def test_host_only_and_mixed_plans(epsm):
    """Host-only plans travel inside the batch; output is unchanged."""
    texts, host, pairs = make_batch(seed=21, n_texts=30)
    mixed = []
    for k, (ti, p) in enumerate(pairs):
        flags = epsm.PLAN_HOST_ONLY if k % 3 else 0
        if k % 5 == 0 and len(p) >= 15:
            flags |= epsm.PLAN_FORCE_FINGERPRINT
        if k % 11 == 0 and len(p) >= 15:
            flags |= epsm.PLAN_FORCE_FINGERPRINT | epsm.PLAN_COLLIDE
        mixed.append((ti, epsm.Plan(p, flags)))
    # the same plan object in several pairs is uploaded once
    mixed += [mixed[0], mixed[1], mixed[0]]
    say(f"mixed host/device plans pairs={len(mixed)}")
    pos, counts, offsets = epsm.search_batch(texts, mixed)
    pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
    for k, (ti, plan) in enumerate(mixed):
        exp = oracle.positions(host[ti], plan.pattern)
        assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), k


def test_host_only_direct_plans_m17_to_32(epsm):
    """Host-only direct plans of m in [17, 32] (three loads per lane, all of
    the pattern compared from registers): their pattern is not uploaded, so
    no pass may read it; cut patterns make every pass write positions."""
    texts, host, _ = make_batch(seed=33, n_texts=24, min_len=2000)
    rng = np.random.default_rng(33)
    pairs = []
    for ti, t in enumerate(host):
        for m in (17, 20, 24, 31, 32):
            if t.size < m:
                continue
            o = int(rng.integers(0, t.size - m + 1))
            pairs.append((ti, epsm.Plan(t[o:o + m].tobytes(), epsm.PLAN_HOST_ONLY | epsm.PLAN_FORCE_DIRECT)))
    assert any(pl.info()["run_blocks"] == 3 for _, pl in pairs)
    # grouped: the count pass parks the hits; ungrouped: the write pass
    # recomputes every pair (16 bytes from registers, then the tail check
    # against the uploaded pattern)
    for groups in (True, False):
        say(f"host-only direct m 17..32: pairs={len(pairs)} groups={groups}")
        pos, counts, offsets = epsm.search_batch(texts, pairs, groups=groups)
        epsm.stream_check()
        pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
        for k, (ti, plan) in enumerate(pairs):
            exp = oracle.positions(host[ti], plan.pattern)
            assert exp.size >= 1
            assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), (k, groups)


def test_long_patterns_in_batch(epsm):
    """m > 32 needs the tail check against the pattern in device memory."""
    rng = np.random.default_rng(77)
    t = rng.integers(0, 2, 200_000).astype(np.uint8)
    text = torch.from_numpy(t).cuda()
    pats = []
    for m in (33, 40, 64, 100, 300):
        o = int(rng.integers(0, t.size - m))
        pats.append(t[o:o + m].tobytes())
        pats.append((b"\x00\x01" * 200)[:m])
    plans = [(0, epsm.Plan(p, epsm.PLAN_HOST_ONLY if i % 2 else 0)) for i, p in enumerate(pats)]
    say("long patterns in batch")
    pos, counts, offsets = epsm.search_batch([text], plans)
    pos, counts, offsets = pos.cpu().numpy(), counts.cpu().numpy(), offsets.cpu().numpy()
    for k, (ti, plan) in enumerate(plans):
        assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], oracle.positions(t, plan.pattern)), k


def group_batch(seed, n_texts=12, n_pat=70):
    """Texts with many patterns each (several 32-pattern groups): patterns
    sharing their first four bytes (same bucket, different tails), m from 4
    to 100 (past the 32 bytes checked from LDS), dense binary texts, cuts at
    both ends of the text, unaligned starts."""
    rng = np.random.default_rng(seed)
    texts, host, pairs = [], [], []
    for i in range(n_texts):
        n = int(rng.integers(1, 200_000)) if i % 5 else int(rng.integers(1, 64))
        sigma = [2, 4, 64][i % 3]
        t = rng.integers(0, sigma, n).astype(np.uint8)
        off = int(rng.integers(0, 16))
        buf = torch.zeros(n + off + 1, dtype=torch.uint8, device="cuda")
        if n:
            buf[off:off + n] = torch.from_numpy(t).cuda()
        texts.append(buf[off:off + n])
        host.append(t)
        stem = rng.integers(0, sigma, 4).astype(np.uint8).tobytes()
        for j in range(n_pat):
            m = int(rng.choice([1, 3, 4, 5, 8, 15, 16, 17, 31, 32, 33, 40, 64, 100]))
            r = rng.random()
            if n >= m and r < 0.4:
                o = [0, n - m, int(rng.integers(0, n - m + 1))][j % 3]
                p = t[o:o + m].tobytes()
            elif r < 0.7 and m >= 4:
                p = stem + rng.integers(0, sigma, m - 4).astype(np.uint8).tobytes()
            else:
                p = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
            pairs.append((i, p))
    return texts, host, pairs


@pytest.mark.parametrize("waves", [4, 16])
def test_grouped_count_equals_ungrouped_and_oracle(epsm, waves):
    epsm.set_batch_config(waves)
    try:
        texts, host, pairs = group_batch(seed=100 + waves)
        plans = [(ti, epsm.Plan(p, epsm.PLAN_HOST_ONLY if k % 2 else 0)) for k, (ti, p) in enumerate(pairs)]
        say(f"grouped batch waves={waves} pairs={len(plans)}")
        g = [x.cpu().numpy() for x in epsm.search_batch(texts, plans, groups=True)]
        say("ungrouped")
        u = [x.cpu().numpy() for x in epsm.search_batch(texts, plans, groups=False)]
        epsm.stream_check()
        for a, b in zip(g, u):
            assert np.array_equal(a, b)
        pos, counts, offsets = g
        for k, (ti, plan) in enumerate(plans):
            exp = oracle.positions(host[ti], plan.pattern)
            assert np.array_equal(pos[offsets[k]:offsets[k] + counts[k]], exp), (k, ti, plan.m)
    finally:
        epsm.set_batch_config(8)

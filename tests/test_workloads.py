"""Pins of the seeded input generators (no matching arithmetic lives there)."""
import numpy as np
import torch

import workloads as W


def test_splitmix64_tensor_matches_integer_definition():
    ctr = torch.tensor([0, 1, 2, 1 << 40, (1 << 62) + 12345], dtype=torch.int64)
    for key in (0, 1, W.SEED_BASE, (1 << 64) - 1):
        got = W.splitmix64(ctr, key).tolist()
        ref = [W._as_i64(W.splitmix64_int(int(c), key)) for c in ctr.tolist()]
        assert got == ref


def test_splitmix64_known_value():
    # splitmix64 seeded with 0: the first output is 0xE220A8397B1DCDAF
    assert W.splitmix64_int(0, 0) == 0xE220A8397B1DCDAF


def test_subrange_equals_slice_of_full_text():
    spec = W.TextSpec(n=10_000, kind="uniform", key=77, sigma=20)
    full = W.gen_numpy(spec)
    for a, L in [(0, 1), (3, 17), (4, 4), (9_990, 10), (1234, 4321)]:
        assert np.array_equal(W.gen_numpy(spec, a, L), full[a:a + L])
    # chunked generation gives the same bytes
    chunked = W.gen_bytes(spec, 0, spec.n, chunk=999).numpy()
    assert np.array_equal(chunked, full)


def test_uniform_alphabet_and_balance():
    spec = W.TextSpec(n=1 << 20, kind="uniform", key=5, sigma=4, alphabet=b"ACGT")
    t = W.gen_numpy(spec)
    counts = np.bincount(t, minlength=256)
    assert set(np.nonzero(counts)[0].tolist()) == set(b"ACGT")
    assert np.all(np.abs(counts[list(b"ACGT")] / t.size - 0.25) < 0.005)


def test_codes_zero_based():
    spec = W.TextSpec(n=1 << 16, kind="uniform", key=9, sigma=128)
    t = W.gen_numpy(spec)
    assert t.min() == 0 and t.max() == 127


def test_zipf_table_law():
    tab = W.zipf_table()
    order = W.english_rank_order()
    assert len(set(order.tolist())) == 96 and order[0] == 0x20 and 0x0A in order
    slots = np.array([np.count_nonzero(tab == s) for s in order])
    ranks = np.arange(1, 97)
    expect = 65536 * (1 / ranks) / np.sum(1 / ranks)
    assert np.all(np.abs(slots - expect) <= 1.0)


def test_cut_patterns_occur_at_their_offset():
    spec, cases = W.config1(n=1 << 16)
    t = W.gen_numpy(spec)
    assert len(cases) == 100
    for c in cases:
        assert bytes(t[c.offset:c.offset + len(c.pattern)]) == c.pattern


def test_configs_are_deterministic():
    a = W.config2(4, n=1 << 16)[1]
    b = W.config2(4, n=1 << 16)[1]
    assert [c.pattern for c in a] == [c.pattern for c in b]
    q1 = W.config5_queries(W.config5_texts(8, 1 << 12, 1 << 14), 20, 100.0)
    q2 = W.config5_queries(W.config5_texts(8, 1 << 12, 1 << 14), 20, 100.0)
    assert [(q.arrival, q.text, q.patterns) for q in q1] == [(q.arrival, q.text, q.patterns) for q in q2]


def test_small_ranges_equal_tensor_generator():
    """The numpy path for short ranges gives the same bytes as the tensor path."""
    specs = [W.TextSpec(n=1 << 20, kind="uniform", key=W.text_key(4, 3), sigma=64),
             W.TextSpec(n=1 << 20, kind="zipf96", key=W.text_key(3, 0)),
             W.TextSpec(n=1 << 20, kind="uniform", key=W.text_key(1, 0), sigma=4, alphabet=b"ACGT"),
             W.TextSpec(n=1 << 20, kind="periodic", fill=0x61)]
    for spec in specs:
        for start, length in ((0, 1), (3, 17), (1001, 32), (5, 4096), ((1 << 20) - 33, 33), (77, 0)):
            small = W.gen_numpy(spec, start, length)
            ref = W.gen_bytes(spec, start, length, device="cpu").numpy()
            assert small.dtype == np.uint8 and np.array_equal(small, ref), (spec.kind, start, length)

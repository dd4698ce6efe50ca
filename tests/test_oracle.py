"""Pins of the CPU oracle against facts fixed outside the oracle itself.

* the paper's worked examples (Section 3.1), stored under tests/golden/
* closed forms of the exact string matching problem (Introduction, Section 2)
* a library routine: iterated bytes.find yields every (overlapping) occurrence
* exhaustive enumeration on tiny inputs against that routine
"""
import itertools
import random

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def find_all(text: bytes, pat: bytes) -> list[int]:
    """Every occurrence via the library's bytes.find, restarting one past each hit."""
    hits, i = [], text.find(pat)
    while i != -1:
        hits.append(i)
        i = text.find(pat, i + 1)
    return hits


# ---------------------------------------------------------------- worked examples


def test_wscmp_worked_example(golden):
    g = golden("wscmp_example.txt")
    assert oracle.wscmp(g["a"], g["b"]) == g["r"]


def test_wsmatch_worked_example(golden):
    g = golden("wsmatch_example.txt")
    assert oracle.wsmatch(g["a"], g["b"]) == g["r"]


def test_search_reproduces_wsmatch_example(golden):
    """The worked example is an instance of the full problem: Occ(b, a) = {r}."""
    g = golden("wsmatch_example.txt")
    a, b = bytes(g["a"]), bytes(g["b"])
    expected = oracle.mask_set(g["r"])
    assert expected == [1, 5]
    assert oracle.positions(a, b).tolist() == expected
    assert oracle.occurrences_py(g["a"], g["b"]) == expected
    assert oracle.count(a, b) == 2


def test_wsblend_worked_example(golden):
    g = golden("wsblend_example.txt")
    assert oracle.wsblend(g["a"], g["b"]) == g["r"]


def test_wsmatch_relates_to_wscmp_on_single_symbol():
    """wsmatch with k = 1 against a broadcast word is wscmp (Section 3.2's B_j)."""
    a = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5, 8]
    for c in set(a):
        assert oracle.wsmatch(a, [c]) == oracle.wscmp(a, [c] * len(a))


# ---------------------------------------------------------------- closed forms


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (10, 3), (100, 100), (1000, 7), (4097, 16)])
def test_unary_text_all_positions(n, m):
    """a^n with pattern a^m: exactly n-m+1 hits at 0..n-m."""
    t, p = b"a" * n, b"a" * m
    pos, total = oracle.search(t, p)
    assert total == n - m + 1
    assert pos.tolist() == list(range(n - m + 1))
    assert int(pos.sum()) == (n - m) * (n - m + 1) // 2


def test_absent_symbol_gives_zero():
    rng = np.random.default_rng(1)
    t = rng.integers(0, 4, 5000).astype(np.uint8)
    for m in (1, 2, 5, 16, 33):
        p = np.concatenate([rng.integers(0, 4, m - 1), [7]]).astype(np.uint8)
        assert oracle.count(t, p) == 0
        assert oracle.count_mt(t, p, 4) == 0


def test_pattern_longer_than_text_and_empty_text():
    assert oracle.count(b"abc", b"abcd") == 0
    assert oracle.count(b"", b"a") == 0
    assert oracle.positions(b"", b"a").tolist() == []


def test_pattern_equals_text():
    for t in (b"x", b"\x00\x00\x01", bytes(range(256)), b"ab" * 50):
        assert oracle.positions(t, t).tolist() == [0]


def test_period_two_text_even_positions():
    """(ab)^h with pattern (ab)^k: every even s <= 2h - 2k; odd shifts never match."""
    h = 300
    for k in (1, 2, 5, 16):
        t, p = b"ab" * h, b"ab" * k
        assert oracle.positions(t, p).tolist() == list(range(0, 2 * h - 2 * k + 1, 2))
        assert oracle.count(t, b"ba" * k) == h - k


def test_last_position_is_reported():
    """An occurrence ending at t[n-1] (start n-m) is reported."""
    t = b"xxxxxxxxxxABCD"
    assert oracle.positions(t, b"ABCD").tolist() == [len(t) - 4]
    assert oracle.positions(t, b"D").tolist() == [len(t) - 1]


def test_zero_byte_is_a_symbol():
    t = bytes([0, 0, 1, 0, 0, 0, 2, 0])
    assert oracle.positions(t, b"\x00\x00").tolist() == [0, 3, 4]
    assert oracle.positions(t, b"\x00").tolist() == [0, 1, 3, 4, 5, 7]
    assert oracle.positions(t, bytes([0, 2])).tolist() == [5]


def test_high_bytes():
    t = bytes([255, 254, 255, 255, 128, 255])
    assert oracle.positions(t, bytes([255])).tolist() == [0, 2, 3, 5]
    assert oracle.positions(t, bytes([255, 255])).tolist() == [2]


# ---------------------------------------------------------------- library routine


def test_exhaustive_binary_tiny():
    """All texts over {0,1} of length <= 10 x all patterns of length 1..4."""
    pats = [bytes(p) for m in range(1, 5) for p in itertools.product(b"\x00\x01", repeat=m)]
    for n in range(0, 11):
        for tt in itertools.product(b"\x00\x01", repeat=n):
            t = bytes(tt)
            for p in pats:
                expect = find_all(t, p)
                got = oracle.positions(t, p).tolist()
                assert got == expect, (t, p)
                assert oracle.count(t, p) == len(expect)


def test_python_twin_exhaustive_ternary():
    for n in range(0, 7):
        for tt in itertools.product((0, 1, 2), repeat=n):
            for m in (1, 2, 3):
                for p in itertools.product((0, 1, 2), repeat=m):
                    assert oracle.occurrences_py(tt, p) == find_all(bytes(tt), bytes(p))


@pytest.mark.parametrize("sigma", [1, 2, 4, 20, 256])
def test_random_against_find(sigma):
    rng = random.Random(sigma)
    for _ in range(30):
        n = rng.randint(0, 100_000)
        t = bytes(rng.randrange(sigma) for _ in range(n)) if n < 5000 else \
            np.random.default_rng(rng.randrange(1 << 30)).integers(0, sigma, n).astype(np.uint8).tobytes()
        m = rng.randint(1, 40)
        if n >= m and rng.random() < 0.5:
            o = rng.randint(0, n - m)
            p = t[o:o + m]
        else:
            p = bytes(rng.randrange(sigma) for _ in range(m))
        expect = find_all(t, p)
        pos, total = oracle.search(t, p)
        assert total == len(expect)
        assert pos.tolist() == expect
        assert oracle.count_mt(t, p, 7) == len(expect)


def test_truncated_output_is_prefix():
    t, p = b"a" * 1000, b"aa"
    pos, total = oracle.search(t, p, cap=10)
    assert total == 999 and pos.tolist() == list(range(10))


def test_range_partition_concatenates():
    rng = np.random.default_rng(5)
    t = rng.integers(0, 2, 20_000).astype(np.uint8)
    p = bytes([1, 0, 1])
    full = oracle.positions(t, p)
    parts = []
    for a, b in [(0, 777), (777, 5000), (5000, 19_999), (19_999, 40_000)]:
        parts.append(oracle.search_range(t, p, a, b, 20_000)[0])
    assert np.array_equal(np.concatenate(parts), full)


def test_count_mt_matches_single_thread():
    rng = np.random.default_rng(11)
    t = rng.integers(0, 3, 200_003).astype(np.uint8)
    for threads in (1, 2, 3, 8, 64):
        for p in (b"\x00", b"\x01\x02", b"\x00\x00\x00\x00"):
            assert oracle.count_mt(t, p, threads) == oracle.count(t, p)


@pytest.mark.parametrize("sigma", [1, 2, 4, 64])
def test_range_mt_against_find(sigma):
    """Threaded positions over contiguous start ranges equal iterated bytes.find."""
    rng = np.random.default_rng(100 + sigma)
    for trial in range(12):
        n = int(rng.integers(0, 60_000))
        t = rng.integers(0, sigma, n).astype(np.uint8).tobytes()
        m = int(rng.integers(1, 12))
        if n >= m and trial % 2 == 0:
            o = int(rng.integers(0, n - m + 1))
            p = t[o:o + m]
        else:
            p = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
        full = find_all(t, p)
        for threads in (1, 2, 5, 16, 33):
            a = int(rng.integers(0, n + 2))
            b = int(rng.integers(a, n + 10))
            got = oracle.search_range_mt(t, p, a, b, threads)
            assert got.dtype == np.int64
            assert got.tolist() == [s for s in full if a <= s < b]
        assert oracle.search_range_mt(t, p, 0, n, 7).tolist() == full


def test_range_mt_unary_closed_form():
    """a^n with a^m: every start hits, so every thread range is full."""
    n = 1 << 20
    t = b"a" * n
    for m in (1, 3, 16):
        got = oracle.search_range_mt(t, b"a" * m, 0, n, 9)
        assert got.size == n - m + 1
        assert np.array_equal(got, np.arange(n - m + 1, dtype=np.int64))
        assert int(got.sum()) == (n - m) * (n - m + 1) // 2

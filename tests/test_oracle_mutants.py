"""The oracle's pins must catch plausible mistakes in it.

Each mutant is the oracle's C source with one deliberate slip (a dropped
term, a wrong bound, a wrong index, a transposed operand).  The mutants are
compiled into a temporary directory on the CPU and run through the same pin
battery as the real oracle: the real one passes every pin, each mutant fails
at least one.
"""
import itertools
import os
import random

import pytest

import oracle
from tests.conftest import read_golden

SRC = os.path.join(os.path.dirname(oracle.__file__), "epsm_oracle.c")

MUTANTS = {
    # strict bound of the last start (drops the occurrence ending at t[n-1])
    "strict-last-start": ("if (s_end > last + 1)\n        s_end = last + 1;",
                          "if (s_end > last)\n        s_end = last;"),
    # compares only m-1 characters
    "short-compare": ("for (uint64_t j = 0; j < m; j++)", "for (uint64_t j = 0; j + 1 < m; j++)"),
    # skips the first character
    "skip-first": ("for (uint64_t j = 0; j < m; j++)", "for (uint64_t j = 1; j < m; j++)"),
    # pattern read backwards
    "reversed-pattern": ("if (t[s + j] != p[j])", "if (t[s + j] != p[m - 1 - j])"),
    # text and pattern swapped in the inner index
    "transposed": ("if (t[s + j] != p[j])", "if (t[j] != p[j])"),
    # one-based positions
    "one-based": ("out[count] = (int64_t)s;", "out[count] = (int64_t)(s + 1);"),
    # rejects m == n (p = t)
    "m-equals-n": ("if (m == 0 || m > n)\n        return 0;\n    uint64_t last",
                   "if (m == 0 || m >= n)\n        return 0;\n    uint64_t last"),
    # non-overlapping occurrences only
    "no-overlap": ("            count++;\n        }\n    }\n    return count;",
                   "            count++;\n            s += m - 1;\n        }\n    }\n    return count;"),
    # threaded positions: ranges' results not moved together (gaps left between them)
    "mt-no-compaction": ("out[total + k] = jobs[i].out[k];", "out[k] = jobs[i].out[k];"),
    # threaded positions: each range after the first skips its first start
    "mt-split-gap": ("jobs[i].s_begin = s_begin + starts * (uint64_t)i / (uint64_t)threads;",
                     "jobs[i].s_begin = s_begin + starts * (uint64_t)i / (uint64_t)threads + (i > 0);"),
    # threaded positions: drops the last valid start
    "mt-last-start": ("if (s_end > n - m + 1)\n        s_end = n - m + 1;",
                      "if (s_end > n - m)\n        s_end = n - m;"),
}


def find_all(text: bytes, pat: bytes) -> list[int]:
    hits, i = [], text.find(pat)
    while i != -1:
        hits.append(i)
        i = text.find(pat, i + 1)
    return hits


def pin_battery(o: oracle.Oracle) -> list[str]:
    """Names of the failed pins (empty list = all pins hold)."""
    failed = []
    g = read_golden("wsmatch_example.txt")
    if o.positions(bytes(g["a"]), bytes(g["b"])).tolist() != oracle.mask_set(g["r"]):
        failed.append("wsmatch-example")
    for n, m in [(10, 3), (64, 64), (100, 1)]:
        pos, total = o.search(b"a" * n, b"a" * m)
        if total != n - m + 1 or pos.tolist() != list(range(n - m + 1)):
            failed.append(f"unary-{n}-{m}")
    if o.positions(b"ab" * 40, b"abab").tolist() != list(range(0, 77, 2)):
        failed.append("period-two")
    if o.positions(b"xyzABCD", b"xyzABCD").tolist() != [0]:
        failed.append("p-equals-t")
    if o.count(b"abcabc", b"abd") != 0:
        failed.append("absent")
    rng = random.Random(3)
    for n in (1, 2, 5, 97, 4099):
        t = bytes(rng.randrange(2) for _ in range(n))
        for p in (b"\x01", b"\x00\x01", b"\x01\x01\x00"):
            for threads in (1, 3, 7):
                for a, b in ((0, n), (1, n - 1), (n // 3, n + 5)):
                    exp = [s for s in find_all(t, p) if a <= s < b]
                    if o.search_range_mt(t, p, a, b, threads).tolist() != exp:
                        failed.append("range-mt")
                        break
    pats = [bytes(p) for mm in range(1, 4) for p in itertools.product(b"\x00\x01", repeat=mm)]
    for n in range(0, 8):
        for tt in itertools.product(b"\x00\x01", repeat=n):
            t = bytes(tt)
            for p in pats:
                if o.positions(t, p).tolist() != find_all(t, p):
                    failed.append("exhaustive")
                    return failed
    return failed


def test_real_oracle_passes_every_pin():
    assert pin_battery(oracle.Oracle()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(before) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(before, after, 1)
    c_path = tmp_path / "mutant.c"
    c_path.write_text(mutated)
    so_path = str(tmp_path / "libmutant.so")
    oracle.build(so_path, str(c_path))
    failed = pin_battery(oracle.Oracle(oracle.load(so_path)))
    assert failed, f"mutant {name} passed every pin"

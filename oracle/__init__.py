"""CPU oracle for exact string matching.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never
imports it.

Contents
  * search / count / count_mt / search_range / search_range_mt: ctypes wrappers
    over the plain C brute force in epsm_oracle.c (the problem statement of the paper's
    Introduction and Section 2: every s in [0, n-m] with t[s..s+m-1] = p,
    overlaps included, ascending, 0-based).
  * occurrences_py: the same definition as a pure-Python double loop, for
    exhaustive checks on tiny inputs.
  * wscmp, wsmatch, wsblend: the word-size instructions of Section 3.1 written
    out from their definitions over alpha-character words, given as Python
    sequences of symbols.  They are pinned by the paper's worked examples
    (Section 3.1, w = 48, gamma = 4, alpha = 12).

Parity status: every function here is pinned (see tests/test_oracle.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epsm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(out_path: str = _LIB_PATH, src: str = _SRC) -> str:
    """Compile the C oracle with gcc (plain -O2, no vector intrinsics)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
           "-o", out_path, src]
    subprocess.run(cmd, check=True)
    return out_path


def load(path: str = _LIB_PATH):
    """Load a compiled oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    u8p = ctypes.c_void_p
    u64 = ctypes.c_uint64
    lib.oracle_range.argtypes = [u8p, u64, u8p, u64, u64, u64, ctypes.c_void_p, u64]
    lib.oracle_range.restype = u64
    lib.oracle_search.argtypes = [u8p, u64, u8p, u64, ctypes.c_void_p, u64]
    lib.oracle_search.restype = u64
    lib.oracle_count.argtypes = [u8p, u64, u8p, u64]
    lib.oracle_count.restype = u64
    lib.oracle_count_mt.argtypes = [u8p, u64, u8p, u64, ctypes.c_int]
    lib.oracle_count_mt.restype = u64
    lib.oracle_range_mt.argtypes = [u8p, u64, u8p, u64, u64, u64, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_range_mt.restype = u64
    return lib


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load(_LIB_PATH)
    return _lib


def _as_u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    a = np.asarray(x)
    if a.dtype != np.uint8:
        a = a.astype(np.uint8)
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


class Oracle:
    """Bound C oracle (the default instance uses oracle/liboracle.so)."""

    def __init__(self, lib=None):
        self._lib = lib

    @property
    def lib(self):
        return self._lib if self._lib is not None else _get()

    def count(self, text, pattern) -> int:
        t, p = _as_u8(text), _as_u8(pattern)
        return int(self.lib.oracle_count(_ptr(t), t.size, _ptr(p), p.size))

    def search(self, text, pattern, cap: int | None = None) -> tuple[np.ndarray, int]:
        """(first min(cap, count) positions, full count); cap=None means all."""
        t, p = _as_u8(text), _as_u8(pattern)
        if cap is None:
            cap = self.count(t, p)
        out = np.empty(max(cap, 1), dtype=np.int64)
        total = int(self.lib.oracle_search(_ptr(t), t.size, _ptr(p), p.size, out.ctypes.data, cap))
        return out[:min(cap, total)], total

    def positions(self, text, pattern) -> np.ndarray:
        return self.search(text, pattern)[0]

    def search_range(self, text, pattern, s_begin: int, s_end: int, cap: int) -> tuple[np.ndarray, int]:
        t, p = _as_u8(text), _as_u8(pattern)
        out = np.empty(max(cap, 1), dtype=np.int64)
        total = int(self.lib.oracle_range(_ptr(t), t.size, _ptr(p), p.size, s_begin, s_end,
                                          out.ctypes.data, cap))
        return out[:min(cap, total)], total

    def search_range_mt(self, text, pattern, s_begin: int, s_end: int, threads: int) -> np.ndarray:
        """Every occurrence starting in [s_begin, s_end), ascending, by `threads` threads."""
        t, p = _as_u8(text), _as_u8(pattern)
        hi = min(s_end, t.size - p.size + 1)
        out = np.empty(max(hi - s_begin, 1), dtype=np.int64)
        r = int(self.lib.oracle_range_mt(_ptr(t), t.size, _ptr(p), p.size, s_begin, s_end,
                                         out.ctypes.data, threads))
        if r == (1 << 64) - 1:
            raise RuntimeError("oracle_range_mt could not start its threads")
        return out[:r]

    def count_mt(self, text, pattern, threads: int) -> int:
        t, p = _as_u8(text), _as_u8(pattern)
        r = int(self.lib.oracle_count_mt(_ptr(t), t.size, _ptr(p), p.size, threads))
        if r == (1 << 64) - 1:
            raise RuntimeError("oracle_count_mt could not start its threads")
        return r


_default = Oracle()
count = _default.count
search = _default.search
positions = _default.positions
search_range = _default.search_range
count_mt = _default.count_mt
search_range_mt = _default.search_range_mt


# --------------------------------------------------------------------------
# pure-Python twin of the definition (tiny inputs only)


def occurrences_py(text: Sequence[int], pattern: Sequence[int]) -> list[int]:
    """Every s with text[s+j] == pattern[j] for 0 <= j < m, ascending."""
    n, m = len(text), len(pattern)
    if m == 0:
        raise ValueError("the problem requires m > 0")
    hits = []
    for s in range(0, n - m + 1):
        ok = True
        for j in range(m):
            if text[s + j] != pattern[j]:
                ok = False
                break
        if ok:
            hits.append(s)
    return hits


# --------------------------------------------------------------------------
# word-size instructions of Section 3.1, from their definitions.  A word is a
# sequence of alpha symbols a_0 .. a_{alpha-1}; a mask is returned as the list
# of bits r_0 .. r_{alpha-1} in the paper's left-to-right order.


def wscmp(a: Sequence[int], b: Sequence[int]) -> list[int]:
    """r_i = 1 iff a_i = b_i (word-size compare)."""
    if len(a) != len(b):
        raise ValueError("wscmp compares two words of the same length")
    return [1 if a[i] == b[i] else 0 for i in range(len(a))]


def wsmatch(a: Sequence[int], b: Sequence[int]) -> list[int]:
    """r_i = 1 iff a_{i+j} = b_j for j = 0..k-1; r_i = 0 for i > alpha-k."""
    alpha, k = len(a), len(b)
    if not 0 < k <= alpha:
        raise ValueError("wsmatch needs 0 < len(b) <= len(a)")
    r = [0] * alpha
    for i in range(alpha - k + 1):
        if all(a[i + j] == b[j] for j in range(k)):
            r[i] = 1
    return r


def wsblend(a: Sequence[int], b: Sequence[int]) -> list[int]:
    """r = a_{alpha/2} .. a_{alpha-1} b_0 .. b_{alpha/2-1} (word-size blend)."""
    alpha = len(a)
    if len(b) != alpha or alpha % 2:
        raise ValueError("wsblend takes two words of the same even length")
    h = alpha // 2
    return list(a[h:]) + list(b[:h])


def mask_set(r: Sequence[int]) -> list[int]:
    """The set {r} = { i : r_i = 1 } of Section 3.1, ascending."""
    return [i for i, bit in enumerate(r) if bit]

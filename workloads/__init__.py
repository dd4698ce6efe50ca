"""Seeded synthetic inputs for the packed string matching scan.

Texts, patterns, batches and query streams with the shapes of the paper's
experiments (Section 4: genome-, protein- and English-like texts, patterns cut
from the text) and of the benchmark configurations.  This module holds no
string-matching arithmetic: it only draws bytes and sizes.  Both the CPU
oracle and the GPU library consume what it produces; neither is imported here.

Text bytes come from a counter-based generator so that any sub-range of any
text can be produced independently, on the CPU or on a GPU, with identical
results: byte i of a text with key K is derived from splitmix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) of
counter floor(i/4), whose 64-bit output is cut into four 16-bit samples.  A
16-bit sample u is mapped to a symbol by
  * uniform over sigma codes:  code = (u * sigma) >> 16, then an alphabet table
  * Zipf(s=1) over 96 symbols: a 65536-entry table whose slot counts follow
    the Zipf law (probabilities quantised to multiples of 2^-16)
Pattern offsets, random patterns, text lengths and arrival times come from
numpy's PCG64 generator seeded with SEED_BASE + 1000*config + stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

SEED_BASE = 12096449

_MASK64 = (1 << 64) - 1


def _as_i64(x: int) -> int:
    """Reinterpret an unsigned 64-bit value as a signed int64 (torch has no u64)."""
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLDEN = _as_i64(0x9E3779B97F4A7C15)
_MIX1 = _as_i64(0xBF58476D1CE4E5B9)
_MIX2 = _as_i64(0x94D049BB133111EB)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 tensors (torch's >> is arithmetic)."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(counter: torch.Tensor, key: int) -> torch.Tensor:
    """splitmix64 output for state key + (counter+1)*golden; int64 bit patterns."""
    z = (counter + 1) * _GOLDEN + _as_i64(key)
    z = (z ^ _srl(z, 30)) * _MIX1
    z = (z ^ _srl(z, 27)) * _MIX2
    return z ^ _srl(z, 31)


def splitmix64_int(counter: int, key: int) -> int:
    """Pure-integer splitmix64, used to pin the tensor version."""
    z = (key + (counter + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def text_key(config: int, index: int) -> int:
    """Generator key of text `index` of a configuration (splitmix64 of the pair)."""
    return splitmix64_int(config * 1_000_003 + index, SEED_BASE)


def rng(config: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + stream))


# --------------------------------------------------------------------------
# symbol tables

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8).copy()

# 96 symbols: printable ASCII 0x20..0x7E plus newline, in an English-like
# frequency rank order (space, letters by typical English frequency, newline,
# common punctuation, then every remaining printable byte in ASCII order).
_EN_HEAD = " etaoinshrdlcumwfgypbvkjxqz\n.,'\"-ETAOINSHRDLCUMWFGYPBVKJXQZ0123456789"


def english_rank_order() -> np.ndarray:
    seen = []
    for ch in _EN_HEAD:
        b = ord(ch)
        if b not in seen:
            seen.append(b)
    for b in list(range(0x20, 0x7F)) + [0x0A]:
        if b not in seen:
            seen.append(b)
    assert len(seen) == 96, len(seen)
    return np.array(seen, dtype=np.uint8)


def zipf_table(n_symbols: int = 96, s: float = 1.0) -> np.ndarray:
    """65536-entry table: slot u holds the symbol whose Zipf CDF interval holds (u+.5)/65536."""
    ranks = np.arange(1, n_symbols + 1, dtype=np.float64)
    prob = ranks ** (-s)
    prob /= prob.sum()
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    mids = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    rank_idx = np.searchsorted(cdf, mids, side="right")
    rank_idx = np.minimum(rank_idx, n_symbols - 1)
    return english_rank_order()[rank_idx]


def uniform_table(alphabet: np.ndarray) -> np.ndarray:
    """65536-entry table for the uniform law: slot u -> alphabet[(u*sigma) >> 16]."""
    sigma = len(alphabet)
    u = np.arange(65536, dtype=np.int64)
    return np.asarray(alphabet, dtype=np.uint8)[(u * sigma) >> 16]


# --------------------------------------------------------------------------
# text specifications


@dataclass(frozen=True)
class TextSpec:
    """A synthetic text: `kind` in {"uniform", "zipf96", "periodic"}."""

    n: int
    kind: str
    key: int = 0
    sigma: int = 0              # uniform: alphabet size
    alphabet: bytes = b""       # uniform: explicit symbols (default codes 0..sigma-1)
    fill: int = 0x61            # periodic: the repeated byte

    def table(self) -> np.ndarray | None:
        if self.kind == "uniform":
            alpha = (np.frombuffer(self.alphabet, dtype=np.uint8) if self.alphabet
                     else np.arange(self.sigma, dtype=np.uint8))
            return uniform_table(alpha)
        if self.kind == "zipf96":
            return zipf_table()
        if self.kind == "periodic":
            return None
        raise ValueError(self.kind)


_TABLE_CACHE: dict = {}


def _table_tensor(spec: TextSpec, device) -> torch.Tensor:
    k = (spec.kind, spec.sigma, spec.alphabet, str(device))
    if k not in _TABLE_CACHE:
        _TABLE_CACHE[k] = torch.from_numpy(spec.table()).to(device)
    return _TABLE_CACHE[k]


def gen_bytes(spec: TextSpec, start: int = 0, length: int | None = None,
              device="cpu", chunk: int = 1 << 28, out: torch.Tensor | None = None) -> torch.Tensor:
    """Bytes [start, start+length) of the text as a uint8 tensor on `device`."""
    if length is None:
        length = spec.n - start
    if start < 0 or length < 0 or start + length > spec.n:
        raise ValueError("range outside the text")
    if out is None:
        out = torch.empty(length, dtype=torch.uint8, device=device)
    if length == 0:
        return out
    if spec.kind == "periodic":
        out.fill_(spec.fill)
        return out
    table = _table_tensor(spec, out.device)
    pos = 0
    while pos < length:
        take = min(chunk, length - pos)
        a = start + pos
        w0, w1 = a // 4, (a + take + 3) // 4
        ctr = torch.arange(w0, w1, dtype=torch.int64, device=out.device)
        z = splitmix64(ctr, spec.key)
        samples = torch.stack([_srl(z, 16 * j) & 0xFFFF for j in range(4)], dim=1).reshape(-1)
        lo = a - 4 * w0
        out[pos:pos + take] = table[samples[lo:lo + take]]
        pos += take
    return out


_NP_TABLE_CACHE: dict = {}


def _splitmix64_np(counter: np.ndarray, key: int) -> np.ndarray:
    """splitmix64 over a uint64 array (numpy's uint64 arithmetic wraps mod 2^64)."""
    with np.errstate(over="ignore"):
        z = (counter + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(key & _MASK64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _gen_small(spec: TextSpec, start: int, length: int) -> np.ndarray:
    """Bytes [start, start+length) computed with numpy (the same bytes as gen_bytes)."""
    if spec.kind == "periodic":
        return np.full(length, spec.fill, dtype=np.uint8)
    k = (spec.kind, spec.sigma, spec.alphabet)
    if k not in _NP_TABLE_CACHE:
        _NP_TABLE_CACHE[k] = spec.table()
    table = _NP_TABLE_CACHE[k]
    w0, w1 = start // 4, (start + length + 3) // 4
    if w1 - w0 <= 16:
        raw = b"".join(splitmix64_int(c, spec.key).to_bytes(8, "little") for c in range(w0, w1))
        z = np.frombuffer(raw, dtype="<u8")
    else:
        z = _splitmix64_np(np.arange(w0, w1, dtype=np.uint64), spec.key).astype("<u8")
    samples = z.view("<u2")  # sample j of a word is its bits 16j..16j+15
    lo = start - 4 * w0
    return table[samples[lo:lo + length]]


def gen_numpy(spec: TextSpec, start: int = 0, length: int | None = None) -> np.ndarray:
    if length is None:
        length = spec.n - start
    if 0 <= start and 0 <= length <= 65536 and start + length <= spec.n:
        return _gen_small(spec, start, length)
    return gen_bytes(spec, start, length, device="cpu").numpy()


# --------------------------------------------------------------------------
# patterns


def cut_pattern(spec: TextSpec, m: int, g: np.random.Generator) -> tuple[bytes, int]:
    """Pattern of length m cut from the text at a uniform offset in [0, n-m]."""
    off = int(g.integers(0, spec.n - m + 1))
    return bytes(gen_numpy(spec, off, m)), off


def random_pattern(m: int, alphabet: np.ndarray, g: np.random.Generator) -> bytes:
    return bytes(np.asarray(alphabet, dtype=np.uint8)[g.integers(0, len(alphabet), m)])


def alphabet_of(spec: TextSpec) -> np.ndarray:
    if spec.kind == "uniform":
        return (np.frombuffer(spec.alphabet, dtype=np.uint8) if spec.alphabet
                else np.arange(spec.sigma, dtype=np.uint8))
    if spec.kind == "zipf96":
        return english_rank_order()
    return np.array([spec.fill], dtype=np.uint8)


@dataclass
class PatternCase:
    pattern: bytes
    origin: str            # "cut" or "random" or "closed-form"
    offset: int = -1       # cut offset (a guaranteed occurrence)


# --------------------------------------------------------------------------
# benchmark configurations


def config1(n: int = 1 << 20) -> tuple[TextSpec, list[PatternCase]]:
    """1 MiB genome-like text (uniform over ACGT), 25 cut patterns for each m in {2,4,8,16}."""
    spec = TextSpec(n=n, kind="uniform", key=text_key(1, 0), sigma=4, alphabet=b"ACGT")
    g = rng(1, 1)
    cases = []
    for m in (2, 4, 8, 16):
        for _ in range(25):
            p, off = cut_pattern(spec, m, g)
            cases.append(PatternCase(p, "cut", off))
    return spec, cases


CONFIG2_SIGMAS = (2, 4, 20, 64, 128)
CONFIG2_MS = (1, 2, 4, 8, 12, 16, 24, 32)


def config2(sigma: int, n: int = 1 << 30) -> tuple[TextSpec, list[PatternCase]]:
    """1 GiB text uniform over codes 0..sigma-1; per m one cut and one random pattern."""
    spec = TextSpec(n=n, kind="uniform", key=text_key(2, sigma), sigma=sigma)
    g = rng(2, sigma)
    cases = []
    for m in CONFIG2_MS:
        p, off = cut_pattern(spec, m, g)
        cases.append(PatternCase(p, "cut", off))
        cases.append(PatternCase(random_pattern(m, alphabet_of(spec), g), "random"))
    return spec, cases


def config3(n: int = 1 << 32) -> tuple[TextSpec, list[PatternCase], TextSpec, list[PatternCase]]:
    """4 GiB Zipf(1) English-like text with cut patterns m=1..16, plus a^n with a^m."""
    spec = TextSpec(n=n, kind="zipf96", key=text_key(3, 0))
    g = rng(3, 1)
    cases = []
    for m in range(1, 17):
        p, off = cut_pattern(spec, m, g)
        cases.append(PatternCase(p, "cut", off))
    per = TextSpec(n=n, kind="periodic", fill=0x61)
    per_cases = [PatternCase(b"a" * m, "closed-form", 0) for m in range(1, 17)]
    return spec, cases, per, per_cases


@dataclass
class BatchText:
    spec: TextSpec
    patterns: list[bytes] = field(default_factory=list)


def config4(n_texts: int = 10_000, min_len: int = 1 << 10, max_len: int = 1 << 24,
            max_patterns: int = 64, max_m: int = 32, seed_stream: int = 1) -> list[BatchText]:
    """Batch: log-uniform text lengths, sigma 4 or 64, 1..64 patterns of m in [1, 32].

    Half of each text's patterns are cut from it, half are drawn at random.
    """
    g = rng(4, seed_stream)
    lo, hi = math.log(min_len), math.log(max_len)
    out = []
    for i in range(n_texts):
        L = int(math.floor(math.exp(g.uniform(lo, hi))))
        L = max(min_len, min(max_len, L))
        sigma = 4 if g.integers(0, 2) == 0 else 64
        spec = TextSpec(n=L, kind="uniform", key=text_key(4, i), sigma=sigma)
        n_pat = int(g.integers(1, max_patterns + 1))
        pats = []
        for j in range(n_pat):
            m = int(g.integers(1, min(max_m, L) + 1))
            if j % 2 == 0:
                pats.append(cut_pattern(spec, m, g)[0])
            else:
                pats.append(random_pattern(m, alphabet_of(spec), g))
        out.append(BatchText(spec, pats))
    return out


@dataclass
class Query:
    arrival: float          # seconds from the start of the stream
    text: int               # resident text index
    patterns: list[bytes]


def config5_texts(n_texts: int = 256, min_len: int = 1 << 20, max_len: int = 1 << 28,
                  sigma: int = 20) -> list[TextSpec]:
    """Resident serving texts: uniform over 20 codes, log-uniform lengths."""
    g = rng(5, 1)
    lo, hi = math.log(min_len), math.log(max_len)
    specs = []
    for i in range(n_texts):
        L = int(math.floor(math.exp(g.uniform(lo, hi))))
        L = max(min_len, min(max_len, L))
        specs.append(TextSpec(n=L, kind="uniform", key=text_key(5, i), sigma=sigma))
    return specs


def config5_queries(texts: list[TextSpec], n_queries: int, qps: float,
                    max_patterns: int = 256, min_m: int = 2, max_m: int = 32,
                    seed_stream: int = 2) -> list[Query]:
    """Poisson query stream: exponential gaps at rate qps; half cut, half random patterns."""
    g = rng(5, seed_stream)
    t = 0.0
    out = []
    for _ in range(n_queries):
        t += float(g.exponential(1.0 / qps))
        ti = int(g.integers(0, len(texts)))
        spec = texts[ti]
        n_pat = int(g.integers(1, max_patterns + 1))
        pats = []
        for j in range(n_pat):
            m = int(g.integers(min_m, max_m + 1))
            if j % 2 == 0:
                pats.append(cut_pattern(spec, m, g)[0])
            else:
                pats.append(random_pattern(m, alphabet_of(spec), g))
        out.append(Query(t, ti, pats))
    return out

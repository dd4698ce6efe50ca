"""GPU parity: positions and counts from the HIP kernels equal the CPU oracle.

Integer work, so the bar is bit-exact equality of the int64 position arrays
and of the counts.  Each case prints its parameters before touching the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TILE = 128 * 1024  # default workgroup tile (8 waves x 16 KiB)


@pytest.fixture(scope="module")
def epsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as mod
    mod.lib()
    return mod


def say(msg: str) -> None:
    print(msg, flush=True)


def to_gpu(arr: np.ndarray, offset: int = 0) -> torch.Tensor:
    """Device copy of arr starting `offset` bytes into a fresh allocation."""
    buf = torch.zeros(arr.size + offset + 1, dtype=torch.uint8, device="cuda")
    if arr.size:
        buf[offset:offset + arr.size] = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    return buf[offset:offset + arr.size]


def check(epsm, text: np.ndarray, pattern: bytes, flags: int = 0, offset: int = 0, label: str = ""):
    say(f"case {label} n={text.size} m={len(pattern)} flags={flags:#x} offset={offset}")
    t = to_gpu(text, offset)
    plan = epsm.Plan(pattern, flags)
    got = epsm.search(t, plan).cpu().numpy()
    exp = oracle.positions(text, pattern)
    assert got.dtype == np.int64
    assert np.array_equal(got, exp), (label, len(got), len(exp), got[:10], exp[:10])
    assert epsm.count(t, plan) == exp.size
    epsm.stream_check()
    return exp.size


def test_config1_all_patterns(epsm):
    """1 MiB ACGT text, 100 patterns cut from it (25 per m in {2,4,8,16})."""
    spec, cases = W.config1()
    text = W.gen_numpy(spec)
    t = to_gpu(text)
    for i, c in enumerate(cases):
        say(f"config1 pattern {i} m={len(c.pattern)} offset={c.offset}")
        got = epsm.search(t, c.pattern).cpu().numpy()
        exp = oracle.positions(text, c.pattern)
        assert np.array_equal(got, exp), i
        assert c.offset in set(exp.tolist())
    epsm.stream_check()


EDGE_NS = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 1023, 1024, 1025,
           TILE - 1, TILE, TILE + 1, 2 * TILE + 33, 3 * TILE + 7]


@pytest.mark.parametrize("m", list(range(1, 34)) + [40, 64, 100])
def test_edge_lengths_binary_text(epsm, m):
    """sigma = 2 text (many hits), n around lane/wave/tile boundaries, cut patterns."""
    rng = np.random.default_rng(1000 + m)
    for n in [x for x in EDGE_NS if x >= 1] + [m - 1, m, m + 1]:
        if n <= 0:
            continue
        text = rng.integers(0, 2, n).astype(np.uint8)
        if n >= m:
            # patterns cut at the very start and the very end of the text
            check(epsm, text, text[:m].tobytes(), label="start")
            check(epsm, text, text[n - m:].tobytes(), label="end")
        else:
            check(epsm, text, rng.integers(0, 2, m).astype(np.uint8).tobytes(), label="long")


def test_empty_text_and_pattern_longer_than_text(epsm):
    hits = torch.full((1,), 99, dtype=torch.int64, device="cuda")
    plan = epsm.Plan(b"abc")
    empty = torch.zeros(0, dtype=torch.uint8, device="cuda")
    say("case empty text")
    epsm.search_into(plan, empty, None, hits)
    assert int(hits.item()) == 0
    hits.fill_(99)
    say("case m > n")
    epsm.search_into(plan, torch.zeros(2, dtype=torch.uint8, device="cuda"), None, hits)
    assert int(hits.item()) == 0


@pytest.mark.parametrize("offset", range(16))
def test_unaligned_text_start(epsm, offset):
    rng = np.random.default_rng(offset)
    text = rng.integers(0, 3, 3 * TILE + 5).astype(np.uint8)
    for m in (1, 2, 3, 4, 5, 9, 15, 16, 17, 32, 33):
        check(epsm, text, text[:m].tobytes(), offset=offset, label="unaligned-start")
        check(epsm, text, text[-m:].tobytes(), offset=offset, label="unaligned-end")


@pytest.mark.parametrize("sigma", [1, 2, 4, 20, 64, 128, 256])
def test_alphabet_sizes(epsm, sigma):
    rng = np.random.default_rng(sigma)
    n = 5 * TILE + 77
    text = rng.integers(0, sigma, n).astype(np.uint8)
    for m in (1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12, 13, 15, 16, 17, 20, 24, 28, 31, 32, 33, 48):
        o = int(rng.integers(0, n - m + 1))
        check(epsm, text, text[o:o + m].tobytes(), label=f"sigma{sigma}-cut")
        check(epsm, text, rng.integers(0, sigma, m).astype(np.uint8).tobytes(),
              label=f"sigma{sigma}-random")


def test_zero_and_ff_bytes(epsm):
    rng = np.random.default_rng(7)
    n = 2 * TILE + 100
    text = np.where(rng.random(n) < 0.5, 0, 255).astype(np.uint8)
    text[rng.integers(0, n, 200)] = 0x7F
    for m in (1, 2, 3, 4, 7, 8, 12, 16, 19, 32):
        check(epsm, text, bytes([0] * m), label="zeros")
        check(epsm, text, bytes([255] * m), label="ffs")
        o = int(rng.integers(0, n - m))
        check(epsm, text, text[o:o + m].tobytes(), label="mixed")


@pytest.mark.parametrize("m", [15, 16, 17, 20, 24, 31, 32, 33, 40, 64])
def test_forced_variants_agree(epsm, m):
    rng = np.random.default_rng(m)
    text = rng.integers(0, 4, 3 * TILE + 11).astype(np.uint8)
    o = int(rng.integers(0, text.size - m))
    p = text[o:o + m].tobytes()
    check(epsm, text, p, epsm.PLAN_FORCE_DIRECT, label="force-direct")
    check(epsm, text, p, epsm.PLAN_FORCE_FINGERPRINT, label="force-fingerprint")
    check(epsm, text, p, epsm.PLAN_FORCE_FINGERPRINT | epsm.PLAN_COLLIDE, label="collide")


@pytest.mark.parametrize("m", [5, 6, 7, 8, 9, 11, 12, 13, 15])
@pytest.mark.parametrize("sigma", [1, 2, 4, 256])
def test_prefix_widths_agree(epsm, m, sigma):
    """The direct filter's 64-bit prefix (default for m >= 5) and its 4-byte
    prefix (EPSM_PLAN_PREFIX4) both equal the oracle: dense candidates on
    small alphabets, tiles with a ragged tail, patterns cut at the ends."""
    rng = np.random.default_rng(1000 * sigma + m)
    n = 2 * TILE + 1001
    text = rng.integers(0, sigma, n).astype(np.uint8)
    assert epsm.Plan(b"x" * m, epsm.PLAN_HOST_ONLY).info()["variant"] == epsm.VARIANT_DIRECT
    for o in (0, n - m, int(rng.integers(0, n - m + 1))):
        p = text[o:o + m].tobytes()
        check(epsm, text, p, label=f"prefix8 sigma {sigma}")
        check(epsm, text, p, epsm.PLAN_PREFIX4, label=f"prefix4 sigma {sigma}")
    p = rng.integers(0, max(sigma, 2), m).astype(np.uint8).tobytes()
    check(epsm, text, p, label=f"prefix8 random sigma {sigma}")


@pytest.mark.parametrize("bits", [8, 9, 12, 14])
def test_hash_width_does_not_change_output(epsm, bits):
    rng = np.random.default_rng(bits)
    text = rng.integers(0, 2, 2 * TILE + 3).astype(np.uint8)
    for m in (16, 23, 32):
        o = int(rng.integers(0, text.size - m))
        check(epsm, text, text[o:o + m].tobytes(), epsm.PLAN_HASH_BITS(bits), label=f"k{bits}")


def test_periodic_patterns_collide_in_one_bucket(epsm):
    text = np.frombuffer(b"ab" * (3 * TILE), dtype=np.uint8)
    for m in (16, 17, 20, 32):
        check(epsm, text, (b"ab" * 20)[:m], label="period2")
        check(epsm, text, (b"ba" * 20)[:m], label="period2-shift")


@pytest.mark.parametrize("m", [1, 2, 3, 4, 8, 15, 16, 31, 32, 33])
def test_unary_text_closed_form(epsm, m):
    """a^n with a^m: positions 0..n-m exactly (checked against the closed form)."""
    n = 2 * 1024 * 1024 + 13
    say(f"case unary n={n} m={m}")
    t = torch.full((n,), 0x61, dtype=torch.uint8, device="cuda")
    got = epsm.search(t, b"a" * m)
    assert got.numel() == n - m + 1
    assert torch.equal(got, torch.arange(n - m + 1, dtype=torch.int64, device="cuda"))
    epsm.stream_check()


def test_truncated_output_is_prefix_and_count_is_full(epsm):
    n = 100_000
    t = torch.full((n,), 0x61, dtype=torch.uint8, device="cuda")
    plan = epsm.Plan(b"aa")
    for cap in (0, 1, 17, 5000, n - 1 - 1, n - 1, n + 10):
        say(f"case truncation cap={cap}")
        out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device="cuda")
        hits = torch.zeros(1, dtype=torch.int64, device="cuda")
        epsm.search_into(plan, t, out[:cap] if cap else None, hits)
        assert int(hits.item()) == n - 1
        k = min(cap, n - 1)
        assert torch.equal(out[:k].cpu(), torch.arange(k, dtype=torch.int64))
        if cap > n - 1:
            assert bool((out[n - 1:cap] == -7).all())


def test_repeated_runs_are_identical(epsm):
    rng = np.random.default_rng(3)
    text = rng.integers(0, 2, 7 * TILE + 9).astype(np.uint8)
    t = to_gpu(text)
    for p in (b"\x00", b"\x01\x00\x01", bytes(text[100:117])):
        say(f"case determinism m={len(p)}")
        a = epsm.search(t, p)
        b = epsm.search(t, p)
        assert torch.equal(a, b)


def test_positions_are_sound_and_increasing_random(epsm):
    """Randomised sizes/alphabets/patterns; full equality with the oracle."""
    rng = np.random.default_rng(12345)
    for i in range(60):
        sigma = int(rng.choice([1, 2, 3, 4, 8, 20, 64, 256]))
        n = int(rng.integers(1, 200_000))
        m = int(rng.integers(1, 40))
        text = rng.integers(0, sigma, n).astype(np.uint8)
        if n >= m and rng.random() < 0.6:
            o = int(rng.integers(0, n - m + 1))
            p = text[o:o + m].tobytes()
        else:
            p = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
        check(epsm, text, p, offset=int(rng.integers(0, 16)), label=f"random{i}")


def _tiles():
    import paper_1209_6449_amd as mod
    try:
        return mod.tile_configs()
    except Exception:  # library missing: the fixture reports it
        return [(8, 16)]


def force(epsm, tile, strategy):
    """Every search (all classes) on `tile` with write strategy `strategy`."""
    epsm.set_tune_table([(c, 0, (1 << 64) - 1, *tile, strategy) for c in range(epsm.N_CLASSES)]
                        + [(c, 1, (1 << 64) - 1, *tile, 0) for c in range(epsm.N_CLASSES)])


@pytest.mark.parametrize("strategy", [1, 2], ids=["single_pass", "two_phase"])
@pytest.mark.parametrize("tile", _tiles())
def test_every_built_tile_matches_oracle(epsm, tile, strategy):
    """Each built workgroup tile and write strategy, at lengths around its own
    tile size, with dense (sigma 2: hit masks parked) and sparse (sigma 64:
    offset lists parked) texts, on all three kernel classes."""
    w, p = tile
    tb = w * p * 1024
    force(epsm, tile, strategy)
    try:
        rng = np.random.default_rng(w * 100 + p)
        for n in (tb - 1, tb, tb + 1, 2 * tb + 977, 9 * tb + 13):
            for sigma in (2, 64):
                text = rng.integers(0, sigma, n).astype(np.uint8)
                for m in (1, 3, 4, 6, 9, 13, 16, 33):
                    off = int(rng.integers(0, n - m + 1))
                    check(epsm, text, text[off:off + m].tobytes(),
                          label=f"tile {w}x{p} strategy {strategy} sigma {sigma}")
    finally:
        epsm.set_tune_table([])


@pytest.mark.parametrize("strategy", [1, 2], ids=["single_pass", "two_phase"])
def test_write_strategies_many_groups(epsm, strategy):
    """64 KiB tiles over 9 MiB + a ragged tail: several 64-tile count groups
    and 8-tile expand workgroups; mixed densities along the text (a dense
    run, a sparse run), unaligned start, truncated output."""
    force(epsm, (8, 8), strategy)
    try:
        n = 9 * (1 << 20) + 4097
        rng = np.random.default_rng(77)
        text = rng.integers(0, 64, n).astype(np.uint8)
        text[(3 << 20):(3 << 20) + 300_000] = rng.integers(0, 2, 300_000)  # dense stretch
        for m, offset in ((1, 0), (2, 5), (5, 11), (17, 3)):
            check(epsm, text, bytes(text[(3 << 20) + 1000:(3 << 20) + 1000 + m]), offset=offset,
                  label=f"groups strategy {strategy}")
        t = to_gpu(text, 7)
        p = bytes(text[(3 << 20) + 50:(3 << 20) + 51])
        exp = oracle.positions(text, p)
        for cap in (0, 1, exp.size // 3, exp.size - 1):
            out = torch.full((cap + 4,), -1, dtype=torch.int64, device="cuda")
            hits = torch.zeros(1, dtype=torch.int64, device="cuda")
            plan = epsm.Plan(p)
            epsm.search_into(plan, t, out[:cap], hits)
            torch.cuda.synchronize()
            assert int(hits.item()) == exp.size
            got = out.cpu().numpy()
            assert np.array_equal(got[:cap], exp[:cap]) and (got[cap:] == -1).all(), cap
        epsm.stream_check()
    finally:
        epsm.set_tune_table([])


def test_unary_text_two_phase_closed_form(epsm):
    """a^n with a^m under the two-phase write: every tile parks masks."""
    force(epsm, (8, 16), 2)
    try:
        n = 5 * (1 << 20) + 3
        t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
        for m in (1, 7, 16, 31):
            say(f"unary two-phase m={m}")
            got = epsm.search(t, b"a" * m)
            assert got.numel() == n - m + 1
            assert torch.equal(got, torch.arange(n - m + 1, dtype=torch.int64, device="cuda"))
        epsm.stream_check()
    finally:
        epsm.set_tune_table([])


@pytest.mark.parametrize("strategy", [1, 2], ids=["single_pass", "two_phase"])
def test_unary_text_beyond_2_32_positions(epsm, strategy):
    """a^n with n > 2^32 on 64 KiB tiles: 65 539 tiles (several chunks of the
    per-tile count sums and offsets), more than 2^32 positions (34 GB of
    int64) and counts above 2^32; positions checked against i in slices."""
    force(epsm, (8, 8), strategy)
    try:
        n = (1 << 32) + 3 * 65536 + 5
        t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
        for m in (1, 6):
            say(f"unary beyond 2^32 strategy {strategy} n={n} m={m}")
            assert epsm.count(t, b"a" * m) == n - m + 1
            got = epsm.search(t, b"a" * m)
            assert got.numel() == n - m + 1
            step = 1 << 28
            for s in range(0, got.numel(), step):
                e = min(s + step, got.numel())
                assert torch.equal(got[s:e], torch.arange(s, e, dtype=torch.int64, device="cuda")), s
            del got
        epsm.stream_check()
    finally:
        epsm.set_tune_table([])


def planted_text(rng, n, sigma, pattern, spots):
    text = rng.integers(0, sigma, n).astype(np.uint8)
    for o in spots:
        if 0 <= o <= n - len(pattern):
            text[o:o + len(pattern)] = np.frombuffer(pattern, dtype=np.uint8)
    return text


@pytest.mark.parametrize("m", [263, 300, 519, 1031, 2055, 4096])
def test_strided_filter_matches_oracle(epsm, m):
    """Long patterns (strided filter) against the oracle and against the
    per-block filter: planted copies at both text ends, near block boundaries,
    overlapping; sparse and binary texts; unaligned starts; counts."""
    rng = np.random.default_rng(m)
    for sigma in (2, 4, 64):
        pattern = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
        for n in (m, m + 1, 3 * m + 17, 200_000 + m):
            spots = [0, n - m, n // 2, (n // 2) + 1, (n // 3) & ~255, ((n // 3) & ~255) - 1]
            text = planted_text(rng, n, sigma, pattern, spots)
            for offset in (0, 5):
                plan = epsm.Plan(pattern)
                assert plan.info()["variant"] == epsm.VARIANT_STRIDE
                say(f"stride m={m} sigma={sigma} n={n} offset={offset}")
                t = to_gpu(text, offset)
                got = epsm.search(t, plan).cpu().numpy()
                exp = oracle.positions(text, pattern)
                assert np.array_equal(got, exp), (m, sigma, n, offset, got[:5], exp[:5])
                assert epsm.count(t, plan) == exp.size
                base = epsm.search(t, epsm.Plan(pattern, epsm.PLAN_NO_STRIDE)).cpu().numpy()
                assert np.array_equal(base, exp)
    epsm.stream_check()


@pytest.mark.parametrize("m", [263, 520, 2055])
def test_strided_filter_periodic_text(epsm, m):
    """a^n with a^m: every offset of the table is a candidate of every block;
    n - m + 1 hits (closed form), truncated output is the prefix."""
    n = 65_536 + 9
    t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
    plan = epsm.Plan(b"a" * m)
    assert plan.info()["variant"] == epsm.VARIANT_STRIDE
    say(f"stride periodic m={m}")
    got = epsm.search(t, plan)
    assert got.numel() == n - m + 1
    assert torch.equal(got, torch.arange(n - m + 1, dtype=torch.int64, device="cuda"))
    for cap in (0, 1, 1000):
        out = torch.full((cap + 2,), -3, dtype=torch.int64, device="cuda")
        hits = torch.zeros(1, dtype=torch.int64, device="cuda")
        epsm.search_into(plan, t, out[:cap], hits)
        assert int(hits.item()) == n - m + 1
        assert torch.equal(out[:cap].cpu(), torch.arange(cap, dtype=torch.int64))
        assert bool((out[cap:] == -3).all())
    epsm.stream_check()


@pytest.mark.parametrize("m", [39, 40, 71, 72, 135, 136, 200, 262])
def test_small_stride_rows_match_oracle(epsm, m):
    """A variant-table row asking for the strided filter below m = 263
    (S = 32, 64, 128 between inspected blocks): planted copies at the ends,
    near block boundaries and overlapping, sparse and binary texts,
    unaligned starts; and a^n with a^m (closed form)."""
    epsm.set_variant_table([(39, 262, 0, 256, epsm.VARIANT_STRIDE, 0)])
    try:
        rng = np.random.default_rng(1000 + m)
        for sigma in (2, 4, 64):
            pattern = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
            plan = epsm.Plan(pattern)
            info = plan.info()
            S = 1 << (m - 7).bit_length() - 1
            assert (info["variant"], info["stride"]) == (epsm.VARIANT_STRIDE, min(S, 2048))
            for n in (m, 3 * m + 17, 100_000 + m):
                spots = [0, n - m, n // 2, n // 2 + 1, (n // 3) & ~31, ((n // 3) & ~31) - 1]
                text = planted_text(rng, n, sigma, pattern, spots)
                for offset in (0, 7):
                    say(f"small stride m={m} S={info['stride']} sigma={sigma} n={n} offset={offset}")
                    t = to_gpu(text, offset)
                    got = epsm.search(t, plan).cpu().numpy()
                    exp = oracle.positions(text, pattern)
                    assert np.array_equal(got, exp), (m, sigma, n, offset, got[:5], exp[:5])
                    assert epsm.count(t, plan) == exp.size
        n = 50_000 + 3
        t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
        got = epsm.search(t, epsm.Plan(b"a" * m))
        assert torch.equal(got, torch.arange(n - m + 1, dtype=torch.int64, device="cuda"))
        epsm.stream_check()
    finally:
        epsm.set_variant_table([])


@pytest.mark.parametrize("shift", [0, 8, 4, 1])
def test_output_pointer_alignment(epsm, shift):
    """Positions written to an output that starts `shift` bytes past a
    16-byte boundary (16-byte pair stores, the single entry before the first
    boundary, and the unaligned fallback), dense single-pass and sparse
    two-phase outputs, exact and truncated capacities."""
    import ctypes
    L = epsm.lib()
    dense = torch.full((3 * TILE + 5,), ord("a"), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(7)
    sparse_h = rng.integers(0, 64, 40 * TILE + 3).astype(np.uint8)
    sparse = torch.from_numpy(sparse_h).cuda()
    for t, pat in ((dense, b"aa"), (sparse, bytes(sparse_h[5000:5002]))):
        host = t.cpu().numpy()
        exp = oracle.positions(host, pat)
        plan = epsm.Plan(pat)
        for cap in (exp.size, exp.size - 1, 3, 1):
            say(f"output alignment shift={shift} n={t.numel()} hits={exp.size} cap={cap}")
            buf = torch.full((cap * 8 + 32,), 0xEE, dtype=torch.uint8, device="cuda")
            base = (buf.data_ptr() + 15) // 16 * 16 + shift
            hits = torch.zeros(1, dtype=torch.int64, device="cuda")
            st = L.epsm_search(plan.handle, t.data_ptr(), t.numel(), ctypes.c_void_p(base), cap,
                               hits.data_ptr(), None)
            assert st == 0
            epsm.stream_check()
            assert int(hits.item()) == exp.size
            raw = buf.cpu().numpy()
            start = base - buf.data_ptr()
            got = raw[start:start + 8 * cap].view(np.int64)
            assert np.array_equal(got, exp[:cap]), (shift, cap)
            assert (raw[:start] == 0xEE).all() and (raw[start + 8 * cap:] == 0xEE).all()

"""Packed 2-bit DNA texts: packing is bit-exact, and every search over a
packed text equals the oracle run on the unpacked codes (positions count
symbols).  Integer work: bit-exact equality."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

TILE = 128 * 1024  # default tile, in coordinates (symbols for packed texts)


@pytest.fixture(scope="module")
def epsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as mod
    mod.lib()
    return mod


def say(msg):
    print(msg, flush=True)


def pack_np(codes: np.ndarray) -> np.ndarray:
    """Reference 2-bit packing: symbol i at bits 2*(i%4) of byte i//4."""
    n = codes.size
    out = np.zeros((n + 3) // 4, dtype=np.uint8)
    for r in range(4):
        part = codes[r::4].astype(np.uint8) & 3
        out[:part.size] |= part << (2 * r)
    return out


def packed_on_gpu(epsm, codes: np.ndarray, offset: int = 0) -> torch.Tensor:
    """Pack on the device into a buffer whose text starts `offset` bytes in."""
    n = codes.size
    c = torch.from_numpy(np.ascontiguousarray(codes)).cuda() if n else torch.zeros(0, dtype=torch.uint8,
                                                                                     device="cuda")
    buf = torch.full(((n + 3) // 4 + offset + 1,), 0xA5, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + (n + 3) // 4]
    if n:
        epsm.lib().epsm_pack_dna(c.data_ptr(), n, view.data_ptr(), None)
    return view


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 15, 16, 17, 63, 1000, (1 << 20) + 3])
def test_pack_matches_reference(epsm, n):
    rng = np.random.default_rng(n)
    codes = rng.integers(0, 256, n).astype(np.uint8)  # only the low two bits count
    say(f"pack n={n}")
    got = epsm.pack_dna(torch.from_numpy(codes).cuda()).cpu().numpy() if n else np.zeros(0, np.uint8)
    assert np.array_equal(got, pack_np(codes))


def check(epsm, codes, pattern, offset=0, label=""):
    say(f"dna {label} n={codes.size} m={len(pattern)} offset={offset}")
    packed = packed_on_gpu(epsm, codes, offset)
    plan = epsm.Plan(pattern, epsm.PLAN_DNA)
    got = epsm.search_dna(packed, codes.size, plan).cpu().numpy()
    exp = oracle.positions(codes, pattern)
    assert np.array_equal(got, exp), (label, got[:8], exp[:8], got.size, exp.size)
    assert epsm.count_dna(packed, codes.size, plan) == exp.size
    epsm.stream_check()
    return exp.size


MS = [1, 2, 5, 7, 8, 11, 15, 16, 17, 31, 32, 33, 47, 48, 49, 64, 100]


@pytest.mark.parametrize("m", MS)
def test_edges_and_sigmas(epsm, m):
    rng = np.random.default_rng(500 + m)
    for n in (m, m + 1, 1023, 1024, 1025, TILE - 1, TILE + 17, 3 * TILE + 5):
        if n < m:
            continue
        for sigma in (2, 4):
            codes = rng.integers(0, sigma, n).astype(np.uint8)
            for o in (0, n - m, int(rng.integers(0, n - m + 1))):
                check(epsm, codes, codes[o:o + m].tobytes(), label=f"sigma {sigma} cut {o}")
        codes = rng.integers(0, 4, n).astype(np.uint8)
        check(epsm, codes, rng.integers(0, 4, m).astype(np.uint8).tobytes(), label="random")


@pytest.mark.parametrize("offset", [0, 1, 3, 7, 15])
def test_unaligned_packed_start(epsm, offset):
    rng = np.random.default_rng(offset)
    codes = rng.integers(0, 4, 300_001).astype(np.uint8)
    for m in (3, 16, 21, 40):
        check(epsm, codes, codes[77:77 + m].tobytes(), offset=offset, label="unaligned")


@pytest.mark.parametrize("strategy", [1, 2], ids=["single_pass", "two_phase"])
def test_dna_write_strategies(epsm, strategy):
    """Both write strategies on a multi-tile text, dense (unary, binary) and
    sparse outputs."""
    epsm.set_tune_table([(epsm.CLASS_DNA, 0, (1 << 64) - 1, 8, 8, strategy)])
    try:
        rng = np.random.default_rng(strategy)
        n = 9 * (1 << 20) + 11
        for sigma, m in ((1, 1), (1, 20), (2, 6), (4, 12), (4, 30)):
            codes = rng.integers(0, sigma, n).astype(np.uint8)
            hits = check(epsm, codes, codes[1000:1000 + m].tobytes(), label=f"strategy {strategy}")
            if sigma == 1:
                assert hits == n - m + 1  # closed form of a^n with a^m
    finally:
        epsm.set_tune_table([])


def test_truncated_dna_output(epsm):
    codes = np.zeros(100_000, dtype=np.uint8)
    packed = packed_on_gpu(epsm, codes)
    plan = epsm.Plan(b"\x00\x00", epsm.PLAN_DNA)
    for cap in (0, 1, 33, 99_998, 99_999, 100_010):
        out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device="cuda")
        hits = torch.zeros(1, dtype=torch.int64, device="cuda")
        epsm.search_dna_into(plan, packed, codes.size, out[:cap] if cap else None, hits)
        assert int(hits.item()) == 99_999
        k = min(cap, 99_999)
        assert torch.equal(out[:k].cpu(), torch.arange(k, dtype=torch.int64))


def test_dna_plan_and_byte_search_do_not_mix(epsm):
    t = torch.zeros(64, dtype=torch.uint8, device="cuda")
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(epsm.EpsmError):
        epsm.count_into(epsm.Plan(b"\x01", epsm.PLAN_DNA), t, hits)
    with pytest.raises(epsm.EpsmError):
        epsm.count_dna_into(epsm.Plan(b"\x01"), t, 64, hits)
    with pytest.raises(epsm.EpsmError):
        epsm.search_batch([t], [(0, epsm.Plan(b"\x01", epsm.PLAN_DNA))])


@pytest.mark.parametrize("m", [3, 6, 7, 8, 12, 15, 16, 20, 33, 49])
def test_wide_write_path_planted(epsm, m):
    """Sparse outputs take the wide-lane write pass (count pass, tile offsets,
    then only the tiles with hits): 2^25 + 12345 symbols (129 tiles of 2^18),
    the pattern planted at both ends, around tile and piece boundaries, at
    lane starts of one piece, and back to back over 20000 symbols of one
    wave's span (more hits than its slot parks: that wave re-reads its span);
    unaligned packed starts; truncated output keeps the ascending prefix.
    Below m = 6 the text avoids symbol 3 and the pattern holds it, so only
    the planted copies occur and the output stays sparse."""
    rng = np.random.default_rng(7000 + m)
    n = (1 << 25) + 12345
    codes = rng.integers(0, 4 if m >= 6 else 3, n).astype(np.uint8)
    pattern = rng.integers(0, 4, m).astype(np.uint8)
    if m < 6:
        pattern[m // 2] = 3
    tile, piece = 1 << 18, 4096
    spots = [0, n - m, 1, 63, 64, 65, piece - 1, piece, 5 * piece + 17]
    spots += [k * tile + d for k in (1, 2, 63, 127) for d in (-m, -1, 0, 1, 30)]
    spots += [3 * tile + 4096 + 64 * lane for lane in range(0, 64, 9)]
    for o in spots:
        if 0 <= o <= n - m:
            codes[o:o + m] = pattern
    # a dense stretch inside one wave's span (8 pieces of 4096 symbols): more
    # hits than the wave's slot parks, so that wave re-reads its span
    dense0 = 5 * tile + 2 * 32768 + 100
    for o in range(dense0, dense0 + 20000 - m, m):
        codes[o:o + m] = pattern
    for offset in (0, 5):
        check(epsm, codes, pattern.tobytes(), offset=offset, label="wide planted")
    exp = oracle.positions(codes, pattern.tobytes())
    packed = packed_on_gpu(epsm, codes, 3)
    plan = epsm.Plan(pattern.tobytes(), epsm.PLAN_DNA)
    for cap in (1, exp.size // 2):
        out = torch.full((cap + 2,), -7, dtype=torch.int64, device="cuda")
        nh = torch.zeros(1, dtype=torch.int64, device="cuda")
        epsm.search_dna_into(plan, packed, n, out[:cap], nh)
        assert int(nh.item()) == exp.size
        got = out.cpu().numpy()
        assert np.array_equal(got[:cap], exp[:cap]) and (got[cap:] == -7).all(), cap


def test_wide_write_dense_pieces(epsm):
    """Through the wide-lane write (sparse on average over 2^25 symbols), a
    run of 20000 zero symbols in a text over {1, 2, 3}
    gives pieces where every start hits for the pattern 00: those pieces
    hold more hits than the wave's LDS stage and are written lane by lane,
    between staged pieces at the run's ends; unaligned packed start and a
    truncated output too."""
    rng = np.random.default_rng(9100)
    n = (1 << 25) + 999
    codes = rng.integers(1, 4, n).astype(np.uint8)
    run0 = 7 * (1 << 18) + 3 * 32768 + 1234  # inside one wave's span and the next
    codes[run0:run0 + 20000] = 0
    codes[5:7] = 0
    codes[n - 2:] = 0
    pattern = bytes([0, 0])
    for offset in (0, 9):
        assert check(epsm, codes, pattern, offset=offset, label="wide dense pieces") == 20001
    exp = oracle.positions(codes, pattern)
    packed = packed_on_gpu(epsm, codes, 0)
    plan = epsm.Plan(pattern, epsm.PLAN_DNA)
    cap = 10007
    out = torch.full((cap + 2,), -7, dtype=torch.int64, device="cuda")
    nh = torch.zeros(1, dtype=torch.int64, device="cuda")
    epsm.search_dna_into(plan, packed, n, out[:cap], nh)
    assert int(nh.item()) == exp.size
    got = out.cpu().numpy()
    assert np.array_equal(got[:cap], exp[:cap]) and (got[cap:] == -7).all()
    epsm.stream_check()

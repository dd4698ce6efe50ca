"""epsm_search_noalloc (static device scratch, no allocation) against epsm_search.

Each case runs two no-allocation calls in a row on one stream, the second on
a smaller input, and compares each with epsm_search on the same input
element by element (positions and full count): the scratch keeps the first
call's contents, so the second shows that nothing stale is read.  Cases cover
the two-phase layout that fits the scratch, the fall-back to the single pass
when it does not, dense single-pass output, counts only, truncated output,
fingerprint and strided plans, a forced give-up of a bounded wait, and the
size limit (a text whose single-pass scratch exceeds the array is rejected
before any launch, and the same text at the default tile is searched).
"""
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
    mod.set_tune_table([])
    return mod


def say(msg: str) -> None:
    print(msg, flush=True)


def gpu_text(n, sigma, seed):
    spec = W.TextSpec(n=n, kind="uniform", key=W.text_key(91, seed), sigma=sigma)
    return W.gen_bytes(spec, device="cuda")


def both(epsm, plan, t, cap):
    """(positions, count) from epsm_search and from epsm_search_noalloc."""
    ref_out = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda")
    ref_hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    epsm.search_into(plan, t, ref_out[:cap] if cap else None, ref_hits)
    out = torch.full((max(cap, 1),), -2, dtype=torch.int64, device="cuda")
    hits = torch.full((1,), -3, dtype=torch.int64, device="cuda")
    epsm.search_noalloc_into(plan, t, out[:cap] if cap else None, hits)
    epsm.stream_check()
    return ref_out[:cap], int(ref_hits.item()), out[:cap], int(hits.item())


def two_calls(epsm, label, plan, big, small, cap_big=None, cap_small=None):
    for name, t, cap in (("first", big, cap_big), ("second (smaller)", small, cap_small)):
        if cap is None:
            cap = epsm.count(t, plan)
        say(f"noalloc {label}: {name} call n={t.numel()} m={plan.m} cap={cap}")
        ref, ref_n, got, got_n = both(epsm, plan, t, cap)
        assert got_n == ref_n, (label, name, got_n, ref_n)
        assert torch.equal(got, ref), (label, name)
        k = min(cap, ref_n)
        assert k == 0 or int(got[k - 1].item()) >= 0


def test_sparse_two_phase_fallback_then_fitting(epsm):
    """64 MiB sparse: epsm_search writes in two phases (about 8 MiB of slots,
    more than the scratch), the no-allocation call falls back to the single
    pass; then a 4 MiB text whose two-phase layout fits the scratch."""
    big = gpu_text(64 * (1 << 20) + 77, 64, 1)
    small = gpu_text(4 * (1 << 20) + 5, 64, 2)
    pat = bytes(big[123_456:123_460].cpu().numpy())
    two_calls(epsm, "sparse m=4", epsm.Plan(pat), big, small)
    pat2 = bytes(big[9_000_001:9_000_003].cpu().numpy())
    two_calls(epsm, "sparse m=2", epsm.Plan(pat2), big, small)


def test_dense_single_pass(epsm):
    """a^n with a^m: every start hits (single pass with look-back)."""
    big = torch.full((9 * (1 << 20) + 3,), ord("a"), dtype=torch.uint8, device="cuda")
    small = torch.full((3 * TILE + 1,), ord("a"), dtype=torch.uint8, device="cuda")
    for m in (1, 9, 16):
        plan = epsm.Plan(b"a" * m)
        two_calls(epsm, f"dense m={m}", plan, big, small)
    ref = torch.arange(big.numel(), dtype=torch.int64, device="cuda")
    out = torch.empty(big.numel(), dtype=torch.int64, device="cuda")
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    epsm.search_noalloc_into(epsm.Plan(b"a"), big, out, hits)
    epsm.stream_check()
    assert int(hits.item()) == big.numel() and torch.equal(out, ref)


def test_count_only_and_truncated(epsm):
    big = gpu_text(20 * TILE + 9, 4, 3)
    small = gpu_text(2 * TILE + 1, 4, 4)
    plan = epsm.Plan(bytes(big[5000:5003].cpu().numpy()))
    two_calls(epsm, "count only", plan, big, small, cap_big=0, cap_small=0)
    two_calls(epsm, "truncated", plan, big, small, cap_big=1000, cap_small=17)


def test_fingerprint_and_strided_plans(epsm):
    big = gpu_text(48 * (1 << 20) + 11, 4, 5)
    small = gpu_text(1 << 20, 4, 6)
    for lo, m in ((777_777, 20), (31_000_000, 32), (2_000_000, 300)):
        plan = epsm.Plan(bytes(big[lo:lo + m].cpu().numpy()))
        two_calls(epsm, f"m={m} variant={plan.info()['variant']}", plan, big, small)


def test_matches_oracle_on_host_text(epsm):
    """The no-allocation path against the oracle directly (not only against epsm_search)."""
    rng = np.random.default_rng(7)
    for n, sigma, m in ((5 * TILE + 3, 2, 7), (40 * TILE + 1, 20, 3), (777, 4, 2)):
        text = rng.integers(0, sigma, n).astype(np.uint8)
        pat = text[n // 3:n // 3 + m].tobytes()
        exp = oracle.positions(text, pat)
        say(f"noalloc vs oracle n={n} sigma={sigma} m={m} hits={exp.size}")
        t = torch.from_numpy(text).cuda()
        out = torch.full((max(exp.size, 1),), -1, dtype=torch.int64, device="cuda")
        hits = torch.zeros(1, dtype=torch.int64, device="cuda")
        epsm.search_noalloc_into(epsm.Plan(pat), t, out[:exp.size], hits)
        epsm.stream_check()
        assert int(hits.item()) == exp.size
        assert np.array_equal(out[:exp.size].cpu().numpy(), exp)


def test_forced_giveup_surfaces(epsm):
    """A give-up of the single pass's bounded wait (forced from the host;
    every kernel exits) is reported by the next stream check."""
    t = torch.full((3 * TILE,), ord("a"), dtype=torch.uint8, device="cuda")
    plan = epsm.Plan(b"aa")
    out = torch.empty(t.numel(), dtype=torch.int64, device="cuda")
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    epsm.debug_force_giveup(True)
    try:
        epsm.search_noalloc_into(plan, t, out, hits)
        with pytest.raises(epsm.EpsmError):
            epsm.stream_check()
    finally:
        epsm.debug_force_giveup(False)
    epsm.stream_check()  # reported once, then cleared
    epsm.search_noalloc_into(plan, t, out, hits)
    epsm.stream_check()
    assert int(hits.item()) == t.numel() - 1


def test_size_limit(epsm):
    """64 GiB + 128 KiB of a: at 64 KiB tiles the single pass needs one
    status word per tile, 8 MiB + 24 bytes, more than the scratch: rejected
    before any launch.  At the default 128 KiB tile (half the words) the same
    text is searched for its count."""
    torch.cuda.empty_cache()
    n = (64 << 30) + 2 * 65536
    t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
    hits = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    plan = epsm.Plan(b"a")
    epsm.set_tile_config(4, 16)
    try:
        say(f"noalloc size limit: n={n} at 64 KiB tiles (expect EPSM_EUNSUPPORTED)")
        with pytest.raises(epsm.EpsmError) as ei:
            epsm.search_noalloc_into(plan, t, None, hits)
        assert ei.value.status == 4
        torch.cuda.synchronize()
        assert int(hits.item()) == -1  # nothing was launched
    finally:
        epsm.set_tile_config(8, 16)
    say(f"noalloc size limit: n={n} at 128 KiB tiles (count only)")
    epsm.search_noalloc_into(plan, t, None, hits)
    epsm.stream_check()
    assert int(hits.item()) == n
    del t
    torch.cuda.empty_cache()

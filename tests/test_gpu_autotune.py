"""Autotuner on the GPU: every timed variant gives the default's output, and
searches under the tuned table equal the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def at():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_6449_amd as epsm
    from paper_1209_6449_amd import autotune
    epsm.lib()
    yield epsm, autotune
    autotune.reset()


def say(msg):
    print(msg, flush=True)


def test_small_tune_and_apply(at, tmp_path):
    epsm, autotune = at
    say("tune: sizes 64 KiB, 1 MiB")
    cache = autotune.tune(sizes=(1 << 16, 1 << 20), reps=1, batch=False, log=say)
    assert len(cache["table"]) == 2 * 2 * len(autotune.CLASS_MS)
    assert all(len(r) == 6 and r[5] in (0, 1, 2) for r in cache["table"])
    built = [list(t) for t in epsm.tile_configs()]
    assert all(list(r[3:5]) in built for r in cache["table"])
    assert 8 <= cache["hash_bits"] <= 14
    path = str(tmp_path / "tune.json")
    autotune.save(cache, path)
    loaded = autotune.load(path)
    assert autotune.matches(loaded, autotune.device_key())
    autotune.apply(loaded)
    try:
        for n in (1000, 70_000, 1 << 20, 3 << 20):
            spec = W.TextSpec(n=n, kind="uniform", key=W.text_key(90, n), sigma=4)
            host = W.gen_numpy(spec, 0, n)
            text = torch.from_numpy(host.copy()).cuda()
            g = np.random.default_rng(n)
            for m in (1, 3, 5, 12, 16, 27):
                off = int(g.integers(0, n - m + 1))
                p = bytes(host[off:off + m])
                say(f"tuned search n={n} m={m}")
                got = epsm.search(text, p).cpu().numpy()
                assert np.array_equal(got, oracle.positions(host, p)), (n, m)
                assert epsm.count(text, p) == got.size
        epsm.stream_check()
    finally:
        autotune.reset()


def test_batch_tile_tuning_identical(at):
    epsm, autotune = at
    say("batch tile tuning (small)")
    best, per = autotune.tune_batch(n_texts=24, max_len=1 << 18, reps=1, log=say)
    assert best in autotune.BATCH_WAVES and set(per) == {str(w) for w in autotune.BATCH_WAVES}


def test_variant_tuning_and_hinted_searches(at):
    """The variant stage on small texts: every candidate gave the built-in
    variant's output (checked inside), and searches whose plans carry an
    alphabet hint, under the resulting table, equal the oracle."""
    epsm, autotune = at
    say("variant tuning (4 MiB texts)")
    rows, timings = autotune.tune_variants([], 11, n=1 << 22, reps=1, log=say)
    assert len(timings) == len(autotune.VARIANT_SIGMAS) * len(autotune.VARIANT_MS)
    for r in rows:
        assert len(r) == 6 and r[4] in (epsm.VARIANT_DIRECT, epsm.VARIANT_FINGERPRINT)
    # whatever was measured, force a table that exercises every row kind
    table = [(17, 64, 1, 2, epsm.VARIANT_DIRECT, epsm.PLAN_SHORT_RUN),
             (16, 16, 1, 4, epsm.VARIANT_DIRECT, 0),
             (15, 15, 0, 256, epsm.VARIANT_FINGERPRINT, epsm.PLAN_HASH_BITS(13)),
             (17, 40, 3, 9, epsm.VARIANT_DIRECT, 0)] + [tuple(r) for r in rows]
    epsm.set_variant_table(table)
    try:
        for sigma in (2, 4, 20, 64):
            n = (1 << 21) + 77
            spec = W.TextSpec(n=n, kind="uniform", key=W.text_key(93, sigma), sigma=sigma)
            host = W.gen_numpy(spec)
            text = torch.from_numpy(host.copy()).cuda()
            est = epsm.estimate_alphabet(text)
            assert abs(est - sigma) <= max(1, sigma // 30), (sigma, est)
            g = np.random.default_rng(sigma)
            for m in (15, 16, 17, 20, 24, 31, 32, 40, 64):
                off = int(g.integers(0, n - m + 1))
                for p in (bytes(host[off:off + m]), bytes(g.integers(0, sigma, m).astype(np.uint8))):
                    plan = epsm.Plan(p, epsm.PLAN_SIGMA(est))
                    info = plan.info()
                    say(f"hinted search sigma={sigma} m={m} variant={info['variant']} "
                        f"run={info['run_blocks']} row={info['table_row']}")
                    got = epsm.search(text, plan).cpu().numpy()
                    assert np.array_equal(got, oracle.positions(host, p)), (sigma, m)
                    assert epsm.count(text, plan) == got.size
        epsm.stream_check()
    finally:
        epsm.set_variant_table([])


def test_estimate_alphabet(at):
    epsm, _ = at
    n = 1 << 20
    a = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    assert epsm.estimate_alphabet(a) == 1
    assert epsm.estimate_alphabet(a[:0]) == 0
    assert epsm.estimate_alphabet(a[:1]) == 1
    spec, _, _, _ = W.config3(n=n)
    z = W.gen_bytes(spec, device="cuda")
    # Zipf(1) over 96 symbols: sum p^2 is about 0.0617, so about 16
    assert 14 <= epsm.estimate_alphabet(z) <= 18
    # the estimate is the definition applied to the first 64 KiB
    h = np.bincount(z[:65536].cpu().numpy(), minlength=256).astype(np.int64)
    assert epsm.estimate_alphabet(z) == int(round(65536 ** 2 / int((h * h).sum())))
    two = torch.tensor([0, 1] * 100, dtype=torch.uint8, device="cuda")
    assert epsm.estimate_alphabet(two) == 2

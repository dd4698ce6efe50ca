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

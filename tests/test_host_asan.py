"""The host side of the library under AddressSanitizer (host code only; the
device code is compiled as usual and never runs here): plan building for
every variant, plan info, tune tables and error paths, in a subprocess with
the sanitizer runtime preloaded.  Any invalid host memory access aborts it."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
sys.path.insert(0, sys.argv[2])
from paper_1209_6449_amd import _lib
_lib.load(sys.argv[1])
import numpy as np
import paper_1209_6449_amd as epsm
H = epsm.PLAN_HOST_ONLY
rng = np.random.default_rng(7)
for m in list(range(1, 40)) + [64, 100, 262, 263, 300, 519, 1031, 2055, 4096]:
    for sigma in (1, 2, 4, 256):
        p = rng.integers(0, sigma, m).astype(np.uint8).tobytes()
        for flags in (0, epsm.PLAN_NO_STRIDE, epsm.PLAN_FORCE_DIRECT, epsm.PLAN_HASH_BITS(14), epsm.PLAN_PREFIX4):
            info = epsm.Plan(p, flags | H).info()
            assert info["m"] == m
        if m >= 15:
            epsm.Plan(p, epsm.PLAN_FORCE_FINGERPRINT | epsm.PLAN_COLLIDE | H).info()
        codes = rng.integers(0, 4, m).astype(np.uint8).tobytes()
        epsm.Plan(codes, epsm.PLAN_DNA | H).info()
for bad, flags in ((b"", 0), (b"a" * 4097, 0), (b"\x05", epsm.PLAN_DNA), (b"ab", 0x2000000)):
    try:
        epsm.Plan(bad, flags | H)
        raise SystemExit("expected an error")
    except epsm.EpsmError:
        pass
tiles = epsm.tile_configs()
epsm.set_tune_table([(c, co, 1 << 20, *tiles[-1], 2) for c in range(epsm.N_CLASSES) for co in (0, 1)])
epsm.set_tune_table([])
epsm.set_default_hash_bits(13)
epsm.set_default_hash_bits(0)
L = epsm.lib()
for st in range(6):
    L.epsm_status_string(st)
L.epsm_last_error()
print("host asan ok")
'''


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm*/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def asan_lib(tmp_path_factory):
    rt = asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime")
    from paper_1209_6449_amd import build
    out = str(tmp_path_factory.mktemp("asan") / "libepsm_asan.so")
    build.build(out=out, extra=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                                "-g1"])
    return rt, out


def test_host_code_under_address_sanitizer(asan_lib):
    rt, lib = asan_lib
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", SCRIPT, lib, ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "host asan ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])

"""Host-side checks of the C ABI (no GPU compute): symbols, plan logic, errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1209_6449_amd as epsm
from paper_1209_6449_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epsm.h")


def declared_functions() -> list[str]:
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epsm_[a-z_]+)\s*\(", src)) - {"epsm_plan_s"})


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "epsm_search" in names and "epsm_search_batch" in names and "epsm_count" in names
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares the same set
    assert sorted(_lib.SIGNATURES) == names


def test_version_and_status_strings():
    L = epsm.lib()
    assert L.epsm_version() >= 100
    assert L.epsm_status_string(0) == b"EPSM_OK"
    assert L.epsm_status_string(4) == b"EPSM_EUNSUPPORTED"


def host_plan(p: bytes, flags: int = 0) -> dict:
    return epsm.Plan(p, flags | epsm.PLAN_HOST_ONLY).info()


@pytest.mark.parametrize("m", list(range(1, 16)))
def test_short_patterns_use_direct_variant(m):
    info = host_plan(bytes(range(1, m + 1)))
    assert info["variant"] == epsm.VARIANT_DIRECT and info["table"] is None
    assert info["device"] == -1


@pytest.mark.parametrize("m", [16, 17, 24, 31, 32, 33, 100])
def test_long_patterns_use_fingerprint_variant(m):
    info = host_plan(bytes((7 * i) % 251 for i in range(m)))
    assert info["variant"] == epsm.VARIANT_FINGERPRINT and info["hash_bits"] == 11


def test_packed_words_and_masks_little_endian():
    p = bytes([0x00, 0x11, 0x22, 0x33, 0x44, 0x55])
    info = host_plan(p)
    assert info["words"][0] == 0x33221100 and info["words"][1] == 0x5544
    assert info["masks"][0] == 0xFFFFFFFF and info["masks"][1] == 0xFFFF and info["masks"][2] == 0
    assert info["prefix_words"] == 2


def le32(b: bytes, at: int) -> int:
    return int.from_bytes(b[at:at + 4], "little")


@pytest.mark.parametrize("bits", [8, 11, 14])
def test_fingerprint_table_is_section_3_4_bucket_map(bits):
    """Bucket h(p[j..j+7]) holds offset j (bit 8-j) for j in 0..7, and nothing else."""
    L = epsm.lib()
    rng = np.random.default_rng(bits)
    for m in (15, 16, 20, 32, 40):
        p = rng.integers(0, 4, m).astype(np.uint8).tobytes()
        flags = epsm.PLAN_HASH_BITS(bits) | (epsm.PLAN_FORCE_FINGERPRINT if m == 15 else 0)
        info = host_plan(p, flags)
        table = info["table"]
        assert len(table) == 1 << bits
        expect = [0] * (1 << bits)
        for j in range(8):
            v = L.epsm_fingerprint(le32(p, j), le32(p, j + 4), bits, 0)
            assert v < (1 << bits)
            expect[v] |= 1 << (8 - j)
        assert table == expect


def test_collide_mode_puts_every_offset_in_bucket_zero():
    info = host_plan(bytes(range(20)), epsm.PLAN_COLLIDE)
    assert info["table"][0] == 0b111111110 and not any(info["table"][1:])


@pytest.mark.parametrize("m,flags,width", [
    (1, 0, 1), (3, 0, 3), (4, 0, 4), (5, 0, 5), (7, 0, 7), (8, 0, 8), (15, 0, 8),
    (5, epsm.PLAN_PREFIX4, 4), (8, epsm.PLAN_PREFIX4, 4), (15, epsm.PLAN_PREFIX4, 4), (16, 0, 0),
    (20, epsm.PLAN_FORCE_DIRECT, 4),
])
def test_direct_prefix_width(m, flags, width):
    """The direct filter compares min(m, 8) prefix bytes (one 64-bit word for
    m >= 5) unless EPSM_PLAN_PREFIX4 (4); a register run of three loads
    (direct m > 16) keeps 4; other variants report 0."""
    assert host_plan(bytes((5 * i + 2) % 256 for i in range(m)), flags)["prefix_bytes"] == width


def test_force_flags():
    assert host_plan(b"x" * 20, epsm.PLAN_FORCE_DIRECT)["variant"] == epsm.VARIANT_DIRECT
    assert host_plan(b"x" * 15, epsm.PLAN_FORCE_FINGERPRINT)["variant"] == epsm.VARIANT_FINGERPRINT


@pytest.mark.parametrize("pattern,flags", [
    (b"", 0),                                                        # m == 0
    (b"abc", epsm.PLAN_FORCE_FINGERPRINT),                           # needs m >= 15
    (b"abc", epsm.PLAN_FORCE_DIRECT | epsm.PLAN_FORCE_FINGERPRINT),  # exclusive
    (b"abc", 0x2000000),                                             # unknown flag
    (b"abc", epsm.PLAN_SIGMA(300)),                                  # alphabet hint above 256
    (b"a" * 20, epsm.PLAN_HASH_BITS(5)),                             # k out of range
])
def test_plan_rejects_bad_arguments(pattern, flags):
    with pytest.raises(epsm.EpsmError) as e:
        epsm.Plan(pattern, flags | epsm.PLAN_HOST_ONLY)
    assert e.value.status == _lib.EPSM_EINVAL and e.value.detail


def test_plan_rejects_too_long_pattern():
    with pytest.raises(epsm.EpsmError) as e:
        epsm.Plan(b"a" * (epsm.MAX_M + 1), epsm.PLAN_HOST_ONLY)
    assert e.value.status == _lib.EPSM_EUNSUPPORTED


def test_null_arguments_rejected():
    L = epsm.lib()
    out = ctypes.c_void_p()
    assert L.epsm_plan(None, 3, 0, ctypes.byref(out)) == _lib.EPSM_EINVAL
    assert L.epsm_plan_get_info(None, None) == _lib.EPSM_EINVAL
    assert L.epsm_search(None, None, 0, None, 0, None, None) == _lib.EPSM_EINVAL
    assert L.epsm_count(None, None, 0, None, None) == _lib.EPSM_EINVAL
    assert L.epsm_search_batch(None, None) == _lib.EPSM_EINVAL


def test_host_only_plan_is_rejected_by_search():
    plan = epsm.Plan(b"abc", epsm.PLAN_HOST_ONLY)
    L = epsm.lib()
    dummy = ctypes.c_uint64()
    st = L.epsm_search(plan.handle, ctypes.addressof(dummy), 8, None, 0, ctypes.addressof(dummy), None)
    assert st == _lib.EPSM_EINVAL
    assert b"host-only" in L.epsm_last_error()


def test_server_null_arguments():
    L = epsm.lib()
    out = ctypes.c_void_p()
    assert L.epsm_server_create(None, None) == _lib.EPSM_EINVAL
    assert L.epsm_server_add_text(None, None, 0, None) == _lib.EPSM_EINVAL
    assert L.epsm_server_submit(None, 0, None, None, 0, None) == _lib.EPSM_EINVAL
    n = ctypes.c_uint32()
    assert L.epsm_server_poll(None, None, 0, ctypes.byref(n), 0) == _lib.EPSM_EINVAL
    assert L.epsm_server_release(None, 1) == _lib.EPSM_EINVAL
    assert L.epsm_server_get_stats(None, None) == _lib.EPSM_EINVAL
    assert L.epsm_server_now(None) == 0.0
    L.epsm_server_destroy(None)


def test_batch_plan_null_arguments():
    L = epsm.lib()
    assert L.epsm_batch_prepare(None, None) == _lib.EPSM_EINVAL
    assert L.epsm_batch_launch(None, None) == _lib.EPSM_EINVAL
    assert L.epsm_batch_get_info(None, None, None, None) == _lib.EPSM_EINVAL
    L.epsm_batch_destroy(None)


# ---- tuning: built tiles, tune table, default fingerprint width -------------

def test_tile_configs_listed_and_accepted():
    tiles = epsm.tile_configs()
    assert tiles[0] == (8, 16) and (4, 32) in tiles and len(set(tiles)) == len(tiles)
    for w, p in tiles:
        epsm.set_tile_config(w, p)
    epsm.set_tile_config(*tiles[0])
    with pytest.raises(epsm.EpsmError) as e:
        epsm.set_tile_config(3, 16)
    assert e.value.status == _lib.EPSM_EUNSUPPORTED


@pytest.mark.parametrize("m,flags,cls", [
    (1, 0, epsm.CLASS_BYTES), (3, 0, epsm.CLASS_BYTES), (4, 0, epsm.CLASS_WORDS),
    (15, 0, epsm.CLASS_WORDS), (16, 0, epsm.CLASS_FINGERPRINT), (40, 0, epsm.CLASS_FINGERPRINT),
    (20, epsm.PLAN_FORCE_DIRECT, epsm.CLASS_WORDS), (15, epsm.PLAN_FORCE_FINGERPRINT, epsm.CLASS_FINGERPRINT),
])
def test_kernel_class_of_plan(m, flags, cls):
    assert host_plan(bytes((3 * i + 1) % 256 for i in range(m)), flags)["kernel_class"] == cls


@pytest.mark.parametrize("m", [1, 7, 8, 12, 15, 16, 17, 33, 48, 49, 100])
def test_dna_plan_packs_codes_two_bits_each(m):
    rng = np.random.default_rng(m)
    codes = rng.integers(0, 4, m).astype(np.uint8)
    info = host_plan(codes.tobytes(), epsm.PLAN_DNA)
    assert info["variant"] == epsm.VARIANT_DNA and info["kernel_class"] == epsm.CLASS_DNA
    assert info["prefix_words"] == min((m + 15) // 16, 3)
    for j in range(8):
        syms = codes[16 * j:16 * j + 16]
        assert info["words"][j] == sum(int(c) << (2 * t) for t, c in enumerate(syms))
        assert info["masks"][j] == sum(3 << (2 * t) for t in range(len(syms)))
    if m < 8:
        assert info["table"] is None and info["hash_bits"] == 0
        return
    if m < 16:
        # 4-symbol blocks index the 256-entry table directly: bit j of block j..j+3
        assert info["hash_bits"] == 8 and len(info["table"]) == 256
        exp = [0] * 256
        for j in range(4):
            exp[sum(int(codes[j + t]) << (2 * t) for t in range(4))] |= 1 << j
        assert info["table"] == exp
        return
    # the 8-symbol block filter: bit j of the bucket of block j..j+7
    k = info["hash_bits"]
    assert k == 11 and len(info["table"]) == 1 << k
    L = epsm.lib()
    exp = [0] * (1 << k)
    for j in range(8):
        block = sum(int(codes[j + t]) << (2 * t) for t in range(8))
        exp[L.epsm_fingerprint(block, 0, k, 0)] |= 1 << j
    assert info["table"] == exp


@pytest.mark.parametrize("pattern,flags", [
    (b"\x00\x04", epsm.PLAN_DNA),                                    # code > 3
    (b"\x00\x01", epsm.PLAN_DNA | epsm.PLAN_FORCE_DIRECT),           # no variant flags
    (b"\x00" * 20, epsm.PLAN_DNA | epsm.PLAN_HASH_BITS(12)),          # no fingerprint flags
])
def test_dna_plan_rejects(pattern, flags):
    with pytest.raises(epsm.EpsmError) as e:
        epsm.Plan(pattern, flags | epsm.PLAN_HOST_ONLY)
    assert e.value.status == _lib.EPSM_EINVAL


def test_dna_null_arguments():
    L = epsm.lib()
    assert L.epsm_search_dna(None, None, 0, None, 0, None, None) == _lib.EPSM_EINVAL
    assert L.epsm_count_dna(None, None, 0, None, None) == _lib.EPSM_EINVAL
    assert L.epsm_pack_dna(None, 5, None, None) == _lib.EPSM_EINVAL
    assert L.epsm_pack_dna(None, 0, None, None) == _lib.EPSM_OK      # nothing to pack
    plan = epsm.Plan(b"\x01\x02", epsm.PLAN_DNA | epsm.PLAN_HOST_ONLY)
    dummy = ctypes.c_uint64()
    st = L.epsm_search_dna(plan.handle, ctypes.addressof(dummy), 8, None, 0, ctypes.addressof(dummy), None)
    assert st == _lib.EPSM_EINVAL                                      # host-only plan


def test_tune_table_validation():
    tiles = epsm.tile_configs()
    ok = [(epsm.CLASS_WORDS, 0, 1 << 20, *tiles[1]), (epsm.CLASS_FINGERPRINT, 1, (1 << 64) - 1, *tiles[0])]
    epsm.set_tune_table(ok)
    for bad, status in [((4, 0, 1, 8, 16), _lib.EPSM_EINVAL),          # unknown class
                        ((0, 2, 1, 8, 16), _lib.EPSM_EINVAL),          # unknown mode
                        ((0, 0, 1, 8, 12), _lib.EPSM_EUNSUPPORTED),    # tile not built
                        ((0, 0, 1, 8, 16, 3), _lib.EPSM_EINVAL)]:      # unknown strategy
        with pytest.raises(epsm.EpsmError) as e:
            epsm.set_tune_table(ok + [bad])
        assert e.value.status == status
    with pytest.raises(epsm.EpsmError) as e:
        epsm.set_tune_table([ok[0]] * 257)
    assert e.value.status == _lib.EPSM_EINVAL
    L = epsm.lib()
    assert L.epsm_set_tune_table(None, 1) == _lib.EPSM_EINVAL
    assert L.epsm_set_tune_table(None, 0) == _lib.EPSM_OK
    epsm.set_tune_table([])


def test_default_hash_bits():
    p = bytes(range(30))
    try:
        epsm.set_default_hash_bits(13)
        assert host_plan(p)["hash_bits"] == 13
        assert len(host_plan(p)["table"]) == 1 << 13
        assert host_plan(p, epsm.PLAN_HASH_BITS(9))["hash_bits"] == 9   # explicit k wins
        assert host_plan(p[:10])["hash_bits"] == 0                       # direct variant
        for k in (7, 15):
            with pytest.raises(epsm.EpsmError):
                epsm.set_default_hash_bits(k)
        assert host_plan(p)["hash_bits"] == 13                           # kept on error
    finally:
        epsm.set_default_hash_bits(0)
    assert host_plan(p)["hash_bits"] == 11


def test_autotune_cache_round_trip(tmp_path):
    from paper_1209_6449_amd import autotune
    tiles = epsm.tile_configs()
    cache = {"version": autotune.CACHE_VERSION, "device": {"arch": "gfx950", "cus": 256},
             "table": [[epsm.CLASS_BYTES, 0, 1 << 24, *tiles[3]], [epsm.CLASS_WORDS, 1, (1 << 64) - 1, *tiles[2]]],
             "hash_bits": 12, "batch_waves": 16}
    path = str(tmp_path / "t.json")
    autotune.save(cache, path)
    got = autotune.load(path)
    assert got == cache
    assert autotune.matches(got, {"arch": "gfx950", "cus": 256})
    assert not autotune.matches(got, {"arch": "gfx942", "cus": 304})
    assert not autotune.matches(dict(got, table=[[0, 0, 1, 8, 12]]))
    assert not autotune.matches(dict(got, version=0))
    try:
        autotune.apply(got)
        assert host_plan(bytes(range(20)))["hash_bits"] == 12
    finally:
        autotune.reset()
    assert host_plan(bytes(range(20)))["hash_bits"] == 11


def test_header_constants_match_binding():
    """Every numeric #define of include/epsm.h has the same value in the binding."""
    src = open(HEADER).read()
    defs = dict(re.findall(r"#define EPSM_([A-Z0-9_]+) (0x[0-9a-fA-F]+|\d+)u", src))
    assert len(defs) >= 15
    for name, val in defs.items():
        assert hasattr(_lib, name), name
        assert getattr(_lib, name) == int(val, 0), name


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """The ctypes mirrors have the sizes and field offsets gcc gives the
    structs of include/epsm.h."""
    import ctypes as C
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    mirrors = {"epsm_plan_info": _lib.PlanInfo, "epsm_tune_entry": _lib.TuneEntry,
               "epsm_text_ref": _lib.TextRef, "epsm_pair_ref": _lib.PairRef, "epsm_batch": _lib.Batch,
               "epsm_server_config": _lib.ServerConfig, "epsm_query_result": _lib.QueryResult,
               "epsm_server_stats": _lib.ServerStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "epsm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


@pytest.mark.parametrize("m,flags,variant,stride", [
    (262, 0, epsm.VARIANT_FINGERPRINT, 0),
    (263, 0, epsm.VARIANT_STRIDE, 256),
    (518, 0, epsm.VARIANT_STRIDE, 256),
    (519, 0, epsm.VARIANT_STRIDE, 512),
    (4096, 0, epsm.VARIANT_STRIDE, 2048),
    (1000, epsm.PLAN_NO_STRIDE, epsm.VARIANT_FINGERPRINT, 0),
    (1000, epsm.PLAN_FORCE_FINGERPRINT, epsm.VARIANT_FINGERPRINT, 0),
    (1000, epsm.PLAN_COLLIDE, epsm.VARIANT_FINGERPRINT, 0),
    (1000, epsm.PLAN_FORCE_DIRECT, epsm.VARIANT_DIRECT, 0),
])
def test_long_pattern_variant_and_stride(m, flags, variant, stride):
    """The stride is the largest power of two <= min(m - 7, 2048), at least 256."""
    info = host_plan(bytes((5 * i + 3) % 256 for i in range(m)), flags)
    assert info["variant"] == variant and info["stride"] == stride
    if variant == epsm.VARIANT_STRIDE:
        assert info["kernel_class"] == epsm.CLASS_FINGERPRINT and info["table"] is not None


def test_variant_table_chooses_the_plan_variant():
    """Rows are matched by m and the alphabet hint, first match wins; a plan
    without a hint matches only rows whose sigma range holds 0."""
    V = epsm
    try:
        V.set_variant_table([
            (17, 32, 1, 2, V.VARIANT_DIRECT, V.PLAN_SHORT_RUN),
            (16, 16, 1, 4, V.VARIANT_DIRECT, 0),
            (15, 15, 0, 256, V.VARIANT_FINGERPRINT, V.PLAN_HASH_BITS(13)),
            (16, 600, 0, 256, V.VARIANT_FINGERPRINT, 0),
        ])
        short = host_plan(b"ab" * 10, V.PLAN_SIGMA(2))
        assert (short["variant"], short["run_blocks"], short["prefix_bytes"], short["table_row"]) == \
            (V.VARIANT_DIRECT, 2, 8, 1)
        assert host_plan(b"ab" * 10, V.PLAN_SIGMA(2) | V.PLAN_PREFIX4)["prefix_bytes"] == 4
        d16 = host_plan(b"x" * 16, V.PLAN_SIGMA(4))
        assert (d16["variant"], d16["run_blocks"], d16["table_row"]) == (V.VARIANT_DIRECT, 2, 2)
        f15 = host_plan(b"x" * 15)
        assert (f15["variant"], f15["hash_bits"], f15["table_row"]) == (V.VARIANT_FINGERPRINT, 13, 3)
        assert host_plan(b"x" * 15, V.PLAN_HASH_BITS(9))["hash_bits"] == 9  # the plan's own k wins
        # no hint: the sigma 1..2 row does not match, the generic one does
        g = host_plan(b"ab" * 10)
        assert (g["variant"], g["table_row"]) == (V.VARIANT_FINGERPRINT, 4)
        # a per-block fingerprint row keeps the stride off
        long = host_plan(bytes(range(256)) * 2)
        assert (long["variant"], long["stride"], long["table_row"]) == (V.VARIANT_FINGERPRINT, 0, 4)
        # forced plans ignore the table
        assert host_plan(b"ab" * 10, V.PLAN_SIGMA(2) | V.PLAN_FORCE_FINGERPRINT)["table_row"] == 0
        # outside every row: the built-in choice
        b = host_plan(b"x" * 40, V.PLAN_SIGMA(2))
        assert (b["variant"], b["run_blocks"], b["table_row"]) == (V.VARIANT_FINGERPRINT, 2, 4)
        assert host_plan(b"x" * 12, V.PLAN_SIGMA(2))["table_row"] == 0
    finally:
        V.set_variant_table([])
    assert host_plan(b"ab" * 10, V.PLAN_SIGMA(2))["table_row"] == 0
    assert host_plan(b"ab" * 10, V.PLAN_SIGMA(2))["variant"] == V.VARIANT_FINGERPRINT
    assert host_plan(bytes(range(256)) * 2)["variant"] == V.VARIANT_STRIDE


@pytest.mark.parametrize("row", [
    (0, 10, 0, 256, 1, 0),               # m_min 0
    (10, 9, 0, 256, 1, 0),               # empty m range
    (16, 32, 5, 4, 1, 0),                # empty sigma range
    (16, 32, 0, 300, 1, 0),              # sigma above 256
    (16, 32, 0, 256, 3, 0),              # DNA is not a table variant
    (14, 32, 0, 256, 2, 0),              # fingerprint below 15
    (30, 400, 0, 256, 4, 0),             # strided below 39
    (16, 32, 0, 256, 1, 0x1),            # a flag rows may not add
    (16, 32, 0, 256, 2, 0x500),          # k = 5
])
def test_variant_table_rejects_bad_rows(row):
    epsm.set_variant_table([(20, 20, 0, 256, epsm.VARIANT_DIRECT, 0)])
    try:
        with pytest.raises(epsm.EpsmError) as e:
            epsm.set_variant_table([row])
        assert e.value.status == _lib.EPSM_EINVAL and e.value.detail
        assert host_plan(b"y" * 20)["table_row"] == 1  # the old table is kept
    finally:
        epsm.set_variant_table([])


@pytest.mark.parametrize("m,S", [(39, 32), (71, 64), (72, 64), (135, 128), (262, 128), (263, 256), (600, 512)])
def test_stride_rows_below_263(m, S):
    epsm.set_variant_table([(39, 4096, 0, 256, epsm.VARIANT_STRIDE, 0)])
    try:
        info = host_plan((bytes(range(256)) * 3)[:m])
        assert (info["variant"], info["stride"], info["table_row"]) == (epsm.VARIANT_STRIDE, S, 1)
    finally:
        epsm.set_variant_table([])
    info = host_plan((bytes(range(256)) * 3)[:m])
    assert info["variant"] == (epsm.VARIANT_STRIDE if m >= 263 else epsm.VARIANT_FINGERPRINT)


def test_variant_rows_merge():
    from paper_1209_6449_amd.autotune import merge_variant_rows
    D, F, SR = epsm.VARIANT_DIRECT, epsm.VARIANT_FINGERPRINT, epsm.PLAN_SHORT_RUN
    rows = [(16, 17, 1, 2, D, 0), (16, 17, 3, 9, D, 0), (16, 17, 10, 256, F, 0),
            (18, 22, 1, 2, D, SR), (18, 22, 3, 9, D, SR), (18, 22, 10, 256, D, SR), (18, 22, 0, 0, D, SR),
            (23, 28, 0, 0, D, SR), (23, 28, 1, 256, D, SR), (29, 40, 1, 256, D, SR)]
    assert merge_variant_rows(rows) == [
        (16, 17, 1, 2, D, 0), (16, 17, 3, 9, D, 0), (16, 17, 10, 256, F, 0),
        (18, 28, 0, 256, D, SR), (29, 40, 1, 256, D, SR)]
    assert merge_variant_rows([]) == []

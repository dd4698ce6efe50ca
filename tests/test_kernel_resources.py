"""Register and scratch use of the built gfx950 kernels, read from the code
object inside libepsm.so (CPU only: the ROCm binutils read our own build).

A private array indexed at run time, or a 64-bit value the compiler turns
into one access of a register run, silently moves that run to scratch
memory; a loop-carried value past the VGPR cap spills.  Either costs the
scans up to 3x, so no kernel may use scratch, and the batch kernels (which
hold every compare variant at once) must keep their occupancy."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1209_6449_amd", "libepsm.so")
LLVM = "/opt/rocm/llvm/bin"


def tool(name):
    path = os.path.join(LLVM, name)
    return path if os.path.exists(path) else shutil.which(name)


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    bundler, readelf, objcopy = tool("clang-offload-bundler"), tool("llvm-readelf"), shutil.which("objcopy")
    if not (bundler and readelf and objcopy):
        pytest.skip("ROCm binutils not available")
    if not os.path.exists(LIB):
        pytest.skip("libepsm.so not built")
    d = tmp_path_factory.mktemp("co")
    fatbin = str(d / "fatbin.bin")
    subprocess.run([objcopy, "-O", "binary", "--only-section=.hip_fatbin", LIB, fatbin], check=True)
    # one offload bundle per source file, back to back in the section
    data = open(fatbin, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [m.start() for m in re.finditer(re.escape(magic), data)]
    assert starts, "no offload bundle in .hip_fatbin"
    out = {}
    for i, a in enumerate(starts):
        part, co = str(d / f"b{i}.bin"), str(d / f"b{i}.o")
        with open(part, "wb") as f:
            f.write(data[a:starts[i + 1] if i + 1 < len(starts) else len(data)])
        subprocess.run([bundler, "--unbundle", "--type=o", f"--input={part}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True)
        notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
        cur = None
        for line in notes.splitlines():
            m = re.match(r"\s+\.(name|private_segment_fixed_size|vgpr_count):\s+(\S+)", line)
            if not m:
                continue
            if m.group(1) == "name":
                cur = m.group(2)
                out[cur] = {}
            elif cur is not None:
                out[cur][m.group(1)] = int(m.group(2))
    return out


def test_every_kernel_is_listed(kernels):
    names = " ".join(kernels)
    for k in ("scan_kernel", "expand_kernel", "tile_offsets_kernel", "sum_tiles_kernel", "batch_kernel",
              "stride_kernel", "pack_dna_kernel"):
        assert k in names, k


def test_no_kernel_uses_scratch(kernels):
    spilled = {k: v["private_segment_fixed_size"] for k, v in kernels.items()
               if v.get("private_segment_fixed_size", 0)}
    assert not spilled, spilled


def test_batch_kernels_keep_their_occupancy(kernels):
    """The batch kernels are latency bound: the 4-wave count and write
    kernels keep six waves per SIMD (80 registers), the others five (96)."""
    seen = 0
    for k, v in kernels.items():
        if "batch_kernel_" in k:
            seen += 1
            cap = 80 if "ILi4E" in k else 96
            assert v["vgpr_count"] <= cap, (k, v)
    assert seen == 6

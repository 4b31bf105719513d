"""Register budget of the hot kernels, read from the built library (CPU).

The step, adjoint and spin-derivative kernels are written to run two
wavefronts per SIMD (at most 256 registers per wavefront) without spilling;
small source changes can tip a kernel near that limit into spilling, which
costs 10-30 % and shows in no parity test.  This test extracts the gfx950
code objects from libteuk.so (clang offload bundles in its .hip_fatbin
section), reads each kernel's register counts from the code-object metadata
(llvm-readelf --notes) and holds the hot kernels to that budget.
"""
import os
import re
import shutil
import struct
import subprocess

import pytest

from paper_1010_3816_amd import binding

LLVM = "/opt/rocm/llvm/bin"
OBJCOPY, READELF = os.path.join(LLVM, "llvm-objcopy"), os.path.join(LLVM, "llvm-readelf")
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

# kernel (demangled prefix) -> most spilled VGPRs allowed
HOT = {
    "lw_step2_kernel<true, false,": 0,
    "lw_step_kernel<true, false,": 0,
    "lw_batch2_kernel": 0,
    "lw_batch_kernel": 0,
    "lw_tangent_kernel": 0,
    "lw_spin_tangent_kernel": 0,
    "lw_adjoint2_kernel": 0,
    "lw_adjoint_kernel<false,": 0,
    "lw_adjoint_kernel<true, false,": 2,  # the stored-state route: two spilled at 256 (measured, documented)
}


def _code_objects(lib, tmp):
    fat = os.path.join(tmp, "fatbin.bin")
    subprocess.run([OBJCOPY, f"--dump-section=.hip_fatbin={fat}", lib, os.path.join(tmp, "copy.so")], check=True,
                   capture_output=True)
    data = open(fat, "rb").read()
    out, pos = [], 0
    while (i := data.find(MAGIC, pos)) >= 0:
        count = struct.unpack_from("<Q", data, i + len(MAGIC))[0]
        off = i + len(MAGIC) + 8
        for _ in range(count):
            eo, es, tl = struct.unpack_from("<QQQ", data, off)
            triple = data[off + 24:off + 24 + tl].decode()
            off += 24 + tl
            if "gfx950" in triple and es > 0:
                path = os.path.join(tmp, f"co{len(out)}.elf")
                open(path, "wb").write(data[i + eo:i + eo + es])
                out.append(path)
        pos = i + 1
    return out


def _kernels(elf):
    """{mangled name: {key: int}} from the code object's metadata notes."""
    text = subprocess.run([READELF, "--notes", elf], check=True, capture_output=True, text=True).stdout
    ks, cur = {}, None
    for line in text.splitlines():
        if re.match(r"^\s+- \.(agpr_count|args):", line):  # first key of a kernel's map
            cur = {}
        m = re.match(r"^\s+-?\s*\.(\w+):\s+(\S+)", line)
        if m and cur is not None:
            cur[m.group(1)] = m.group(2)
            if m.group(1) == "name":
                ks[m.group(2)] = cur
    return ks


def _demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True)
    return [re.sub(r"\(.*", "", n.replace("teuk::(anonymous namespace)::", "").replace("void ", ""))
            for n in r.stdout.splitlines()]


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not (os.path.exists(OBJCOPY) and os.path.exists(READELF) and shutil.which("c++filt")):
        pytest.skip("LLVM tools not available")
    tmp = str(tmp_path_factory.mktemp("co"))
    ks = {}
    for co in _code_objects(binding.LIB_PATH, tmp):
        ks.update(_kernels(co))
    names = list(ks)
    return {d: ks[n] for d, n in zip(_demangle(names), names)}


def test_hot_kernels_fit_two_wavefronts_per_simd(kernels):
    seen = set()
    for name, md in kernels.items():
        for prefix, max_spill in HOT.items():
            if name.startswith(prefix):
                seen.add(prefix)
                regs = int(md.get("vgpr_count", 0)) + int(md.get("agpr_count", 0))
                spill = int(md.get("vgpr_spill_count", 0))
                assert regs <= 256, (name, regs)
                assert spill <= max_spill, (name, spill)
    assert seen == set(HOT), set(HOT) - seen


def test_block_kernel_fits_its_workgroup(kernels):
    """The small-grid block pass runs workgroups of up to 1024 threads, 16
    wavefronts on one CU: four per SIMD, so at most 128 VGPRs, no spills."""
    found = [n for n in kernels if n.startswith("lw_block_kernel")]
    assert found
    for name in found:
        md = kernels[name]
        regs = int(md.get("vgpr_count", 0)) + int(md.get("agpr_count", 0))
        assert regs <= 128, (name, regs)
        assert int(md.get("vgpr_spill_count", 0)) == 0, name

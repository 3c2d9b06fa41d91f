"""Checks on the gfx950 code the HIP kernels compile to (CPU only).

* No inline assembly in device code: an inline s_min_u32 once clobbered SCC
  between a compare and its branch, which sent the cost prefetch past the end
  of a slice.  The kernels use compiler builtins only.
* No packed-FP32 instructions (v_pk_add/mul/fma_f32).
* No scratch (register spills) in the aggregation kernels.
"""
import os
import re
import subprocess
import tempfile

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1610_04121_amd", "csrc")
SOURCES = ["sgm_kernels.hip"]


@pytest.fixture(scope="module")
def device_asm():
    from paper_1610_04121_amd import build
    text = []
    with tempfile.TemporaryDirectory() as d:
        for src in build.SOURCES:
            if not src.endswith(".hip"):
                continue
            out = os.path.join(d, src + ".s")
            cmd = [build.HIPCC, "--offload-arch=gfx950", "--cuda-device-only", "-S", "-O3", "-std=c++17",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-I", os.path.join(ROOT, "include"), "-o", out, os.path.join(CSRC, src)]
            subprocess.run(cmd, check=True, capture_output=True)
            text.append(open(out).read())
    return "\n".join(text)


def test_no_inline_asm_in_device_code(device_asm):
    assert "ASMSTART" not in device_asm


def test_no_packed_fp32(device_asm):
    assert not re.search(r"v_pk_(add|mul|fma)_f32", device_asm)


def test_aggregation_and_final_pass_kernels_do_not_spill(device_asm):
    names = re.findall(r"^(_Z\S*(?:aggregate_(?:batch_)?|final_pass_)kernel\S*):", device_asm, re.M)
    assert names
    for n in names:
        meta = device_asm[device_asm.index(n + ":"):]
        m = re.search(r"; ScratchSize: (\d+)", meta)
        assert m and int(m.group(1)) == 0, n


def test_no_scalar_cache_writes(device_asm):
    # every store and atomic goes through the vector memory path
    for pat in (r"\bs_store_", r"\bs_atomic_", r"\bs_buffer_store", r"\bs_buffer_atomic", r"\bs_dcache_wb",
                r"\bs_dcache_discard"):
        assert not re.search(pat, device_asm), pat


def _kernel_bodies(asm):
    """{kernel symbol: its instructions} for every function in the listing."""
    out = {}
    for m in re.finditer(r"^(_Z\S+):(?:[ \t]*;[^\n]*)?$", asm, re.M):
        name = m.group(1)
        end = asm.find(".Lfunc_end", m.end())
        out[name] = asm[m.end():end if end >= 0 else len(asm)]
    return out


def _descriptor(asm, name):
    i = asm.index(f".amdhsa_kernel {name}\n")
    return asm[i:asm.index(".end_amdhsa_kernel", i)]


def test_f16_minimum_kernels_keep_f16_denormals(device_asm):
    # On u8 planes the three-way minimum is a packed f16 minimum over integer
    # bit patterns below 0x1000, most of them f16 subnormals: it equals the
    # integer minimum only while the kernel keeps f16 denormals (mode 3 = no
    # flushing of inputs or outputs).
    users = [n for n, body in _kernel_bodies(device_asm).items() if "v_pk_minimum3_f16" in body]
    assert any("aggregate_kernel" in n for n in users)
    for n in users:
        assert re.search(r"\.amdhsa_float_denorm_mode_16_64 3\b", _descriptor(device_asm, n)), n


def test_f16_order_equals_unsigned_order_below_0x1000():
    # Exhaustive over every pair of u16 patterns below 0x1000 (zero, the f16
    # subnormals and the small normals): the IEEE minimum of the two values
    # read as f16 is the smaller pattern read as an unsigned integer.
    import numpy as np
    a = np.arange(0x1000, dtype=np.uint16)
    fa = a.view(np.float16)
    for lo in range(0, 0x1000, 0x400):
        b = np.arange(lo, lo + 0x400, dtype=np.uint16)
        got = np.minimum(fa[:, None], b.view(np.float16)[None, :]).view(np.uint16)
        want = np.minimum(a[:, None], b[None, :])
        assert np.array_equal(got, want)
    # and 0x0FFF (the kernels' stand-in for a missing neighbour) is above every
    # real candidate: Cmax + largest penalty <= 255 < 0x0FFF
    assert float(np.uint16(0x0FFF).view(np.float16)) > float(np.uint16(255 + 255).view(np.float16))

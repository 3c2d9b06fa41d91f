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


def test_aggregation_kernels_do_not_spill(device_asm):
    names = re.findall(r"^(_Z\S*aggregate_(?:batch_)?kernel\S*):", device_asm, re.M)
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

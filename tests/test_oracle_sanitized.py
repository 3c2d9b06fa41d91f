"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only) over small cases that reach every option and edge shape:
no memory error or undefined behaviour is reported, and every output equals
the regular build's."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from paper_1610_04121_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize", "run_cases.c")
ORACLE_SRC = os.path.join(os.path.dirname(HERE), "oracle", "sgm_oracle.c")

# (W, H, D, P1, P2, n_paths, cw, ch, median, lr, csct, lr_full, subpixel, adaptive, thr)
CASES = [
    (1, 1, 1, 7, 86, 4, 9, 7, 0, 0, 0, 0, 0, 0, 1),
    (1, 9, 8, 7, 86, 8, 9, 7, 1, 1, 0, 0, 0, 0, 1),
    (9, 1, 16, 7, 86, 8, 9, 7, 1, 1, 0, 1, 0, 0, 0),
    (5, 4, 12, 7, 86, 2, 9, 7, 0, 1, 0, 0, 1, 0, 2),
    (23, 17, 40, 7, 86, 4, 9, 7, 1, 1, 0, 0, 0, 0, 1),
    (23, 17, 40, 7, 86, 8, 9, 7, 1, 1, 1, 0, 1, 0, 1),
    (31, 12, 64, 5, 300, 8, 7, 5, 1, 1, 0, 1, 1, 1, 1),
    (12, 31, 70, 200, 100, 4, 3, 3, 0, 1, 0, 0, 0, 1, 0),
    (40, 6, 256, 7, 86, 8, 9, 7, 1, 1, 0, 1, 1, 1, 1),
    (17, 13, 20, 0, 0, 2, 5, 5, 1, 0, 1, 0, 0, 0, 1),
]


@pytest.fixture(scope="module")
def sanitized_binary(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "run_cases")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, DRIVER, ORACLE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def test_sanitized_oracle_matches_regular_build(sanitized_binary):
    blob, expect = bytearray(), []
    for k, c in enumerate(CASES):
        W, H, D, P1, P2, P, cw, ch, med, lr, csct, lrf, sub, ada, thr = c
        pair = synth.make_pair(W, H, D, "RS", seed=1610041400 + k)
        flags = (oracle.MEDIAN * med) | (oracle.LRCHECK * lr) | (oracle.CSCT * csct) | (oracle.LRFULL * lrf) | \
            (oracle.SUBPIXEL * sub) | (oracle.ADAPTIVE * ada)
        blob += struct.pack("<10i", W, H, D, P1, P2, P, cw, ch, flags, thr)
        blob += pair.left.tobytes() + pair.right.tobytes()
        want = oracle.sgm(pair.left, pair.right, D, P1, P2, P, cw, ch, median=bool(med), lr=bool(lr),
                          csct=bool(csct), lr_thr=thr, lr_full=bool(lrf), subpixel=bool(sub),
                          adaptive=bool(ada)).out
        expect.append(want)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=97:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    r = subprocess.run([sanitized_binary], input=bytes(blob), capture_output=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-2000:]
    assert b"runtime error" not in r.stderr and b"Sanitizer" not in r.stderr, r.stderr[-2000:]
    buf, pos = r.stdout, 0
    for k, want in enumerate(expect):
        (rc,) = struct.unpack_from("<i", buf, pos)
        pos += 4
        assert rc == 0, (k, rc)
        n = want.size * 2
        got = np.frombuffer(buf[pos:pos + n], dtype="<u2").reshape(want.shape)
        pos += n
        assert np.array_equal(got, want), k
    assert pos == len(buf)

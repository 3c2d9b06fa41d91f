"""The library used from C: tests/capi/capi_check.c links libsgm.so and the
oracle, allocates device buffers with hipMalloc, runs three pipelines on its
own stream, compares with the oracle and checks the documented errors."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(__file__), "capi", "capi_check")


def test_c_caller(gpu):
    assert os.path.exists(EXE), "tests/capi/capi_check is not built: run __graft_entry__.build()"
    print("running the C caller", flush=True)
    res = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0, res.stderr
    assert "capi_check OK" in res.stdout

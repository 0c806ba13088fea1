"""The library from plain C: tests/c/abi_roundtrip.c (built by build() with
gcc against include/mpewald.h and the in-tree libmpewald.so) runs forward,
adjoint, region split and octupole estimate through the C ABI on the GPU and
checks them against the oracle it links; it must exit 0."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_roundtrip")


def test_plain_c_consumer():
    assert os.path.exists(EXE), "tests/c/abi_roundtrip is missing: run __graft_entry__.build() first"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "all checks passed" in r.stdout

"""The C-ABI from a program that links libsphfilt.so and uses no Python or
PyTorch (tests/c_abi/abi_check.cpp, built by __graft_entry__.build()): the
dot-product identity <F x, y> = <x, F^T y> to 1e-13, F(2x) = 2 F(x) bit for
bit, in place equal to out of place, a batch equal to the plan and the
allocation-free call equal to the batch call, hybrid decisions replayed bit
for bit and the replayed adjoint the transpose, and status codes for bad
arguments."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "abi_check")


def test_c_abi_program():
    assert os.path.exists(EXE), "tests/c_abi/abi_check is not built: run __graft_entry__.build()"
    print("[gpu] c_abi/abi_check", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_check: ok" in r.stdout

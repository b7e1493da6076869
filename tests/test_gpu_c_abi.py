"""The C ABI driven from a C program (tests/c/abi_from_c.c, built by
__graft_entry__.build()): conservation of mass, momentum growth N F per step,
the in-place run's FP64 totals equal to the two-buffer run's, and argument
errors, all through plain C calls."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_from_c")


def test_c_program_drives_the_abi():
    assert os.path.exists(BIN), f"{BIN} is missing: run __graft_entry__.build()"
    print("case abi_from_c", flush=True)
    res = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0, res.stderr
    assert "abi_from_c ok" in res.stdout

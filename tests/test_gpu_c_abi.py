"""The library driven from C++ through its C ABI alone (no Python, no torch
in that process; buffers from hipMalloc): tests/c_abi/c_abi_step.cpp, built
by build().  A constant field under a constant velocity with matching
exterior values stays constant over 10 steps, its mass equals the volume,
and an invalid stage comes back as SDG_E_ARG with a message."""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(__file__), "c_abi", "c_abi_step")


def test_c_program_steps_through_the_c_abi():
    if not os.path.exists(EXE):
        raise RuntimeError(f"{EXE} is not built; run __graft_entry__.build()")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "c_abi_step:" in r.stdout

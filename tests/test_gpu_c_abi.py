"""The C ABI from plain C, with no Python in the path: a C99 program
(tests/c_abi/pcg_c_smoke.c) allocates with hipMalloc, solves a 32^3 Poisson
problem with shifted pipelined CG through include/pcg.h and libpcg.so, and
checks the solution and two argument errors.  It runs as a child process."""
import importlib.util
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _builder():
    spec = importlib.util.spec_from_file_location("c_abi_build", os.path.join(HERE, "c_abi", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_c_program_solves_through_the_abi():
    binary = _builder().build()  # built by build(); compiled here only when missing or stale
    r = subprocess.run([binary], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "status 0" in r.stdout and "rejects null workspace 1, mismatched grid 1" in r.stdout

"""The C ABI from a plain C program (tests/c_abi/mortar_c_example.c: upload,
workspace, pair search, pattern, integration and backward on a flat tied
interface, checked against the area, partition-of-unity, zero-gap and
zero-in-plane-gradient properties), built with gcc against the library and
the HIP runtime and run in a child process."""

import os
import subprocess

import pytest

from tests.test_capi import build_c_example

pytestmark = pytest.mark.gpu


def test_c_program_on_flat_tied_interface(tmp_path):
    exe = build_c_example(tmp_path)
    print(f"[gpu] running {exe}", flush=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=dict(os.environ))
    print(r.stdout)
    print(r.stderr)
    assert r.returncode == 0 and "c abi ok" in r.stdout

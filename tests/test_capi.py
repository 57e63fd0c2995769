"""CPU checks of the boundary: the HIP library loads and exports every entry
point the C header declares, and the binding declares exactly those."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mortar_mi355x.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mt_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("mt_create", "mt_upload", "mt_build_pairs", "mt_csr_pattern", "mt_integrate", "mt_backward",
              "mt_batch_forward", "mt_batch_backward", "mt_batch_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2202_03933_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_capi.LIB_PATH)  # loading runs no GPU code
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(_capi.SIGNATURES) == declared()


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_2202_03933_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError):
        _capi.lib()


C_EXAMPLE = os.path.join(ROOT, "tests", "c_abi", "mortar_c_example.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_example(outdir):
    """gcc build of the plain-C example against the header, the library and
    the HIP runtime (C host API only); returns the executable's path."""
    import shutil
    import subprocess
    from paper_2202_03933_amd import _capi
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("gcc or the HIP headers are not installed")
    libdir = os.path.dirname(_capi.LIB_PATH)
    exe = os.path.join(str(outdir), "mortar_c_example")
    cmd = [gcc, "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), C_EXAMPLE, "-L", libdir, "-lmortar_mi355x",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", f"-Wl,-rpath,{libdir}:{os.path.join(ROCM, 'lib')}",
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_header_is_c_and_the_example_links(tmp_path):
    # the header compiles as C99 and every entry point the C example calls
    # resolves against the built library (nothing is run here)
    from paper_2202_03933_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    assert os.path.exists(build_c_example(tmp_path))

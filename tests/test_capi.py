"""CPU checks of the boundary: the HIP library loads and exports every entry
point the C header declares, and the binding declares exactly those."""

import ctypes
import os
import re
import shutil
import subprocess

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


def test_binding_structs_match_the_header(tmp_path):
    # every struct the binding passes by pointer has, in C, the size and the
    # field offsets and sizes of its ctypes twin (a field renamed, retyped or
    # moved in the header shows here)
    from paper_2202_03933_amd import _capi as C
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = [C.mt_params, C.mt_stats, C.mt_capacity, C.mt_timings, C.mt_batch_tuning]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mortar_mi355x.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append(f'  printf("{n} . %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{n} {f} %zu %zu\\n", offsetof({n}, {f}), sizeof((({n}*)0)->{f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        n, f, *v = line.split()
        st = getattr(C, n)
        if f == ".":
            assert int(v[0]) == ctypes.sizeof(st), n
        else:
            fd = getattr(st, f)
            assert (int(v[0]), int(v[1])) == (fd.offset, fd.size), (n, f)
        seen += 1
    assert seen == sum(len(st._fields_) + 1 for st in structs)


def test_default_params_sets_fields_and_refuses_unknown_names():
    # mt_default_params is host code only (no device call), so it runs here
    from paper_2202_03933_amd import _capi as C, default_params
    p = default_params(delta=2.5e-3, dual=True, nodal_normals=True, rule=3, single_stream=1)
    assert (p.delta, p.lm_basis, p.normals, p.rule, p.single_stream) == (2.5e-3, C.MT_BASIS_DUAL,
                                                                          C.MT_NORMALS_NODAL, 3, 1)
    q = default_params()
    assert (q.lm_basis, q.normals, q.rule, q.newton_maxit) == (C.MT_BASIS_STANDARD, C.MT_NORMALS_ELEMENT, 7, 30)
    with pytest.raises(TypeError):
        default_params(delat=1e-3)


def test_mesh_shapes_checked_before_any_device_call():
    # the kernels read 3 coordinates per node and 4 node indices per element:
    # the binding refuses other shapes, and a coordinate update that changes
    # the node count, before anything reaches the library
    import numpy as np
    from paper_2202_03933_amd.interface import _check_mesh_shapes
    X, conn = np.zeros((9, 3)), np.zeros((4, 4), np.int32)
    _check_mesh_shapes(X, conn, "slave")
    _check_mesh_shapes(X, None, "slave", n_nodes=9)
    for bad in (dict(X=np.zeros((9, 2)), conn=conn), dict(X=np.zeros(27), conn=conn),
                dict(X=X, conn=np.zeros((4, 3), np.int32)), dict(X=X, conn=np.zeros(16, np.int32))):
        with pytest.raises(ValueError):
            _check_mesh_shapes(bad["X"], bad["conn"], "slave")
    with pytest.raises(ValueError):
        _check_mesh_shapes(np.zeros((10, 3)), None, "master", n_nodes=9)


def test_value_buffers_checked_before_any_device_call():
    # weights, values and gradients: float64, on the interface's device,
    # contiguous, at least the counted length (gradients exactly (3, n));
    # unknown counts (a search without read-back) skip the length only
    import torch
    from paper_2202_03933_amd.interface import _check_f64
    cpu = torch.device("cpu")
    _check_f64(torch.zeros(10, dtype=torch.float64), 10, "W_D", cpu)
    _check_f64(torch.zeros(12, dtype=torch.float64), 10, "W_D", cpu)  # a capacity-sized buffer
    _check_f64(torch.zeros(3, dtype=torch.float64), None, "W_D", cpu)
    _check_f64(torch.zeros(3, 7, dtype=torch.float64), 7, "gXs", cpu, rows=3)
    with pytest.raises(ValueError):
        _check_f64(torch.zeros(9, dtype=torch.float64), 10, "W_D", cpu)
    with pytest.raises(TypeError):
        _check_f64(torch.zeros(10, dtype=torch.float32), 10, "W_D", cpu)
    with pytest.raises(TypeError):
        _check_f64([0.0] * 10, 10, "W_D", cpu)
    with pytest.raises(ValueError):
        _check_f64(torch.zeros(10, 2, dtype=torch.float64)[:, 0], 10, "D", cpu)  # strided view
    with pytest.raises(ValueError):
        _check_f64(torch.zeros(7, 3, dtype=torch.float64), 7, "gXs", cpu, rows=3)  # (n, 3) instead of (3, n)
    with pytest.raises(ValueError):
        _check_f64(torch.zeros(3, 8, dtype=torch.float64), 7, "gXs", cpu, rows=3)
    with pytest.raises(ValueError):
        _check_f64(torch.zeros(10, dtype=torch.float64), 10, "W_D", torch.device("cuda", 0))

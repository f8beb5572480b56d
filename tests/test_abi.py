"""The C-ABI library loads and exports every entry point include/lp.h declares
(no compute: runs without a GPU), and host-side validation works."""

import os
import re
import subprocess

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lp.h")
LIB = os.path.join(ROOT, "paper_2002_08014_amd", "liblp.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = declared()
    for must in ("lp_create", "lp_run", "lp_sin_theta", "lp_destroy", "lp_workspace_size"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblp.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s+(\S+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblp.so not built")
def test_library_loads_and_binds():
    from paper_2002_08014_amd import _lib
    L = _lib.load()
    for n in declared():
        assert hasattr(L, n)
    assert L.lp_strerror(0).decode() == "ok"
    assert _lib.EXPORTS == tuple(n for n in _lib.EXPORTS if n in declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblp.so not built")
def test_workspace_size_validation_on_host():
    from paper_2002_08014_amd import _lib
    offs = np.array([0, 500, 1000, 1500, 2000])
    b = _lib.lp_workspace_size(torch.float64, 2000, 100, offs, 5)
    assert b > 4 * 100 * 5 * 8 * 3
    with pytest.raises(_lib.LPError) as e:
        _lib.lp_workspace_size(torch.float64, 2000, 100, np.array([0, 500, 500, 2000]), 5)
    assert e.value.status == _lib.LP_EINVAL
    with pytest.raises(_lib.LPError):
        _lib.lp_workspace_size(torch.float64, 2000, 100, np.array([0, 2001]), 5)
    with pytest.raises(_lib.LPError):
        _lib.lp_workspace_size(torch.float32, 2000, 100, offs, 65)     # k_max > 64
    with pytest.raises(_lib.LPError):
        _lib.lp_workspace_size(torch.float32, 2000, 4, offs, 5)        # k_max > d


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblp.so not built")
def test_abi_from_plain_c(tmp_path):
    """The header compiles as C99 (-Wall -Wextra -pedantic, warnings are errors) and a
    C program linked against liblp.so gets the same answers as the Python binding."""
    import shutil
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_from_c")
    libdir = os.path.dirname(LIB)
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-o", exe,
                    os.path.join(ROOT, "tests", "host", "abi_from_c.c"), "-L" + libdir, "-llp",
                    "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    from paper_2002_08014_amd import _lib
    st, nbytes = out[0].split()
    assert int(st) == _lib.LP_OK
    assert int(nbytes) == _lib.lp_workspace_size(torch.float64, 2000, 100,
                                                 np.array([0, 500, 1000, 1500, 2000]), 5)
    assert out[1].startswith(f"{_lib.LP_EINVAL} ") and out[2]


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding passes across the ABI has the C compiler's size
    and field offsets (a missing or misplaced field would shift the rest)."""
    import ctypes
    import shutil
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_layout")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I" + os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(ROOT, "tests", "host", "abi_layout.c")], check=True)
    lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    from paper_2002_08014_amd import _lib
    types = {"lp_run_opts": _lib.RunOpts, "lp_solve_opts": _lib.SolveOpts, "lp_run_stats": _lib.RunStats,
             "lp_solve_stats": _lib.SolveStats, "lp_tuning": _lib.Tuning, "lp_job": _lib.Job,
             "lp_job_result": _lib.JobResult}
    checked = 0
    for ln in lines:
        if not ln:
            continue
        name, val = ln.split()
        if "." in name:
            t, f = name.split(".")
            assert getattr(types[t], f).offset == int(val), name
        else:
            assert ctypes.sizeof(types[name]) == int(val), name
        checked += 1
    assert checked > 40

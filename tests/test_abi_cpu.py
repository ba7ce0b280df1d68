"""Host-side checks of the C ABI: the library loads and exports what the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpi3d.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpi3d_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mpi3d_forward", "mpi3d_adjoint", "mpi3d_solve", "mpi3d_plan_create", "mpi3d_batch_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2511_06627_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib._SIGS, name


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the C compiler's size and field
    offsets (a C program built from the header prints them)."""
    import shutil
    import subprocess
    import tempfile
    from paper_2511_06627_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mpi3d_geometry": _lib.Geometry, "mpi3d_plan_info": _lib.PlanInfo,
               "mpi3d_solve_opts": _lib.SolveOpts, "mpi3d_solve_report": _lib.SolveReport}
    cname_of = {"lam": "lambda"}      # a Python keyword in C
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpi3d.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, cname_of.get(f, f)))
    lines += ["return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_strerror_is_host_only():
    from paper_2511_06627_amd import _lib
    lib = _lib.load()
    assert lib.mpi3d_strerror(0) == b"ok"
    assert lib.mpi3d_strerror(-1) == b"invalid argument"
    assert lib.mpi3d_strerror(-99) == b"unknown status"


def test_null_arguments_rejected_without_device():
    from paper_2511_06627_amd import _lib
    lib = _lib.load()
    assert lib.mpi3d_plan_create(None, 0, None) == -1
    assert lib.mpi3d_forward(None, 0, None, None, None, 0, None) == -1
    assert lib.mpi3d_solve(None, None, None, None, None, 0, None, None, None) == -1

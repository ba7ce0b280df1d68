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


def test_struct_layouts_match_header_sizes():
    """ctypes mirrors of the ABI structs have the C sizes (alignment included)."""
    from paper_2511_06627_amd import _lib
    # computed from the header's field list with natural alignment on x86-64
    assert ctypes.sizeof(_lib.Geometry) == 96
    assert ctypes.sizeof(_lib.PlanInfo) == 80
    assert ctypes.sizeof(_lib.SolveOpts) == 32
    assert ctypes.sizeof(_lib.SolveReport) == 24


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

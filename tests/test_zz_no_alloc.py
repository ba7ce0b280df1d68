"""mpi3d_forward_noalloc through the C ABI: the forward operator with the
library's static scratch array instead of a caller workspace.

Checked against mpi3d_forward with a caller workspace (the same kernels in the
same order: equal bit for bit) and against the FP64 oracle, in FP32, mixed
and precomposed precision, on two calls in a row whose second input is smaller (the array
keeps the first call's contents); a plan whose workspace exceeds the array is
refused before anything is enqueued.
"""
import ctypes
import sys

import numpy as np
import pytest

from oracle import operator as oop
from helpers import oracle_geometry, rel_l2, random_volume

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _case(nx, ny, nz, M, T, khi, D):
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, T / 256 + 1 / 3, 2.0, 1, khi, D), iters_min=30, rtol=1e-9)
    return g


def _noalloc(plan, prec, x, out, torch_mod):
    from paper_2511_06627_amd import _lib
    from paper_2511_06627_amd.plan import PRECISION
    lib = _lib.load()
    st = ctypes.c_void_p(torch_mod.cuda.current_stream().cuda_stream)
    return lib.mpi3d_forward_noalloc(plan._h, PRECISION[prec], ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), st)


def test_noalloc_forward_matches_workspace_forward(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    cases = [(64, 48, 20, 9, 4096, 20, 2), (32, 32, 6, 4, 2048, 10, 1)]     # the second is smaller
    for i, (nx, ny, nz, M, T, khi, D) in enumerate(cases):
        _log("noalloc case %d: %dx%dx%d, %d angles, T %d" % (i, nx, ny, nz, M, T))
        g = _case(nx, ny, nz, M, T, khi, D)
        plan = Plan(nx, ny, nz, M, T, g.drive_cycles, g.psf_width, 1, khi, D, g.op_scale,
                    precisions=("fp32", "mixed", "precomposed"))
        x = random_volume(g, 50 + i)
        xd = torch_mod.from_numpy(x).float().cuda()
        want = oop.forward(g, x)
        for prec, tol in (("fp32", 1e-5), ("mixed", 5e-3), ("precomposed", 1e-5)):
            ref = plan.forward(xd, precision=prec)
            out = torch_mod.full(plan.data_shape, float("nan"), dtype=torch_mod.complex64, device="cuda")
            rc = _noalloc(plan, prec, xd, out, torch_mod)
            torch_mod.cuda.synchronize()
            assert rc == 0, rc
            err = rel_l2(out.cpu().numpy(), want)
            _log("  %s: equal to mpi3d_forward %s, rel err vs oracle %.3e"
                 % (prec, bool(torch_mod.equal(out, ref)), err))
            assert torch_mod.equal(out, ref)
            assert err <= tol


def test_noalloc_refuses_what_does_not_fit(torch_mod):
    from paper_2511_06627_amd import _lib
    from paper_2511_06627_amd.plan import Plan
    # 131072 lines of 256 floats: the projected lines alone need 128 MiB
    plan = Plan(256, 256, 1024, 128, 256, 256 / 256 + 1 / 3 + 1, 2.0, 1, 2, 0, 1.0)
    assert plan.info.op_ws_bytes > _lib.NOALLOC_SCRATCH_BYTES
    x = torch_mod.zeros(plan.shape, dtype=torch_mod.float32, device="cuda")
    out = torch_mod.zeros(plan.data_shape, dtype=torch_mod.complex64, device="cuda")
    assert _noalloc(plan, "fp32", x, out, torch_mod) == -2       # MPI3D_ENOMEM
    torch_mod.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    small = Plan(16, 16, 2, 2, 512, 512 / 256 + 1 / 3 + 1, 2.0, 1, 2, 0, 1.0, precisions=("fp32", "precomposed"))
    xs = torch_mod.zeros(small.shape, dtype=torch_mod.float32, device="cuda")
    os_ = torch_mod.zeros(small.data_shape, dtype=torch_mod.complex64, device="cuda")
    assert _noalloc(small, "mixed", xs, os_, torch_mod) == -1         # no mixed tables: EINVAL

"""Degenerate and extreme geometries on the GPU against the FP64 oracle: the
smallest scan, one slice and one angle, the widest compiled detector, the
largest angle count, a time grid that is not a whole number of 32-sample
chunks, and one-slice raster / dual-drive scans (where each variant reduces
to fewer line groups).

Tolerances: FP32 1e-5 and mixed 5e-3 relative L2, as for the other scans.
"""
import sys

import numpy as np
import pytest

from oracle import geometry, operator as oop
from helpers import rel_l2, random_volume

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_MIX_OP = 5e-3

# name: geometry keywords (oracle names) and the precisions to check
CASES = {
    # 2 x 2 x 1 voxels, one angle, T = 32 (one time chunk), two bins
    "smallest": dict(nx=2, ny=2, nz=1, n_angles=1, n_t=32, drive_cycles=32 / 16 + 1 / 3, psf_width=1.0,
                     harm_lo=1, harm_hi=2, half_band=0),
    # one slice, one angle, an ordinary line
    "one_line": dict(nx=40, ny=24, nz=1, n_angles=1, n_t=512, drive_cycles=512 / 64 + 1 / 3, psf_width=2.0,
                     harm_lo=1, harm_hi=6, half_band=1),
    # n_u = 256, the widest compiled detector, wider than the volume
    "widest": dict(nx=48, ny=48, nz=2, n_angles=3, n_t=1024, drive_cycles=1024 / 64 + 1 / 3, psf_width=2.5,
                   harm_lo=1, harm_hi=10, half_band=2, n_u=256),
    # 4096 angles (the largest accepted) of a small slice
    "most_angles": dict(nx=12, ny=12, nz=1, n_angles=4096, n_t=64, drive_cycles=64 / 16 + 1 / 3, psf_width=1.5,
                        harm_lo=1, harm_hi=3, half_band=0),
    # T = 1000: the last time chunk is partly padding
    "ragged_time": dict(nx=32, ny=32, nz=3, n_angles=4, n_t=1000, drive_cycles=1000 / 64 + 1 / 3, psf_width=2.0,
                        harm_lo=1, harm_hi=8, half_band=1),
    # one-slice raster (a single sweep direction) and one-slice dual drive
    "raster_one_slice": dict(nx=32, ny=32, nz=1, n_angles=5, n_t=1024, drive_cycles=1024 / 64 + 1 / 3,
                             psf_width=2.0, harm_lo=1, harm_hi=8, half_band=1, drive_amp=6.0, raster_sweep=12.0),
    "dual_one_slice": dict(nx=32, ny=32, nz=1, n_angles=5, n_t=1024, drive_cycles=1024 / 64 + 1 / 3,
                           psf_width=2.0, harm_lo=1, harm_hi=8, half_band=1, drive_axes=2),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _plan(kw, op_scale):
    from paper_2511_06627_amd.plan import Plan
    return Plan(kw["nx"], kw["ny"], kw["nz"], kw["n_angles"], kw["n_t"], kw["drive_cycles"], kw["psf_width"],
                kw["harm_lo"], kw["harm_hi"], kw["half_band"], op_scale, n_u=kw.get("n_u", 0),
                drive_amp=kw.get("drive_amp", 0.0), raster_sweep=kw.get("raster_sweep", 0.0),
                drive_axes=kw.get("drive_axes", 1), precisions=("fp32", "mixed"))


@pytest.mark.parametrize("name", list(CASES))
def test_edge_geometry_parity(name, torch_mod):
    kw = CASES[name]
    g = oop.normalised(geometry.Geometry(**kw), iters_min=30, rtol=1e-9)
    plan = _plan(kw, g.op_scale)
    x = random_volume(g, 1)
    rng = np.random.default_rng(2)
    shape = (g.n_data_lines, g.n_bins)
    y = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    want_f, want_a = oop.forward(g, x), oop.adjoint(g, y)
    xd = torch_mod.from_numpy(x).float().cuda()
    yd = torch_mod.from_numpy(y.reshape(plan.data_shape)).to(torch_mod.complex64).cuda()
    for prec, tol in (("fp32", TOL32), ("mixed", TOL_MIX_OP)):
        ef = rel_l2(plan.forward(xd, precision=prec).cpu().numpy(), want_f)
        ea = rel_l2(plan.adjoint(yd, precision=prec).cpu().numpy(), want_a)
        _log("%s %s rel err forward %.3e adjoint %.3e" % (name, prec, ef, ea))
        assert ef <= tol and ea <= tol

"""GPU parity of the FP32 operator with the band DFT factored over drive cycles.

The plan takes the factored form (t = n1 + P n2, a C-point sum over the drive
cycles at the residues of the kept bins mod C, then a P-point sum per bin)
when it needs less MFMA work than the dense band DFT.  These geometries are
chosen to take it and to cover its edges: a ragged last line tile, a phase
count P that is not a multiple of the kernels' 8- and 16-phase stages, one and
two 32-column residue tiles, C = 32 and C = 64 (one and two 32-cycle chunks
per phase), n_u padded to 64 and 128, a receive filter, and the three ways the
forward outer sum moves a line's 8-phase stage of Y into LDS (under 64
16-byte pieces: one partial instruction, R = 12; exactly 64, R = 14; over 64:
a last run overlapping the one before, R = 22).  Each forward and
adjoint is compared with the FP64 oracle (which evaluates the dense
definition) at the FP32 tolerance of the other operator tests; the full-size
factored scans are covered by the realistic and high-resolution tests.
"""
import sys

import numpy as np
import pytest

from oracle import operator as oop
from oracle.geometry import kept_bins
from helpers import oracle_geometry, rel_l2, random_volume, random_data

pytestmark = pytest.mark.gpu

TOL32 = 1e-5

# name: (nx, ny, nz, M, T, drive cycles, w, k_lo, k_hi, half band, C the plan takes, receive filter)
CASES = {
    # 35 lines (last tile 3 rows), P = 125 phases
    "ragged_p125": (32, 32, 5, 7, 4000, 4000 / 256 + 1 / 3, 2.0, 1, 20, 2, 32, False),
    # 14 residues: one 32-column tile; C = 64, two 32-cycle chunks per phase
    "one_tile_c64": (40, 24, 6, 5, 4096, 4096 / 128 + 0.1, 2.0, 1, 20, 2, 64, False),
    # C = 64 with 7 bins per harmonic, and a receive filter
    "c64_filter": (48, 40, 4, 5, 8192, 8192 / 128 + 1 / 3, 2.0, 1, 15, 3, 64, True),
    # n_u = 100 padded to 128; 22 residues: two column tiles
    "u128": (100, 60, 3, 6, 4096, 4096 / 256 + 1 / 3, 2.5, 1, 20, 2, 32, False),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _filter(nx, ny, nz, M, T, P, w, klo, khi, D):
    # an inductive receive coil: gain growing with frequency and a group delay
    om = np.asarray(kept_bins(oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D)), dtype=np.float64)
    return (om / om.max()) * np.exp(-2j * np.pi * om * 3.5 / T)


@pytest.mark.parametrize("name", list(CASES))
def test_factored_parity(name, torch_mod):
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D, C, filt = CASES[name]
    _log("case %s" % name)
    d = _filter(nx, ny, nz, M, T, P, w, klo, khi, D) if filt else None
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D, rx_filter=d), iters_min=30, rtol=1e-9)
    plan = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, g.op_scale, rx_filter=d)
    assert plan.dft_cycles == C, "plan took C = %d" % plan.dft_cycles
    x = random_volume(g, 61)
    y = random_data(g, 62)
    got = plan.forward(torch_mod.from_numpy(np.ascontiguousarray(x)).float().cuda()).cpu().numpy()
    ef = rel_l2(got, oop.forward(g, x))
    got = plan.adjoint(torch_mod.from_numpy(np.ascontiguousarray(y)).to(torch_mod.complex64).cuda()).cpu().numpy()
    ea = rel_l2(got, oop.adjoint(g, y))
    _log("%s (C = %d): forward rel err %.3e, adjoint rel err %.3e" % (name, C, ef, ea))
    assert ef <= TOL32 and ea <= TOL32

"""GPU parity of the operator A, its adjoint and their stages against the FP64 oracle.

Tolerance: FP32 path within 1e-5 relative L2 of the oracle (whole output
vector, complex values as (re, im) pairs), per result.
"""
import sys

import numpy as np
import pytest

from oracle import operator as oop, projector as oproj, signal as osig
from paper_2511_06627_amd import configs
from helpers import oracle_geometry, config_geometry, rel_l2, random_volume, random_data

pytestmark = pytest.mark.gpu

TOL32 = 1e-5

# name: geometry (nx, ny, nz, M, T, P, w, k_lo, k_hi, D)
CASES = {
    # the 32^3 parity scan
    "parity_32": (32, 32, 32, 8, 2048, 2048 / 256 + 1 / 3, 2.0, 1, 15, 2),
    # ragged everywhere: n_u 40 -> padded 64, 35 lines (one partial tile), T = 47 chunks,
    # 54 real columns -> 64
    "ragged": (40, 36, 5, 7, 1504, 1504 / 256 + 1 / 3, 2.0, 1, 9, 1),
    # several line tiles with a ragged last one, 7 column tiles, non-square slice
    "multi_tile": (64, 48, 20, 9, 4096, 4096 / 256 + 1 / 3, 3.0, 1, 20, 2),
    # odd detector width (the precomposed stage reads its lines one float at a time)
    "odd_u": (41, 30, 3, 5, 1504, 1504 / 256 + 1 / 3, 2.0, 1, 9, 1),
    # n_u = 128 (the remaining compiled detector width) with 13 harmonics
    "mid_128": (128, 96, 4, 5, 2048, 2048 / 256 + 1 / 3, 2.5, 1, 13, 2),
    # a slice too large for LDS (staged in two row bands), with the 90 degree
    # angle whose central rays run exactly along the band edge
    "banded": (220, 220, 3, 6, 1024, 1024 / 256 + 1 / 3, 2.0, 1, 7, 1),
    # enough lines that each block walks several time chunks (540 lines, 128
    # chunks), with a per-chunk operand stream that is not a multiple of 8
    "many_lines": (64, 64, 60, 9, 4096, 4096 / 256 + 1 / 3, 3.0, 1, 20, 2),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _make(name, torch_mod):
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D = CASES[name]
    g = oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D)
    g = oop.normalised(g, iters_min=30, rtol=1e-9)
    plan = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, g.op_scale)
    return g, plan


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_mod):
    _log("case %s" % request.param)
    return request.param, _make(request.param, torch_mod)


def _to_dev(torch_mod, a, dtype):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def test_forward_parity(case, torch_mod):
    name, (g, plan) = case
    x = random_volume(g, 1)
    want = oop.forward(g, x)
    got = plan.forward(_to_dev(torch_mod, x, torch_mod.float32)).cpu().numpy()
    err = rel_l2(got, want)
    _log("%s forward rel err %.3e" % (name, err))
    assert err <= TOL32


def test_adjoint_parity(case, torch_mod):
    name, (g, plan) = case
    y = random_data(g, 2)
    want = oop.adjoint(g, y)
    got = plan.adjoint(_to_dev(torch_mod, y, torch_mod.complex64)).cpu().numpy()
    err = rel_l2(got, want)
    _log("%s adjoint rel err %.3e" % (name, err))
    assert err <= TOL32


def test_projection_stages(case, torch_mod):
    name, (g, plan) = case
    x = random_volume(g, 3)
    want = oproj.project(g, x)
    got = plan.project(_to_dev(torch_mod, x, torch_mod.float32)).cpu().numpy()
    assert rel_l2(got, want) <= TOL32
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((g.n_angles, g.nz, g.n_u))
    want = oproj.backproject(g, rho)
    got = plan.backproject(_to_dev(torch_mod, rho, torch_mod.float32)).cpu().numpy()
    assert rel_l2(got, want) <= TOL32


def test_signal_stages(case, torch_mod):
    name, (g, plan) = case
    rng = np.random.default_rng(5)
    rho = rng.uniform(0, 1, (g.n_angles, g.nz, g.n_u))
    want = osig.forward(g, rho.reshape(-1, g.n_u)).reshape(g.n_angles, g.nz, g.n_bins)
    got = plan.signal_fwd(_to_dev(torch_mod, rho, torch_mod.float32)).cpu().numpy()
    assert rel_l2(got, want) <= TOL32
    y = random_data(g, 6)
    want = osig.adjoint(g, y.reshape(-1, g.n_bins)).reshape(g.n_angles, g.nz, g.n_u)
    got = plan.signal_adj(_to_dev(torch_mod, y, torch_mod.complex64)).cpu().numpy()
    assert rel_l2(got, want) <= TOL32


def test_gpu_adjoint_identity(case, torch_mod):
    """<A x, y> = <x, A^T y> from the GPU's own outputs (FP32 rounding only)."""
    name, (g, plan) = case
    x = random_volume(g, 7)
    y = random_data(g, 8)
    Ax = plan.forward(_to_dev(torch_mod, x, torch_mod.float32)).cpu().numpy().astype(np.complex128)
    ATy = plan.adjoint(_to_dev(torch_mod, y, torch_mod.complex64)).cpu().numpy().astype(np.float64)
    lhs = np.vdot(Ax, y.astype(np.complex64).astype(np.complex128)).real
    rhs = np.vdot(x.astype(np.float32).astype(np.float64), ATy)
    scale = np.linalg.norm(Ax) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_zero_input_gives_zero(case, torch_mod):
    name, (g, plan) = case
    z = torch_mod.zeros(plan.shape, dtype=torch_mod.float32, device="cuda")
    assert float(plan.forward(z).abs().max()) == 0.0
    zb = torch_mod.zeros(plan.data_shape, dtype=torch_mod.complex64, device="cuda")
    assert float(plan.adjoint(zb).abs().max()) == 0.0


def test_invalid_arguments_rejected(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    from paper_2511_06627_amd._lib import Mpi3dError
    with pytest.raises(Mpi3dError):   # bins beyond T/2
        Plan(16, 16, 2, 2, 64, 10.3, 2.0, 1, 9, 1, 1.0)
    with pytest.raises(Mpi3dError):   # overlapping bands
        Plan(16, 16, 2, 2, 1024, 2.1, 2.0, 1, 5, 2, 1.0)
    with pytest.raises(Mpi3dError):
        Plan(16, 16, 2, 2, 1024, 4.3, -1.0, 1, 5, 1, 1.0)


# ---------------------------------------------------------------------------
# Full-size realistic scan (192 x 192 x 96, 36 angles, T = 8192): every output
# line / slice the oracle can compute one at a time.  A is the same operator on
# each z-slice, so one slice of the oracle gives the exact reference for the
# corresponding lines of the GPU output.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def realistic(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.REALISTIC_192
    _log("case realistic_192x192x96")
    g = config_geometry(cfg)
    plan = Plan.from_config(cfg, g.op_scale)
    return cfg, g, plan


@pytest.mark.parametrize("slices", [(0, 41, 95)])
def test_realistic_forward_sampled(realistic, torch_mod, slices):
    cfg, g, plan = realistic
    x = configs.make_phantom(cfg)
    got = plan.forward(_to_dev(torch_mod, x, torch_mod.float32)).cpu().numpy()
    gs = g.slice_geometry()
    for k in slices:
        want = oop.forward(gs, x[k:k + 1])[:, 0, :]
        err = rel_l2(got[:, k, :], want)
        _log("realistic forward slice %d rel err %.3e" % (k, err))
        assert err <= TOL32


@pytest.mark.parametrize("slices", [(3, 50, 94)])
def test_realistic_adjoint_sampled(realistic, torch_mod, slices):
    cfg, g, plan = realistic
    y = random_data(g, 9)
    got = plan.adjoint(_to_dev(torch_mod, y, torch_mod.complex64)).cpu().numpy()
    gs = g.slice_geometry()
    for k in slices:
        want = oop.adjoint(gs, y[:, k:k + 1, :])[0]
        err = rel_l2(got[k], want)
        _log("realistic adjoint slice %d rel err %.3e" % (k, err))
        assert err <= TOL32


@pytest.mark.parametrize("name", ["parity_32", "ragged"])
def test_device_normalisation_matches_oracle(name, torch_mod):
    """op_scale = 0 asks the plan to find c_A (||A||_2 = 1) by power iteration
    on the device; it agrees with the oracle's FP64 power iteration."""
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D = CASES[name]
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D), iters_min=30, rtol=1e-12)
    plan = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, 0.0)
    rel = abs(plan.op_scale - g.op_scale) / g.op_scale
    _log("%s device c_A %.9e (%d iterations), oracle %.9e, rel %.2e"
         % (name, plan.op_scale, plan.norm_iters, g.op_scale, rel))
    assert plan.norm_iters > 0
    assert rel <= 1e-5


def test_receive_filter_and_harmonics_from_two(torch_mod):
    """A receive filter D_Gamma on the kept bins (eq. DCmodel) -- here the
    response of an inductive receive coil, growing with frequency and with a
    group delay -- and the paper's harmonic set from 2 (the fundamental notched
    out): FP32 and mixed operators against the oracle."""
    from paper_2511_06627_amd.plan import Plan
    from oracle.geometry import kept_bins
    nx, ny, nz, M, T = 48, 40, 6, 7, 2048
    P = T / 256 + 1 / 3
    base = oracle_geometry(nx, ny, nz, M, T, P, 2.0, 2, 12, 2)
    om = np.asarray(kept_bins(base), dtype=np.float64)
    d = (om / om.max()) * np.exp(-2j * np.pi * om * 3.5 / T)
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, P, 2.0, 2, 12, 2, rx_filter=d), iters_min=30, rtol=1e-9)
    plan = Plan(nx, ny, nz, M, T, P, 2.0, 2, 12, 2, g.op_scale, rx_filter=d, precisions=("fp32", "mixed"))
    x = random_volume(g, 51)
    y = random_data(g, 52)
    for prec, tol in (("fp32", TOL32), ("mixed", 5e-3)):
        got = plan.forward(_to_dev(torch_mod, x, torch_mod.float32), precision=prec).cpu().numpy()
        ef = rel_l2(got, oop.forward(g, x))
        got = plan.adjoint(_to_dev(torch_mod, y, torch_mod.complex64), precision=prec).cpu().numpy()
        ea = rel_l2(got, oop.adjoint(g, y))
        _log("receive filter %s: forward rel err %.3e, adjoint rel err %.3e" % (prec, ef, ea))
        assert ef <= tol and ea <= tol


@pytest.mark.parametrize("name", ["parity_32", "ragged", "odd_u", "mid_128"])
def test_precomposed_operator(name, torch_mod):
    """The precomposed-line operator (G = F^T K formed once per plan, the signal
    stage as float32 GEMMs) is the same linear map: A, A^T and the signal stages
    against the oracle's time-domain definition."""
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D = CASES[name]
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D), iters_min=30, rtol=1e-9)
    plan = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, g.op_scale, precisions=("fp32", "precomposed"))
    x = random_volume(g, 61)
    y = random_data(g, 62)
    got = plan.forward(_to_dev(torch_mod, x, torch_mod.float32), precision="precomposed").cpu().numpy()
    ef = rel_l2(got, oop.forward(g, x))
    got = plan.adjoint(_to_dev(torch_mod, y, torch_mod.complex64), precision="precomposed").cpu().numpy()
    ea = rel_l2(got, oop.adjoint(g, y))
    rho = oproj.project(g, x)
    got = plan.signal_fwd(_to_dev(torch_mod, rho, torch_mod.float32), precision="precomposed").cpu().numpy()
    es = rel_l2(got, osig.forward(g, rho.reshape(-1, g.n_u)).reshape(g.n_angles, g.nz, g.n_bins))
    _log("%s precomposed: forward %.3e adjoint %.3e signal %.3e" % (name, ef, ea, es))
    assert ef <= TOL32 and ea <= TOL32 and es <= TOL32

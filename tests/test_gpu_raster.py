"""GPU parity of the raster scan (the zig-zag focus-field sweep: forward on even
z-rows, backward on odd ones, two PSF tables) against the FP64 oracle.

Tolerances: FP32 path within 1e-5 relative L2 of the oracle, mixed operator
within 5e-3 (bf16 gathers, fp16 contractions), mixed refinement within 1e-4
of the FP64 minimiser -- the bars of the one-trajectory scan.
"""
import sys

import numpy as np
import pytest

from oracle import geometry, operator as oop, signal as osig, solvers
from helpers import rel_l2, random_volume, random_data

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_MIX_OP = 5e-3
TOL_MIXED = 1e-4

# name: (nx, ny, nz, M, T, P, w, k_lo, k_hi, D, drive amplitude, sweep S)
CASES = {
    # ragged and odd nz: per angle 3 forward and 2 backward lines, 35 lines
    "raster_odd": (40, 36, 5, 7, 1504, 1504 / 256 + 1 / 3, 2.0, 1, 9, 1, 6.0, 24.0),
    # several line tiles per trajectory class, a drive that covers a quarter of
    # the fast axis and a sweep that carries it across the rest
    "raster_tiles": (64, 48, 20, 9, 4096, 4096 / 256 + 1 / 3, 3.0, 1, 20, 2, 10.0, 40.0),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _geom(name, op_scale=1.0):
    nx, ny, nz, M, T, P, w, klo, khi, D, a, S = CASES[name]
    return geometry.Geometry(nx=nx, ny=ny, nz=nz, n_angles=M, n_t=T, drive_cycles=P, psf_width=w,
                             harm_lo=klo, harm_hi=khi, half_band=D, op_scale=op_scale, drive_amp=a,
                             raster_sweep=S)


def _plan(name, op_scale, precisions=("fp32", "mixed"), sweep=None):
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D, a, S = CASES[name]
    return Plan(nx, ny, nz, M, T, P, w, klo, khi, D, op_scale, drive_amp=a, precisions=precisions,
                raster_sweep=S if sweep is None else sweep)


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_mod):
    _log("case %s" % request.param)
    g = oop.normalised(_geom(request.param), iters_min=30, rtol=1e-9)
    return request.param, g, _plan(request.param, g.op_scale)


def _dev(torch_mod, a, dtype):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _cplx(torch_mod, y):
    return _dev(torch_mod, y, torch_mod.complex64)


def test_raster_forward_parity(case, torch_mod):
    name, g, plan = case
    x = random_volume(g, 1)
    want = oop.forward(g, x)
    xd = _dev(torch_mod, x, torch_mod.float32)
    for prec, tol in (("fp32", TOL32), ("mixed", TOL_MIX_OP)):
        got = plan.forward(xd, precision=prec).cpu().numpy()
        err = rel_l2(got, want)
        _log("%s forward %s rel err %.3e" % (name, prec, err))
        assert err <= tol


def test_raster_adjoint_parity(case, torch_mod):
    name, g, plan = case
    y = random_data(g, 2)
    want = oop.adjoint(g, y)
    yd = _cplx(torch_mod, y)
    for prec, tol in (("fp32", TOL32), ("mixed", TOL_MIX_OP)):
        got = plan.adjoint(yd, precision=prec).cpu().numpy()
        err = rel_l2(got, want)
        _log("%s adjoint %s rel err %.3e" % (name, prec, err))
        assert err <= tol


def test_raster_signal_stages(case, torch_mod):
    """The signal stage alone on random lines: each line through its own
    class's table, in both directions."""
    name, g, plan = case
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((g.n_lines, g.n_u))
    want = osig.forward(g, rho)
    got = plan.signal_fwd(_dev(torch_mod, rho.reshape(g.n_angles, g.nz, g.n_u), torch_mod.float32)).cpu().numpy()
    err_f = rel_l2(got.reshape(g.n_lines, g.n_bins), want)
    y = random_data(g, 4).reshape(g.n_lines, g.n_bins)
    want_a = osig.adjoint(g, y)
    got_a = plan.signal_adj(_cplx(torch_mod, y.reshape(g.n_angles, g.nz, g.n_bins))).cpu().numpy()
    err_a = rel_l2(got_a.reshape(g.n_lines, g.n_u), want_a)
    _log("%s signal stages rel err fwd %.3e adj %.3e" % (name, err_f, err_a))
    assert err_f <= TOL32 and err_a <= TOL32


def test_raster_gpu_adjoint_identity(case, torch_mod):
    name, g, plan = case
    x = random_volume(g, 5)
    y = random_data(g, 6)
    ax = plan.forward(_dev(torch_mod, x, torch_mod.float32)).cpu().numpy().astype(np.complex128)
    aty = plan.adjoint(_cplx(torch_mod, y)).cpu().numpy().astype(np.float64)
    lhs = np.vdot(ax, y.astype(np.complex64).astype(np.complex128)).real
    rhs = float(np.vdot(x.astype(np.float32).astype(np.float64), aty))
    scale = np.linalg.norm(ax) * np.linalg.norm(y)
    _log("%s <Ax,y> %.9e <x,A^T y> %.9e" % (name, lhs, rhs))
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_raster_zero_sweep_is_the_plain_scan(torch_mod):
    """S = 0 builds one table: outputs equal the plain plan's bit for bit."""
    from paper_2511_06627_amd.plan import Plan
    nx, ny, nz, M, T, P, w, klo, khi, D, a, S = CASES["raster_odd"]
    p0 = _plan("raster_odd", 0.7, sweep=0.0)
    pp = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, 0.7, drive_amp=a, precisions=("fp32", "mixed"))
    x = _dev(torch_mod, random_volume(_geom("raster_odd"), 7), torch_mod.float32)
    for prec in ("fp32", "mixed"):
        assert torch_mod.equal(p0.forward(x, precision=prec), pp.forward(x, precision=prec))


def test_raster_precomposed(torch_mod):
    """The precomposed variant (one line matrix per sweep direction, the
    classes' lines as strided GEMMs) against the oracle's time-domain A."""
    name = "raster_odd"
    g = oop.normalised(_geom(name), iters_min=30, rtol=1e-9)
    plan = _plan(name, g.op_scale, precisions=("fp32", "precomposed"))
    x = random_volume(g, 12)
    y = random_data(g, 13)
    ef = rel_l2(plan.forward(_dev(torch_mod, x, torch_mod.float32), precision="precomposed").cpu().numpy(),
                oop.forward(g, x))
    ea = rel_l2(plan.adjoint(_cplx(torch_mod, y), precision="precomposed").cpu().numpy(), oop.adjoint(g, y))
    _log("raster precomposed rel err forward %.3e adjoint %.3e" % (ef, ea))
    assert ef <= TOL32 and ea <= TOL32


def test_raster_device_normalisation(torch_mod):
    """c_A from the device power iteration: the norm is the larger of the two
    sweep directions' slice norms, as the oracle's two-slice iteration finds."""
    g = oop.normalised(_geom("raster_odd"), iters_min=30, rtol=1e-12)
    plan = _plan("raster_odd", 0.0, precisions=("fp32",))
    rel = abs(plan.op_scale - g.op_scale) / g.op_scale
    _log("raster_odd device c_A %.9e (%d its) oracle %.9e rel %.2e"
         % (plan.op_scale, plan.norm_iters, g.op_scale, rel))
    assert rel <= 1e-5


@pytest.fixture(scope="module")
def raster_problem(torch_mod):
    name = "raster_odd"
    g = oop.normalised(_geom(name), iters_min=30, rtol=1e-9)
    rng = np.random.default_rng(8)
    phantom = np.zeros((g.nz, g.ny, g.nx))
    zz, yy, xx = np.meshgrid(*(np.arange(n) for n in phantom.shape), indexing="ij")
    for _ in range(4):
        c = rng.uniform(0.2, 0.8, 3) * np.array(phantom.shape)
        s = rng.uniform(1.5, 4.0)
        amp = 10 ** rng.uniform(-2, 0)
        phantom += amp * np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) / (2 * s * s))
    b, _ = oop.make_data(g, phantom, 0.01, 9)
    lam = 1e-3
    op = oop.Operator(g)
    xs, n = solvers.reference_minimiser(op, b, lam, tol=1e-12)
    return g, _plan(name, g.op_scale), b, lam, xs, n


def test_raster_cgls_and_mixed_refinement_reach_minimiser(raster_problem, torch_mod):
    g, plan, b, lam, xs, n = raster_problem
    bd = _cplx(torch_mod, b)
    x, rep = plan.solve(bd, lam, iters=max(80, n + 20))
    err32 = rel_l2(x.cpu().numpy(), xs)
    xm, repm = plan.solve(bd, lam, precision="mixed", refine_sweeps=5, inner_iters=20)
    errm = rel_l2(xm.cpu().numpy(), xs)
    _log("raster CGLS %d its vs x*: %.3e; mixed 5x20: %.3e (oracle needed %d)"
         % (rep.iters_done, err32, errm, n))
    assert rep.status == 0 and repm.status == 0
    assert err32 <= TOL32 and errm <= TOL_MIXED

"""Mixed-precision path: bf16 projection gathers, fp16 MFMA signal contractions
with fp32 accumulation and power-of-two line and band scaling, refined by FP32
residual sweeps.  Errors are stated per result against the FP64 oracle.

The mixed operator itself carries fp16 rounding (unit roundoff 2^-11 ~ 4.9e-4
on the tables, the scaled operand rows and the time tile, bf16 2^-8 ~ 3.9e-3
on the gathered volume samples, which average down over each ray sum): its
bar is 5e-3 relative L2.  The refined solve is held to the path's 1e-4.
"""
import sys

import numpy as np
import pytest

from oracle import operator as oop, solvers
from paper_2511_06627_amd import configs
from helpers import oracle_geometry, config_geometry, rel_l2, random_volume, random_data

pytestmark = pytest.mark.gpu
TOL_OP16 = 5e-3
TOL_MIXED = 1e-4


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


CASES = {
    "parity_32": (32, 32, 32, 8, 2048, 2048 / 256 + 1 / 3, 2.0, 1, 15, 2),
    "multi_tile": (64, 48, 20, 9, 4096, 4096 / 256 + 1 / 3, 3.0, 1, 20, 2),
    "many_lines": (64, 64, 60, 9, 4096, 4096 / 256 + 1 / 3, 3.0, 1, 20, 2),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_mod):
    from paper_2511_06627_amd.plan import Plan
    _log("mixed case %s" % request.param)
    nx, ny, nz, M, T, P, w, klo, khi, D = CASES[request.param]
    g = oop.normalised(oracle_geometry(nx, ny, nz, M, T, P, w, klo, khi, D), iters_min=30, rtol=1e-9)
    plan = Plan(nx, ny, nz, M, T, P, w, klo, khi, D, g.op_scale, precisions=("fp32", "mixed"))
    return request.param, g, plan


def _dev(torch_mod, a, dtype):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def test_mixed_forward(case, torch_mod):
    name, g, plan = case
    x = random_volume(g, 31)
    got = plan.forward(_dev(torch_mod, x, torch_mod.float32), precision="mixed").cpu().numpy()
    err = rel_l2(got, oop.forward(g, x))
    _log("%s mixed forward rel err %.3e" % (name, err))
    assert err <= TOL_OP16


def test_mixed_adjoint(case, torch_mod):
    name, g, plan = case
    y = random_data(g, 32)
    got = plan.adjoint(_dev(torch_mod, y, torch_mod.complex64), precision="mixed").cpu().numpy()
    err = rel_l2(got, oop.adjoint(g, y))
    _log("%s mixed adjoint rel err %.3e" % (name, err))
    assert err <= TOL_OP16


def test_mixed_adjoint_sees_weak_bands(case, torch_mod):
    """Data confined to the weakest harmonic band: band scaling keeps the fp16
    adjoint accurate even though that band is far below the line maximum."""
    name, g, plan = case
    bw = 2 * g.half_band + 1
    y = np.zeros((g.n_angles, g.nz, g.n_bins), dtype=complex)
    rng = np.random.default_rng(33)
    y[..., -bw:] = 1e-3 * (rng.standard_normal((g.n_angles, g.nz, bw)) + 1j * rng.standard_normal((g.n_angles, g.nz, bw)))
    y[..., :bw] = rng.standard_normal((g.n_angles, g.nz, bw))  # a strong first band on the same lines
    got_full = plan.adjoint(_dev(torch_mod, y, torch_mod.complex64), precision="mixed").cpu().numpy()
    assert rel_l2(got_full, oop.adjoint(g, y)) <= TOL_OP16


def test_mixed_subnormal_rows_stay_finite(case, torch_mod):
    """Lines whose values are subnormal in fp32 (a faint blob's far tail): the
    per-line fp16 scale stays finite, so the outputs do too, and every other
    line keeps its accuracy."""
    name, g, plan = case
    y = random_data(g, 35)
    y[:, 0, :] *= 1e-40
    got = plan.adjoint(_dev(torch_mod, y, torch_mod.complex64), precision="mixed").cpu().numpy()
    assert np.isfinite(got).all()
    want = oop.adjoint(g, y)
    assert rel_l2(got[1:], want[1:]) <= TOL_OP16
    x = random_volume(g, 36)
    x[0] *= 1e-40
    got = plan.forward(_dev(torch_mod, x, torch_mod.float32), precision="mixed").cpu().numpy()
    assert np.isfinite(got).all()
    assert rel_l2(got[:, 1:], oop.forward(g, x)[:, 1:]) <= TOL_OP16


@pytest.fixture(scope="module")
def parity_problem(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.PARITY_32
    g = config_geometry(cfg)
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    b32 = b.astype(np.complex64)
    plan = Plan.from_config(cfg, g.op_scale, precisions=("fp32", "mixed"))
    op = oop.Operator(g, precomposed=True)
    xs, _ = solvers.reference_minimiser(op, b32.astype(np.complex128), cfg.lam, tol=1e-12)
    return cfg, g, plan, op, b32, xs


def test_mixed_refinement_reaches_minimiser(parity_problem, torch_mod):
    """Sweeps of 20 inner mixed iterations, each restarted from the FP32
    residual, converge to the FP64 minimiser: within 1e-4 by the fifth sweep
    (the error after three, the configured schedule, is logged)."""
    cfg, g, plan, op, b32, xs = parity_problem
    bd = torch_mod.from_numpy(b32).cuda()
    errs = {}
    for sweeps in (3, 5):
        x, rep = plan.solve(bd, cfg.lam, precision="mixed", refine_sweeps=sweeps, inner_iters=20)
        errs[sweeps] = rel_l2(x.cpu().numpy(), xs)
        assert rep.status == 0 and rep.iters_done == 20 * sweeps
    _log("parity_32 mixed vs x*: 3x20 %.3e, 5x20 %.3e" % (errs[3], errs[5]))
    assert errs[5] <= TOL_MIXED


def test_mixed_refinement_improves_each_sweep(parity_problem, torch_mod):
    cfg, g, plan, op, b32, xs = parity_problem
    bd = torch_mod.from_numpy(b32).cuda()
    errs = []
    for sweeps in (1, 2, 3):
        x, _ = plan.solve(bd, cfg.lam, precision="mixed", refine_sweeps=sweeps, inner_iters=20)
        errs.append(rel_l2(x.cpu().numpy(), xs))
    _log("parity_32 mixed sweep errors %s" % ["%.2e" % e for e in errs])
    assert errs[2] < errs[0]


def test_mixed_realistic_sampled(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.REALISTIC_192
    _log("mixed case realistic_192x192x96")
    g = config_geometry(cfg)
    plan = Plan.from_config(cfg, g.op_scale, precisions=("fp32", "mixed"))
    x = configs.make_phantom(cfg)
    got = plan.forward(_dev(torch_mod, x, torch_mod.float32), precision="mixed").cpu().numpy()
    gs = g.slice_geometry()
    for k in (7, 60):
        err = rel_l2(got[:, k, :], oop.forward(gs, x[k:k + 1])[:, 0, :])
        _log("realistic mixed forward slice %d rel err %.3e" % (k, err))
        assert err <= TOL_OP16
    y = random_data(g, 34)
    got = plan.adjoint(_dev(torch_mod, y, torch_mod.complex64), precision="mixed").cpu().numpy()
    for k in (11, 90):
        err = rel_l2(got[k], oop.adjoint(gs, y[:, k:k + 1, :])[0])
        _log("realistic mixed adjoint slice %d rel err %.3e" % (k, err))
        assert err <= TOL_OP16

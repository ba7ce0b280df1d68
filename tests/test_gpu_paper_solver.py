"""The paper's own solver on the GPU (eq. iters): fixed-step gradient with the
momentum weight (k-1)/(k+2) and the projection onto x >= 0 every iteration,
with T = I or the finite differences of eq. nummodel, against the oracle's
iteration on the same schedule.

Unlike CGLS, this iteration is a fixed linear map followed by a
non-expansive projection (tau <= 1/L), so operator rounding does not get
amplified: the same-schedule bar is the FP32 path's 1e-5 relative L2.
"""
import sys

import numpy as np
import pytest

from oracle import operator as oop, solvers
from paper_2511_06627_amd import configs
from helpers import config_geometry, rel_l2

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def parity(torch_mod):
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.PARITY_32
    g = config_geometry(cfg)
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    b32 = b.astype(np.complex64)
    plan = Plan.from_config(cfg, g.op_scale)
    return cfg, g, plan, oop.Operator(g, precomposed=True), b32


@pytest.mark.parametrize("reg,lam", [("identity", 1e-3), ("fd", 1e-2)])
def test_momentum_matches_oracle(parity, torch_mod, reg, lam):
    cfg, g, plan, op, b32 = parity
    shape = (g.nz, g.ny, g.nx)
    tau = solvers.paper_tau(1.0, lam, reg, shape)
    bd = torch_mod.from_numpy(b32).cuda()
    for iters in (1, 30):
        want = solvers.momentum_gradient(op, b32.astype(np.complex128), lam, iters, tau, nonneg=True, reg=reg)
        x, rep = plan.solve(bd, lam, iters=iters, solver="momentum", reg=reg, tau=tau, clamp_every=1)
        err = rel_l2(x.cpu().numpy(), want)
        _log("parity_32 momentum %s %d its rel err %.3e" % (reg, iters, err))
        assert rep.status == 0 and err <= TOL32
    # without the projection the iterate may go negative
    want = solvers.momentum_gradient(op, b32.astype(np.complex128), lam, 30, tau, nonneg=False, reg=reg)
    x, _ = plan.solve(bd, lam, iters=30, solver="momentum", reg=reg, tau=tau)
    assert rel_l2(x.cpu().numpy(), want) <= TOL32


def test_momentum_step_from_power_iteration(parity, torch_mod):
    """tau <= 0: the library finds ||A^T A||_2 by power iteration (1 for this
    normalised operator) and uses the paper's tau; the iterate matches the
    run with the closed-form tau."""
    cfg, g, plan, op, b32 = parity
    bd = torch_mod.from_numpy(b32).cuda()
    tau = solvers.paper_tau(1.0, 1e-2, "fd", (g.nz, g.ny, g.nx))
    x1, _ = plan.solve(bd, 1e-2, iters=20, solver="momentum", reg="fd", tau=tau, clamp_every=1)
    x2, _ = plan.solve(bd, 1e-2, iters=20, solver="momentum", reg="fd", tau=0.0, clamp_every=1)
    err = rel_l2(x2.cpu().numpy(), x1.cpu().numpy())
    _log("momentum with power-iteration tau vs closed form: %.3e" % err)
    assert err <= 1e-5


def test_momentum_rejects_unsupported(parity, torch_mod):
    from paper_2511_06627_amd._lib import Mpi3dError
    cfg, g, plan, op, b32 = parity
    bd = torch_mod.from_numpy(b32).cuda()
    with pytest.raises(Mpi3dError):
        plan.solve(bd, 1e-3, iters=5, solver="cgls", reg="fd")


def test_momentum_fd_realistic(torch_mod):
    """The 192 x 192 x 96 scan, FD regulariser, 20 iterations of the paper's
    method against the oracle's."""
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.REALISTIC_192
    _log("case realistic_192x192x96 momentum fd")
    g = config_geometry(cfg)
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    b32 = b.astype(np.complex64)
    plan = Plan.from_config(cfg, g.op_scale)
    lam = 1e-2
    tau = solvers.paper_tau(1.0, lam, "fd", cfg.shape)
    x, rep = plan.solve(torch_mod.from_numpy(b32).cuda(), lam, iters=20, solver="momentum", reg="fd", tau=tau,
                        clamp_every=1)
    want = solvers.momentum_gradient(oop.Operator(g, precomposed=True), b32.astype(np.complex128), lam, 20, tau,
                                     nonneg=True, reg="fd")
    err = rel_l2(x.cpu().numpy(), want)
    _log("realistic momentum fd 20 its rel err %.3e" % err)
    assert rep.status == 0 and err <= TOL32

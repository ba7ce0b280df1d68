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
from helpers import (oracle_geometry, config_geometry, rel_l2, random_volume, random_data, band_errors,
                     band_confined_data, band_table, segment_distance, BAND_TOL32, BAND_TOL16_FWD,
                     BAND_TOL16_ADJ)

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


def _per_band(torch_mod, plan, g, x, y, slices=None, oracle_fwd=None, oracle_adj=None):
    """Per-harmonic relative errors of A (on volume x) and of A^T on band-confined
    data y (slice k holding band k mod n_bands only), both precisions.  With
    `slices`, only those slices are compared (oracle_fwd / oracle_adj give the
    oracle's result for one slice)."""
    bw = 2 * g.half_band + 1
    nbands = g.n_bins // bw
    xd = _dev(torch_mod, x, torch_mod.float32)
    yd = _dev(torch_mod, y, torch_mod.complex64)
    ks = range(g.nz) if slices is None else slices
    want_f = oop.forward(g, x) if slices is None else None
    want_a = oop.adjoint(g, y) if slices is None else None
    rows = {}
    for prec in ("fp32", "mixed"):
        got = plan.forward(xd, precision=prec).cpu().numpy()
        if slices is None:
            rows[prec + " A"] = band_errors(got, want_f, g)
        else:
            rows[prec + " A"] = band_errors(np.stack([got[:, k] for k in ks], 1),
                                            np.stack([oracle_fwd(k) for k in ks], 1), g)
        got = plan.adjoint(yd, precision=prec).cpu().numpy()
        err = np.zeros(nbands)
        for k in ks:
            want_k = want_a[k] if slices is None else oracle_adj(k)
            err[k % nbands] = max(err[k % nbands], rel_l2(got[k], want_k))
        rows[prec + " A^T"] = err
    return rows


def _check_bands(rows):
    assert np.all(rows["fp32 A"] <= BAND_TOL32) and np.all(rows["fp32 A^T"] <= BAND_TOL32)
    assert np.all(rows["mixed A"] <= BAND_TOL16_FWD)
    assert np.all(rows["mixed A^T"] <= BAND_TOL16_ADJ)


def test_per_band_errors(case, torch_mod):
    """Every harmonic band on its own: A's output per band, and A^T of data
    confined to one band (no strong band beside it to hide in), FP32 and
    mixed, against the oracle."""
    name, g, plan = case
    y, band = band_confined_data(g, 33)
    assert len(set(band)) == g.n_bins // (2 * g.half_band + 1), "every band needs a slice"
    rows = _per_band(torch_mod, plan, g, random_volume(g, 31), y)
    _log(band_table(name, rows, g.harm_lo))
    _check_bands(rows)


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


def test_mixed_realistic_per_band(torch_mod):
    """Per-harmonic errors on the 192x192x96 scan (phantom volume for A; data
    confined to band k mod 31 on slice k for A^T), sampled slices."""
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.REALISTIC_192
    _log("mixed case realistic_192x192x96 per band")
    g = config_geometry(cfg)
    gs = g.slice_geometry()
    plan = Plan.from_config(cfg, g.op_scale, precisions=("fp32", "mixed"))
    x = configs.make_phantom(cfg)
    y, band = band_confined_data(g, 37)
    opc = oop.Operator(gs, precomposed=True)
    mass = x.sum(axis=(1, 2))
    fwd_slices = (int(np.argmax(mass)), 7)
    rows = _per_band(torch_mod, plan, g, x, y, slices=list(range(31)),
                     oracle_fwd=lambda k: opc.forward(x[k:k + 1])[:, 0, :],
                     oracle_adj=lambda k: opc.adjoint(y[:, k:k + 1, :])[0])
    # A on the phantom: the organ's middle slice and one through blobs only
    got = {p: plan.forward(_dev(torch_mod, x, torch_mod.float32), precision=p).cpu().numpy() for p in ("fp32", "mixed")}
    for p in ("fp32", "mixed"):
        rows[p + " A"] = band_errors(np.stack([got[p][:, k] for k in fwd_slices], 1),
                                     np.stack([opc.forward(x[k:k + 1])[:, 0, :] for k in fwd_slices], 1), g)
    _log(band_table(cfg.name, rows, g.harm_lo))
    _check_bands(rows)


def test_mixed_realistic_3x20(torch_mod):
    """The configured mixed schedule on the 192x192x96 scan: 3 refinement
    sweeps of 20 inner iterations, against the same schedule's oracle clusters
    (tests/golden/cgls_clusters.json: sweep residuals at the FP32 operator's
    error level, inner operator at the two ends of the mixed operator's range),
    within 4 cluster radii of the segment between their means on the sample
    voxels; the error against the FP64 minimiser x* is stated beside it."""
    import json
    import os
    from paper_2511_06627_amd.plan import Plan
    cfg, m2 = configs.REALISTIC_192, configs.MIXED_192
    _log("mixed case realistic_192x192x96 3x20")
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cgls_clusters.json")))
    g = config_geometry(cfg)
    assert abs(ref["op_scale"] - g.op_scale) <= 1e-9 * g.op_scale
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    plan = Plan.from_config(cfg, g.op_scale, precisions=("fp32", "mixed"))
    x, rep = plan.solve(torch_mod.from_numpy(b.astype(np.complex64)).cuda(), m2.lam, precision="mixed",
                        refine_sweeps=m2.refine_sweeps, inner_iters=m2.inner_iters)
    assert rep.status == 0
    idx = np.array(ref["sample_index"])
    got = x.cpu().numpy().ravel()[idx]
    lo, hi = ref["mixed3x20"]["lo"], ref["mixed3x20"]["hi"]
    err = segment_distance(got, lo["sample_mean"], hi["sample_mean"])
    xs = np.array(ref["xstar"]["sample"])
    ex = float(np.linalg.norm(got - xs) / np.linalg.norm(xs))
    tol = ref["mixed3x20"]["bar_radii"] * max(lo["radius"], hi["radius"])
    _log("realistic mixed 3x20: GPU to the cluster path %.3e (radii %.3e / %.3e, bar %.3e); GPU vs x* %.3e on the "
         "sample (cluster means vs x* over the volume %.3e / %.3e)" % (err, lo["radius"], hi["radius"], tol, ex,
                                                                        lo["mean_to_xstar_full"],
                                                                        hi["mean_to_xstar_full"]))
    assert err <= tol

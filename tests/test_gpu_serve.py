"""Serving on the GPU: batched steps, bitwise batch invariance, admission, end-to-end loop."""
import sys

import numpy as np
import pytest

from oracle import operator as oop, solvers
from helpers import oracle_geometry, rel_l2

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


# Line-table classes (n_u, T, bands, raster sweep S, drive axes, tensor-PSF
# rows R): A-class geometries differ in nz / M but share line tables; B has
# another T; the R-class raster scans (two PSF tables each, odd and even nz)
# share theirs; D1 is a dual-drive scan (x- and z-drive lines); the T-class
# tensor-PSF scans (R + 1 symmetric passes, their line sums in each request's
# own workspace) share theirs, one with both drives.
GEOS = {
    "A1": (48, 48, 12, 6, 2048, 1, 12, 2, 0.0, 1, 0),
    "A2": (48, 48, 20, 9, 2048, 1, 12, 2, 0.0, 1, 0),
    "B1": (64, 64, 16, 8, 4096, 1, 16, 3, 0.0, 1, 0),
    "R1": (48, 48, 7, 5, 2048, 1, 12, 2, 20.0, 1, 0),
    "R2": (48, 48, 10, 6, 2048, 1, 12, 2, 20.0, 1, 0),
    "D1": (48, 48, 12, 5, 2048, 1, 12, 2, 0.0, 2, 0),
    "T1": (48, 48, 9, 5, 2048, 1, 12, 2, 0.0, 1, 2),
    "T2": (48, 48, 13, 4, 2048, 1, 12, 2, 0.0, 1, 2),
    "T3": (48, 48, 11, 4, 2048, 1, 12, 2, 0.0, 2, 2),
}


def _request(name, seed):
    nx, ny, nz, M, T, klo, khi, D, S, axes, R = GEOS[name]
    P = T / 256 + 1 / 3
    a = 8.0 if S else 0.0          # a raster scan's drive covers a third of the fast axis
    g = oracle_geometry(nx, ny, nz, M, T, P, 3.0, klo, khi, D)
    if S:
        g.drive_amp, g.raster_sweep = a, S
    if axes == 2:
        g.drive_axes, g.drive_amp_z = 2, nz / 2.0
    g.psf_rows = R
    g = oop.normalised(g, iters_min=30, rtol=1e-9)
    x = np.random.default_rng(seed).uniform(0, 1, (nz, ny, nx))
    b = oop.forward(g, x).astype(np.complex64)
    geo = dict(nx=nx, ny=ny, nz=nz, n_angles=M, n_t=T, drive_cycles=P, psf_width=3.0, harm_lo=klo, harm_hi=khi,
               half_band=D, op_scale=g.op_scale, drive_amp=a, raster_sweep=S, drive_axes=axes, psf_rows=R)
    return g, geo, b


@pytest.fixture(scope="module")
def reqs(torch_mod):
    return {k: _request(k, i) for i, k in enumerate(GEOS)}


def _run_states(torch_mod, plans, names, reqs, schedule, steps_cap=200):
    from paper_2511_06627_amd.plan import State, batch_step
    states = {}
    for n in names:
        g, geo, b = reqs[n]
        states[n] = State(plans[n], torch_mod.from_numpy(b).cuda(), 1e-3, **schedule)
    for _ in range(steps_cap):
        live = [s for s in states.values() if not s.progress()[1]]
        if not live:
            break
        batch_step(live)
    torch_mod.cuda.synchronize()
    return {n: s.x.clone() for n, s in states.items()}


@pytest.fixture(scope="module")
def plans(torch_mod, reqs):
    from paper_2511_06627_amd.plan import Plan
    return {k: Plan(precisions=("fp32", "mixed"), **reqs[k][1]) for k in GEOS}


@pytest.mark.parametrize("schedule", [dict(precision="fp32", iters=6),
                                      dict(precision="mixed", refine_sweeps=2, inner_iters=3),
                                      dict(precision="fp32", iters=6, clamp_every=2)])
def test_batch_invariance_bitwise(torch_mod, plans, reqs, schedule):
    """A request's result is bitwise the same alone and batched with others."""
    _log("serve invariance %s" % schedule)
    alone = {n: _run_states(torch_mod, plans, [n], reqs, schedule)[n] for n in GEOS}
    mixed = _run_states(torch_mod, plans, list(GEOS), reqs, schedule)
    for n in GEOS:
        assert torch_mod.equal(alone[n], mixed[n]), n


def test_served_solve_matches_oracle(torch_mod, plans, reqs):
    out = _run_states(torch_mod, plans, list(GEOS), reqs, dict(precision="fp32", iters=3))
    for n in GEOS:
        g, geo, b = reqs[n]
        want = solvers.cgls(oop.Operator(g, precomposed=True), b.astype(np.complex128), 1e-3, 3)
        err = rel_l2(out[n].cpu().numpy(), want)
        _log("served %s cgls 3 rel err %.3e" % (n, err))
        assert err <= 1e-5


def test_continuous_batching_loop(torch_mod, reqs):
    """End to end: a burst of requests, admission under a small forced budget
    (every geometry's plan tables plus room for about two requests), results
    equal to the same requests solved alone."""
    from paper_2511_06627_amd.serve import ContinuousBatcher, GpuExecutor, Request, summarize
    rng = np.random.default_rng(3000)
    names = ["A1", "B1", "R1", "T1", "A2", "D1", "T3", "R2", "A1", "T2", "B1", "A2"]
    sched = dict(precision="mixed", refine_sweeps=2, inner_iters=4)
    rq = []
    t = 0.0
    for i, n in enumerate(names):
        t += rng.exponential(1e-4)          # a burst: all arrive before the first can finish
        g, geo, b = reqs[n]
        rq.append(Request(i, t, geo, b, 1e-3, sched))
    ex = GpuExecutor()
    fps = [ex.footprint(r) for r in rq]
    tables = {ex.plan_key(r): ex.plan_bytes(r) for r in rq}
    budget = int(sum(tables.values()) + 2.2 * max(fps))     # plans, and room for about two requests
    bat = ContinuousBatcher(ex, budget_bytes=budget, max_active=8)
    out = bat.run(rq)
    s = summarize(out)
    _log("serve loop: %s (peak %d of %d bytes)" % (s, bat.peak_bytes, budget))
    # charged bytes (plans and live requests, held until each copy-out
    # closed its state) never above the budget, and the budget did bind:
    # some request was admitted only after another was done
    assert bat.peak_bytes <= budget
    events = [ev for _, ev, _ in bat.log]
    assert "admit" in events[events.index("done"):]
    from paper_2511_06627_amd.plan import Plan
    for r, o in zip(rq, out):
        p = Plan(precisions=("fp32", "mixed"), **r.geometry)
        alone = _run_states(torch_mod, {"x": p}, ["x"], {"x": (None, r.geometry, r.b)}, sched)["x"]
        assert np.array_equal(o.x, alone.cpu().numpy()), r.rid

"""Scheduler logic of the serving loop, on the CPU with a fake executor.

The fake executor runs each request's CGLS on the FP64 oracle, one iteration
per tick, so the test also checks that every request ends with its own
solution no matter what it was batched with.
"""
import numpy as np
import pytest

from oracle import operator as oop, solvers
from oracle.geometry import Geometry
from paper_2511_06627_amd.serve import ContinuousBatcher, Request, summarize, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class OracleExecutor:
    """One oracle CGLS iteration per tick; each tick costs `tick_s` of clock."""

    def __init__(self, clock, tick_s=0.01, fp_of=None, plan_bytes_of=None):
        self.clock = clock
        self.tick_s = tick_s
        self.fp_of = fp_of or (lambda r: 100)
        self.plan_bytes_of = plan_bytes_of or (lambda r: 0)
        self.batches = []
        self.copies = 0
        self.released = []

    def footprint(self, r):
        return self.fp_of(r)

    def plan_key(self, r):
        return tuple(sorted(r.geometry.items()))

    def plan_bytes(self, r):
        return self.plan_bytes_of(r)

    def release_plan(self, key):
        self.released.append(key)

    def admit(self, r):
        g = Geometry(**r.geometry)
        return {"r": r, "op": oop.Operator(g, precomposed=True), "it": 0, "x": None}

    def step(self, handles):
        self.batches.append([h["r"].rid for h in handles])
        for h in handles:
            h["it"] += 1
        self.clock.t += self.tick_s

    def done(self, h):
        return h["it"] >= h["r"].schedule["iters"]

    def start_copy_out(self, h):
        r = h["r"]
        h["x"] = solvers.cgls(h["op"], r.b, r.lam, r.schedule["iters"])
        return h

    def poll_copy_out(self, token):
        # the copy takes one poll to finish: the state (and its footprint)
        # stays live for one more tick after it retires
        self.copies += 1
        if not token.get("copied"):
            token["copied"] = True
            return None
        return token["x"]

    def steps(self, token):
        return token["it"]


def _geometry(n, m, seed):
    return dict(nx=n, ny=n, nz=2, n_angles=m, n_t=512, drive_cycles=512 / 256 + 1 / 3 + 2, psf_width=1.5,
                harm_lo=1, harm_hi=4, half_band=1, op_scale=0.5 + 0.1 * seed)


def _requests(k, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(k):
        t += rng.exponential(0.02)
        geo = _geometry(int(rng.choice([8, 12])), int(rng.choice([3, 4])), i)
        g = Geometry(**geo)
        x = rng.uniform(0, 1, (g.nz, g.ny, g.nx))
        b = oop.forward(g, x)
        out.append(Request(i, t, geo, b, 1e-3, {"iters": int(rng.integers(3, 7))}))
    return out


def test_all_requests_complete_with_their_own_solution():
    clock = FakeClock()
    ex = OracleExecutor(clock)
    reqs = _requests(9)
    out = ContinuousBatcher(ex, budget_bytes=10 ** 6, max_active=4, clock=clock, sleep=clock.sleep).run(reqs)
    assert [o.rid for o in out] == list(range(9))
    for r, o in zip(reqs, out):
        want = solvers.cgls(oop.Operator(Geometry(**r.geometry), precomposed=True), r.b, r.lam, r.schedule["iters"])
        assert np.array_equal(o.x, want)
        assert o.steps == r.schedule["iters"]
        assert o.done_s >= o.admit_s >= o.arrival_s


def test_requests_arriving_mid_run_join_the_batch():
    clock = FakeClock()
    ex = OracleExecutor(clock)
    ContinuousBatcher(ex, budget_bytes=10 ** 6, max_active=8, clock=clock, sleep=clock.sleep).run(_requests(9))
    # some tick must carry requests admitted at different times
    sizes = [len(b) for b in ex.batches]
    assert max(sizes) >= 2
    firsts = {}
    for t, b in enumerate(ex.batches):
        for rid in b:
            firsts.setdefault(rid, t)
    assert any(len({firsts[rid] for rid in b}) >= 2 for b in ex.batches)


def test_admission_respects_budget_and_slots():
    clock = FakeClock()
    ex = OracleExecutor(clock, fp_of=lambda r: 60)
    bat = ContinuousBatcher(ex, budget_bytes=130, max_active=8, clock=clock, sleep=clock.sleep)
    bat.run(_requests(7))
    assert max(len(b) for b in ex.batches) <= 2          # 130 bytes hold two 60-byte requests
    clock2 = FakeClock()
    ex2 = OracleExecutor(clock2)
    ContinuousBatcher(ex2, budget_bytes=10 ** 6, max_active=3, clock=clock2, sleep=clock2.sleep).run(_requests(7))
    assert max(len(b) for b in ex2.batches) <= 3


def test_oversized_request_rejected():
    clock = FakeClock()
    ex = OracleExecutor(clock, fp_of=lambda r: 1000)
    with pytest.raises(ValueError):
        ContinuousBatcher(ex, budget_bytes=999, clock=clock, sleep=clock.sleep).run(_requests(2))


def test_fcfs_order_and_summary():
    clock = FakeClock()
    ex = OracleExecutor(clock, fp_of=lambda r: 60)
    bat = ContinuousBatcher(ex, budget_bytes=60, max_active=8, clock=clock, sleep=clock.sleep)
    out = bat.run(_requests(5))
    admits = [rid for _, ev, rid in bat.log if ev == "admit"]
    assert admits == sorted(admits)
    s = summarize(out)
    assert s["requests"] == 5 and s["p99_s"] >= s["p50_s"] > 0


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile([5], 99) == 5


def test_plan_tables_are_charged_to_the_budget():
    """Geometries whose plans hold 50 bytes each, requests of 30 bytes, a
    budget of 130: one plan and two requests fit (110), a second geometry's
    request (50 + 30 more) does not until the first geometry's requests are
    gone and its plan is released, so at most 130 bytes are ever in use."""
    clock = FakeClock()
    reqs = _requests(8)
    geos = sorted({tuple(sorted(r.geometry.items())) for r in reqs})
    assert len(geos) >= 2
    ex = OracleExecutor(clock, fp_of=lambda r: 30, plan_bytes_of=lambda r: 50)
    bat = ContinuousBatcher(ex, budget_bytes=130, max_active=8, clock=clock, sleep=clock.sleep)
    out = bat.run(reqs)
    assert len(out) == 8
    assert bat.peak_bytes <= 130
    # with plans charged, two 30-byte requests of two geometries (50 + 50 + 60)
    # never run together
    for b in ex.batches:
        keys = {tuple(sorted(reqs[rid].geometry.items())) for rid in b}
        assert len(keys) == 1 or len(b) <= 1, b
    assert len(ex.released) >= 1
    with pytest.raises(ValueError):
        ContinuousBatcher(OracleExecutor(clock, fp_of=lambda r: 30, plan_bytes_of=lambda r: 101), budget_bytes=130,
                          clock=clock, sleep=clock.sleep).run(reqs[:1])


def test_footprint_held_until_the_copy_out_closes_the_state():
    """A retired request keeps its footprint until its result has left the
    device: with room for one request, the next is admitted only after the
    previous one's copy-out completed."""
    clock = FakeClock()
    ex = OracleExecutor(clock, fp_of=lambda r: 60)
    bat = ContinuousBatcher(ex, budget_bytes=100, max_active=8, clock=clock, sleep=clock.sleep)
    bat.run(_requests(4))
    ev = [(e, rid) for _, e, rid in bat.log]
    for rid in range(1, 4):
        admit = ev.index(("admit", rid))
        assert any(e == "done" for e, _ in ev[:admit]), ev
    assert bat.peak_bytes <= 100

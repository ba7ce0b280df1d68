"""Continuous-batching reconstruction service.

Requests (a scan geometry, its compressed data and a solve schedule) arrive
over time.  The scheduler admits a request when a slot is free and the
request's HBM footprint fits the budget next to the active ones, then, tick
by tick, advances every active solve by one step through one batched call
(``mpi3d_batch_step``: requests of the same line class share their signal
kernel launches).  A request retires when its schedule is complete; its
volume is copied to host memory on a side stream while the next ticks run.

Budget accounting.  A request's footprint (solver workspace, data, volume)
is charged from admission until its state is closed after the copy-out, and
the device tables of each geometry's plan are charged from the admission of
the first request of that geometry while the plan is cached.  When a request
does not fit, cached plans that no live request uses are released (least
recently used first) before it waits.

The scheduling logic is independent of the GPU: it drives an ``executor``
object (``GpuExecutor`` here; tests also drive a CPU one), so admission,
batching and retirement can be exercised without a device.  Executors
provide footprint(r), plan_key(r), plan_bytes(r), release_plan(key), admit,
step, done, start_copy_out, poll_copy_out and steps.
"""
import heapq
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    arrival_s: float          # seconds after the start of the stream
    geometry: dict            # Plan keyword arguments (nx, ny, nz, n_angles, n_t, ...)
    b: object                 # compressed data (numpy complex64, shape (M, nz, nb))
    lam: float
    schedule: dict            # precision, iters / refine_sweeps, inner_iters, clamp_every


@dataclass
class Outcome:
    rid: int
    arrival_s: float
    admit_s: float
    done_s: float
    steps: int
    x: object = None

    @property
    def latency_s(self):
        return self.done_s - self.arrival_s


def percentile(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class ContinuousBatcher:
    """Admission by footprint and slots; one batched step per tick."""

    def __init__(self, executor, budget_bytes, max_active=16, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = budget_bytes
        self.max_active = max_active
        self.clock = clock
        self.sleep = sleep
        self.log = []             # (time, event, rid)

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        for r in pending:
            need = self.ex.footprint(r) + self.ex.plan_bytes(r)
            if need > self.budget:
                raise ValueError("request %d needs %d bytes with its plan, more than the whole budget" % (r.rid, need))
        queue = []                # arrived, waiting: (arrival, rid, request)
        active = {}               # rid -> (handle, request, admit_s, footprint)
        retiring = {}             # rid -> (token, request, admit_s, footprint)
        outcomes = {}
        charged = {}              # plan key -> (table bytes, live requests, last use)
        used = 0
        self.peak_bytes = 0
        t0 = self.clock()
        i = 0
        while i < len(pending) or queue or active or retiring:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival_s <= now:
                heapq.heappush(queue, (pending[i].arrival_s, pending[i].rid, pending[i]))
                i += 1
            # admission, first come first served
            while queue and len(active) < self.max_active:
                r = queue[0][2]
                fp = self.ex.footprint(r)
                key = self.ex.plan_key(r)
                tables = 0 if key in charged else self.ex.plan_bytes(r)
                if used + fp + tables > self.budget:
                    # release idle cached plans, least recently used first
                    idle = sorted((v[2], k) for k, v in charged.items() if v[1] == 0 and k != key)
                    for _, k in idle:
                        if used + fp + tables <= self.budget:
                            break
                        used -= charged.pop(k)[0]
                        self.ex.release_plan(k)
                        self.log.append((self.clock() - t0, "release_plan", -1))
                    if used + fp + tables > self.budget:
                        break
                heapq.heappop(queue)
                used += fp + tables
                nb, live, _ = charged.get(key, (tables, 0, 0))
                charged[key] = (nb, live + 1, self.clock() - t0)
                self.peak_bytes = max(self.peak_bytes, used)
                active[r.rid] = (self.ex.admit(r), r, self.clock() - t0, fp)
                self.log.append((self.clock() - t0, "admit", r.rid))
            if active:
                self.ex.step([h for h, _, _, _ in active.values()])
                for rid in list(active):
                    h, r, admit_s, fp = active[rid]
                    if self.ex.done(h):
                        del active[rid]
                        self.log.append((self.clock() - t0, "retire", rid))
                        retiring[rid] = (self.ex.start_copy_out(h), r, admit_s, fp)
            for rid in list(retiring):
                token, r, admit_s, fp = retiring[rid]
                x = self.ex.poll_copy_out(token)      # closes the state once the copy is done
                if x is not None:
                    del retiring[rid]
                    used -= fp
                    key = self.ex.plan_key(r)
                    nb, live, last = charged[key]
                    charged[key] = (nb, live - 1, last)
                    t = self.clock() - t0
                    outcomes[rid] = Outcome(rid, r.arrival_s, admit_s, t, self.ex.steps(token), x)
                    self.log.append((t, "done", rid))
            if not active and not retiring and i < len(pending) and not queue:
                # idle until the next arrival
                self.sleep(max(0.0, pending[i].arrival_s - (self.clock() - t0)))
        return [outcomes[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(outcomes):
    lat = [o.latency_s for o in outcomes]
    span = max(o.done_s for o in outcomes) - min(o.arrival_s for o in outcomes)
    return {"requests": len(outcomes), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "mean_s": sum(lat) / len(lat), "span_s": span, "solves_per_s": len(outcomes) / span}


class GpuExecutor:
    """Executor over libmpi3d: plans cached by geometry, one State per request."""

    def __init__(self, device=0, precisions=("fp32", "mixed")):
        import torch
        from .plan import Plan  # noqa: F401  (fails loudly without the library)
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.precisions = precisions
        self.plans = {}
        self.stream = torch.cuda.current_stream(self.device)
        self.copy_stream = torch.cuda.Stream(device=self.device)

    def _plan(self, geometry):
        from .plan import Plan
        key = tuple(sorted(geometry.items()))
        if key not in self.plans:
            self.plans[key] = Plan(precisions=self.precisions, **geometry)
        return self.plans[key]

    def footprint(self, r):
        """Device bytes of one request: its solver workspace, data and volume
        (plan tables are shared by the requests of one geometry: plan_bytes)."""
        p = self._plan(r.geometry)
        return int(p.info.solve_ws_bytes) + 4 * int(p.info.n_data_floats) + 4 * int(p.info.n_vox)

    def plan_key(self, r):
        return tuple(sorted(r.geometry.items()))

    def plan_bytes(self, r):
        """Device bytes held by the plan of the request's geometry (its tables)."""
        return int(self._plan(r.geometry).info.table_bytes)

    def release_plan(self, key):
        p = self.plans.pop(key, None)
        if p is not None:
            self.torch.cuda.synchronize(self.device)
            p.close()

    def admit(self, r):
        from .plan import State
        torch = self.torch
        p = self._plan(r.geometry)
        b = torch.from_numpy(r.b).to(self.device, non_blocking=False)
        s = r.schedule
        st = State(p, b, r.lam, precision=s.get("precision", "fp32"), iters=s.get("iters", 0),
                   refine_sweeps=s.get("refine_sweeps", 0), inner_iters=s.get("inner_iters", 0),
                   clamp_every=s.get("clamp_every", 0))
        return {"state": st, "b": b}

    def step(self, handles):
        from .plan import batch_step
        batch_step([h["state"] for h in handles], stream=self.stream)

    def done(self, h):
        return h["state"].progress()[1]

    def start_copy_out(self, h):
        torch = self.torch
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.copy_stream.wait_event(ev)
        with torch.cuda.stream(self.copy_stream):
            host = torch.empty(h["state"].x.shape, dtype=torch.float32, pin_memory=True)
            host.copy_(h["state"].x, non_blocking=True)
            done = torch.cuda.Event()
            done.record(self.copy_stream)
        return {"h": h, "host": host, "event": done, "steps": h["state"].progress()[0]}

    def poll_copy_out(self, token):
        if not token["event"].query():
            return None
        x = token["host"].numpy().copy()
        token["h"]["state"].close()
        return x

    def steps(self, token):
        return token["steps"]

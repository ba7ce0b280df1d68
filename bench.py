"""Benchmark of the compressed 3D FFL operator on one MI355X.

Default run (python bench.py [--steps K] [--warmup W]):
  workload  the realistic scan: 192 x 192 x 96 voxels, 36 FFL angles,
            96 lines x 8192 time samples per angle, harmonics 1-31 +/- 3 bins
  step      one application of A followed by A^T (mpi3d_forward then
            mpi3d_adjoint), FP32 path, inputs resident in HBM
  value     A^T A applications per second (K steps timed between two device
            synchronisations)
Also reported: per-kernel device times from HIP events and the roofline of
the dominant kernel (with HBM traffic from the committed counter summary while
the kernel sources are unchanged); the mixed-precision and precomposed-line
operators; the CGLS iteration rate; the paper's own solver; time-to-solve at
1e-4 relative error against the FP64 minimiser (32^3 and the realistic scan,
FP32 and mixed); the high-dynamic-range scan in both precisions against the
oracle's stored solve; the serving stream (p50/p99) and closed-loop capacity
at 1e-4; and the FP64 CPU oracle timed on this host (cpu_baseline leg).

Time-to-solve on the realistic scan needs its FP64 minimiser from the oracle
(about a minute of host CPU); --no-tts skips it.
One GPU only: --gpus N with N > 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP16_PEAK_TFLOPS = 2500.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU leg: the FP64 oracle.  Everything that touches oracle/ lives here: the
# workload's normalisation constant and data (inputs for the GPU leg), the
# FP64 minimisers that time-to-solve is measured against, and the timed
# oracle A^T A applications (cpu_baseline).
# ---------------------------------------------------------------------------
def cpu_baseline_leg(cfg, want_minimiser=False, sample_seconds=15.0, small_cfg=None):
    import numpy as np
    from oracle import operator as oop, solvers
    from oracle.geometry import Geometry

    def geom(c):
        g = Geometry(nx=c.nx, ny=c.ny, nz=c.nz, n_angles=c.n_angles, n_t=c.n_t, drive_cycles=c.drive_cycles,
                     psf_width=c.psf_width, harm_lo=c.harm_lo, harm_hi=c.harm_hi, half_band=c.half_band)
        return oop.normalised(g, iters_min=30, rtol=1e-9)

    from paper_2511_06627_amd import configs
    out = {}
    t0 = time.time()
    g = geom(cfg)
    phantom = configs.make_phantom(cfg)
    b, _ = oop.make_data(g, phantom, cfg.noise, cfg.noise_seed)
    out["op_scale"] = g.op_scale
    out["b"] = b.astype(np.complex64)
    out["phantom"] = phantom
    log("oracle setup %.1fs" % (time.time() - t0))

    # timed oracle A^T A at the full workload (time-domain path, as defined)
    op = oop.Operator(g)
    x = phantom
    n = 0
    t0 = time.time()
    while True:
        x = op.adjoint(op.forward(x))
        x /= np.linalg.norm(x)
        n += 1
        if n >= 2 and time.time() - t0 >= sample_seconds:
            break
    dt = time.time() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out["cpu_baseline"] = {"value": n / dt, "unit": "A^T A applies/s", "cores": threads, "kind": "oracle",
                           "sample": "%d applications of A then A^T (FP64 time-domain oracle, C projector with "
                                     "OpenMP, BLAS contractions) at the full %s workload, %.1f s"
                                     % (n, cfg.name, dt)}
    log("oracle A^T A: %.3f /s on %d threads" % (n / dt, threads))

    if small_cfg is not None:
        gs = geom(small_cfg)
        ph = configs.make_phantom(small_cfg)
        bs, _ = oop.make_data(gs, ph, small_cfg.noise, small_cfg.noise_seed)
        bs = bs.astype(np.complex64)
        # oracle beside the GPU on the small scan: A^T A rate (time-domain form)
        # and the configured CGLS solve
        ops = oop.Operator(gs)
        n, t0 = 0, time.time()
        while n < 3 or time.time() - t0 < 2.0:
            ops.adjoint(ops.forward(ph))
            n += 1
        t_small = (time.time() - t0) / n
        t0 = time.time()
        solvers.cgls(ops, bs.astype(np.complex128), small_cfg.lam, small_cfg.iters)
        out["oracle_small"] = {"workload": small_cfg.name, "AtA_per_s": round(1.0 / t_small, 2),
                               "cgls_%d_seconds" % small_cfg.iters: round(time.time() - t0, 3)}
        xs, it = solvers.reference_minimiser(oop.Operator(gs, precomposed=True), bs.astype(np.complex128),
                                             small_cfg.lam, tol=1e-12)
        out["small"] = {"op_scale": gs.op_scale, "b": bs, "xstar": xs, "xstar_iters": it}
    if want_minimiser:
        t0 = time.time()
        xs, it = solvers.reference_minimiser(oop.Operator(g, precomposed=True), out["b"].astype(np.complex128),
                                             cfg.lam, tol=1e-9)
        out["xstar"], out["xstar_iters"] = xs, it
        log("oracle minimiser: %d CGLS iterations, %.1fs" % (it, time.time() - t0))
    return out


def oracle_hdr_inputs():
    """c_A and data of the high-dynamic-range scan from the oracle (same
    recipe as its stored FP64 solve in tests/golden/hdr_reference.json)."""
    import numpy as np
    from oracle import operator as oop
    from oracle.geometry import Geometry
    from paper_2511_06627_amd import configs
    c = configs.HDR_256
    g = Geometry(nx=c.nx, ny=c.ny, nz=c.nz, n_angles=c.n_angles, n_t=c.n_t, drive_cycles=c.drive_cycles,
                 psf_width=c.psf_width, harm_lo=c.harm_lo, harm_hi=c.harm_hi, half_band=c.half_band)
    g = oop.normalised(g, iters_min=30, rtol=1e-9)
    b, _ = oop.make_data(g, configs.make_phantom(c), c.noise, c.noise_seed)
    # one oracle A^T A at this size, on its precomposed per-line form (the
    # time-domain form takes minutes per application here); labelled so
    op = oop.Operator(g, precomposed=True)
    x = np.ones((c.nz, c.ny, c.nx))
    t0 = time.time()
    op.adjoint(op.forward(x))
    t_ata = time.time() - t0
    return {"op_scale": g.op_scale, "b": b.astype(np.complex64),
            "oracle": {"workload": c.name, "AtA_per_s_precomposed": round(1.0 / t_ata, 4)}}


# ---------------------------------------------------------------------------
# GPU leg
# ---------------------------------------------------------------------------
def signal_flops(cfg):
    """Algorithmic flops of one signal contraction (forward or adjoint) over all lines:
    2 L (Nu T + 2 nb T): the PSF contraction plus the band DFT, real arithmetic."""
    L = cfg.n_lines
    return 2.0 * L * (cfg.n_u * cfg.n_t + 2 * cfg.n_bins * cfg.n_t)


def projection_bytes(cfg):
    """Per-angle-stream byte model of one projection: every angle reads the whole
    volume once and writes its lines (fp32)."""
    nvox = cfg.nx * cfg.ny * cfg.nz
    return 4.0 * (cfg.n_angles * nvox + cfg.n_lines * cfg.n_u)


def step_times(torch, step, n=20):
    """Per-step device times (ms) from events on the current stream: median and p99."""
    import numpy as np
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for e0, e1 in ev:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    ts = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return {"median": round(float(np.median(ts)), 4), "p99": round(float(np.percentile(ts, 99)), 4), "n": n}


def kernel_source_hash():
    """sha256 over the library's kernel and launch sources: HBM traffic taken
    from counters is only valid for the code it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2511_06627_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".cpp", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings),
    or None when the sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


def time_to_solve(plan, torch, b, xstar, lam, precision="fp32"):
    """Cheapest schedule whose result is within 1e-4 relative L2 of x*, and the
    wall time of a solve with it (median of 3, device synchronised).  FP32:
    iteration counts in steps of 5; mixed: the refinement schedules in
    MIXED_CANDIDATES, in order of total iterations."""
    import numpy as np
    bd = torch.from_numpy(b).cuda()
    xn = np.linalg.norm(xstar)
    if precision == "fp32":
        cands = [dict(iters=i) for i in range(5, 401, 5)]
    else:
        cands = [dict(precision="mixed", refine_sweeps=sw, inner_iters=n) for sw, n in MIXED_CANDIDATES]
    hit = None
    errs = []
    for kw in cands:
        x, _ = plan.solve(bd, lam, report=False, **kw)
        err = float(np.linalg.norm(x.cpu().numpy() - xstar) / xn)
        errs.append(err)
        if err <= 1e-4:
            hit = kw
            break
    if hit is None:
        return {"schedule": None, "seconds": None, "errors": errs}
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(bd, lam, report=False, **hit)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return {"schedule": hit, "seconds": round(sorted(ts)[1], 5), "rel_err": errs[-1]}


def hdr_leg(torch, inputs):
    """The high-dynamic-range scan, FP32 (100 CGLS iterations, clamp + restart
    every 10) and mixed (10 sweeps of 10, clamp after each): solve time, and
    the faint blobs' recovered amplitudes against the FP64 oracle's solve."""
    import numpy as np
    from paper_2511_06627_amd import configs, phantoms
    from paper_2511_06627_amd.plan import Plan
    cfg = configs.HDR_256
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "hdr_reference.json")))
    plan = Plan.from_config(cfg, inputs["op_scale"], precisions=("fp32", "mixed"))
    bd = torch.from_numpy(inputs["b"]).cuda()
    idx = np.array(ref["sample_index"])
    want = np.array(ref["sample_value"])
    amp_ref = np.array([bl["amp_oracle"] for bl in ref["blobs"]])
    amp_true = np.array([bl["amp_true"] for bl in ref["blobs"]])
    profiles = [phantoms._blob(cfg.shape, bl["centre_xyz"], bl["sigma"], 1.0) for bl in ref["blobs"]]
    out = {"workload": "hdr_256x256x128: 60 angles, 128 lines x 16384 samples, harmonics 1-47 +/-3, "
                       "bright ellipsoid + 30 faint blobs (1e-4..1e-2), 0.1% noise"}
    schedules = {"fp32": dict(iters=cfg.iters, clamp_every=cfg.clamp_every),
                 "mixed": dict(precision="mixed", refine_sweeps=cfg.iters // cfg.clamp_every,
                               inner_iters=cfg.clamp_every, clamp_every=cfg.clamp_every)}
    for prec, kw in schedules.items():
        plan.solve(bd, cfg.lam, report=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, rep = plan.solve(bd, cfg.lam, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xn = x.cpu().numpy().astype(np.float64)
        amp = np.array([float(np.vdot(xn, gb) / np.vdot(gb, gb)) for gb in profiles])
        out[prec] = {"schedule": kw, "seconds": round(dt, 4), "status": rep.status,
                     "samples_rel_l2_vs_oracle": float(np.linalg.norm(xn.ravel()[idx] - want) / np.linalg.norm(want)),
                     "faint_amp_max_rel_err_vs_oracle": float(np.max(np.abs(amp - amp_ref) / np.abs(amp_ref))),
                     "faint_amp_median_rel_err_vs_oracle": float(np.median(np.abs(amp - amp_ref) / np.abs(amp_ref))),
                     "faint_amp_recovered_over_true_median": float(np.median(amp / amp_true))}
        log("hdr %s: %s" % (prec, out[prec]))
    out["oracle_envelope"] = ref["envelope"]
    out["oracle_timing"] = inputs["oracle"]
    return out


# ---------------------------------------------------------------------------
# Serving leg: the request stream, solved by the continuous batcher
# ---------------------------------------------------------------------------
# Refinement schedules (sweeps, inner iterations), in order of cost: a sweep's
# FP32 restart costs about two mixed iterations.
MIXED_CANDIDATES = ((2, 25), (2, 30), (3, 20), (2, 35), (3, 25), (4, 20), (3, 30), (4, 25), (3, 40), (5, 30),
                    (6, 30))


def device_data(torch, plan, phantom, noise, seed):
    """b = A x_phantom by the plan's FP32 operator, plus complex Gaussian noise
    in the kept bins, standard deviation noise * max|b| per bin (seeded)."""
    import numpy as np
    x = torch.from_numpy(phantom).float().cuda()
    b = plan.forward(x).cpu().numpy()
    nrng = np.random.default_rng(seed)
    sigma = noise * float(np.abs(b).max())
    b = b + sigma / np.sqrt(2.0) * (nrng.standard_normal(b.shape) + 1j * nrng.standard_normal(b.shape))
    return b.astype(np.complex64)


def serve_requests(torch, n_requests):
    """The seeded request stream: Poisson arrivals, geometry classes drawn
    uniformly, each request's data made on the device.

    Data: b = A x_phantom by the FP32 operator of the request's plan (c_A
    estimated by the plan, op_scale = 0), plus complex Gaussian noise in the
    kept bins with standard deviation (noise level) x max|b| per bin, drawn
    from the request's own seed.  Returns (requests, plans, build seconds)."""
    import numpy as np
    from paper_2511_06627_amd import configs
    from paper_2511_06627_amd.plan import Plan
    from paper_2511_06627_amd.serve import Request
    rng = np.random.default_rng(configs.SERVE_ARRIVAL_SEED)
    draws = []
    t = 0.0
    for i in range(n_requests):
        t += rng.exponential(1.0 / configs.SERVE_RATE_HZ)
        vol = configs.SERVE_VOLUMES[rng.integers(len(configs.SERVE_VOLUMES))]
        m = configs.SERVE_ANGLES[rng.integers(len(configs.SERVE_ANGLES))]
        nt = configs.SERVE_T[rng.integers(len(configs.SERVE_T))]
        draws.append((t, vol, m, nt))
    plans = {}
    t0 = time.perf_counter()
    for _, vol, m, nt in draws:
        key = (vol, m, nt)
        if key not in plans:
            c = configs.serve_config(vol[0], vol[1], vol[2], m, nt, 0)
            plans[key] = Plan.from_config(c, 0.0, precisions=("fp32", "mixed"))
    torch.cuda.synchronize()
    t_plans = time.perf_counter() - t0
    reqs = []
    for i, (t, vol, m, nt) in enumerate(draws):
        c = configs.serve_config(vol[0], vol[1], vol[2], m, nt, i)
        p = plans[(vol, m, nt)]
        b = device_data(torch, p, configs.make_phantom(c), c.noise, c.noise_seed)
        geo = dict(nx=c.nx, ny=c.ny, nz=c.nz, n_angles=c.n_angles, n_t=c.n_t, drive_cycles=c.drive_cycles,
                   psf_width=c.psf_width, harm_lo=c.harm_lo, harm_hi=c.harm_hi, half_band=c.half_band,
                   op_scale=p.op_scale)
        reqs.append((Request(i, t, geo, b, c.lam, {}), (vol, m, nt)))
    return reqs, plans, t_plans


def serve_leg(torch, n_requests=None, stream=True):
    """The C3 stream (mixed path, 2 x 20) with p50/p99 latency, then closed-loop
    capacity of the FP32 and mixed paths with per-class schedules that reach
    1e-4 relative error against a converged reference."""
    import numpy as np
    from paper_2511_06627_amd import configs
    from paper_2511_06627_amd.serve import ContinuousBatcher, GpuExecutor, Request, summarize
    n_requests = n_requests or configs.SERVE_REQUESTS
    t0 = time.perf_counter()
    reqs, plans, t_plans = serve_requests(torch, n_requests)
    log("serve: %d requests, %d plans (%.1fs), data %.1fs"
        % (len(reqs), len(plans), t_plans, time.perf_counter() - t0))
    ex = GpuExecutor()
    for r, key in reqs:        # share the stream's plans (same geometry keys)
        ex.plans.setdefault(tuple(sorted(r.geometry.items())), plans[key])
    out = {"requests": len(reqs), "rate_hz": configs.SERVE_RATE_HZ, "classes": len(plans),
           "plan_build_s": round(t_plans, 2), "budget_bytes": configs.SERVE_BUDGET_BYTES}

    def with_sched(sched, arrival=None):
        return [Request(r.rid, r.arrival_s if arrival is None else arrival, r.geometry, r.b, r.lam, dict(sched[k]))
                for r, k in reqs]

    def run(rq, max_active=32):
        bat = ContinuousBatcher(ex, budget_bytes=configs.SERVE_BUDGET_BYTES, max_active=max_active)
        res = bat.run(rq)
        return res, summarize(res)

    # warm the executor's code paths once
    run(with_sched({k: dict(precision="mixed", refine_sweeps=1, inner_iters=2) for _, k in reqs}, 0.0)[:4])

    # (1) the stream as configured: Poisson arrivals, mixed path, 2 sweeps x 20
    if stream:
        cfg_sched = {k: dict(precision="mixed", refine_sweeps=2, inner_iters=20) for _, k in reqs}
        res, summ = run(with_sched(cfg_sched))
        out["stream_mixed_2x20"] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in summ.items()}
        log("serve stream (mixed 2x20): %s" % out["stream_mixed_2x20"])

    # (2) per-class schedules at 1e-4 against a converged FP32 reference
    # (150 CGLS iterations: the FP32 path's own accuracy floor, about 1e-6
    # of the FP64 minimiser on the realistic scan)
    ref = {}
    for r, k in reqs:
        p = plans[k]
        bd = torch.from_numpy(r.b).cuda()
        x, _ = p.solve(bd, r.lam, iters=150, report=False)
        ref[r.rid] = x
    first = {}
    for r, k in reqs:
        first.setdefault(k, r)

    def err(p, r, **kw):
        bd = torch.from_numpy(r.b).cuda()
        x, _ = p.solve(bd, r.lam, report=False, **kw)
        return float(torch.linalg.vector_norm(x - ref[r.rid]) / torch.linalg.vector_norm(ref[r.rid]))

    sched32, sched16 = {}, {}
    for k, r in first.items():
        p = plans[k]
        lo, hi = 10, 150            # smallest FP32 iteration count at 1e-4 (bisection)
        while hi - lo > 2:
            mid = (lo + hi) // 2
            if err(p, r, iters=mid) <= 1e-4:
                hi = mid
            else:
                lo = mid
        sched32[k] = dict(precision="fp32", iters=hi)
        sched16[k] = dict(precision="mixed", refine_sweeps=6, inner_iters=30)
        for sw, inner in MIXED_CANDIDATES:
            if err(p, r, precision="mixed", refine_sweeps=sw, inner_iters=inner) <= 1e-4:
                sched16[k] = dict(precision="mixed", refine_sweeps=sw, inner_iters=inner)
                break
    cap = {}
    for name, sched in (("fp32", sched32), ("mixed", sched16)):
        run(with_sched(sched, 0.0)[:8])
        res, summ = run(with_sched(sched, 0.0))
        errs = [float(np.linalg.norm(o.x - ref[o.rid].cpu().numpy()) / np.linalg.norm(ref[o.rid].cpu().numpy()))
                for o in res]
        iters = [sched[k].get("iters", sched[k].get("refine_sweeps", 0) * sched[k].get("inner_iters", 0))
                 for _, k in reqs]
        cap[name] = {"solves_per_s": round(summ["solves_per_s"], 2), "makespan_s": round(summ["span_s"], 4),
                     "p50_s": round(summ["p50_s"], 4), "p99_s": round(summ["p99_s"], 4),
                     "mean_iters": round(float(np.mean(iters)), 1),
                     "rel_err_max": float(max(errs)), "rel_err_median": float(np.median(errs))}
        log("serve closed loop %s: %s" % (name, cap[name]))
    out["closed_loop_at_1e-4"] = cap
    out["mixed_over_fp32"] = round(cap["mixed"]["solves_per_s"] / cap["fp32"]["solves_per_s"], 3)
    out["reference"] = "FP32 CGLS, 150 iterations, per request"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-tts", action="store_true", help="skip time-to-solve on the realistic scan")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy-mib", type=int, default=512,
                    help="size of a plain device copy run once, the reference for HBM byte counters")
    ap.add_argument("--skip-small", action="store_true",
                    help="skip the 32^3 time-to-solve (keeps a profile to the realistic scan)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream and closed-loop capacity")
    ap.add_argument("--serve-requests", type=int, default=0, help="requests in the serving stream (default 64)")
    ap.add_argument("--no-hdr", action="store_true", help="skip the high-dynamic-range scan")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the raster, tensor-PSF and dual-drive legs (their kernels run at other sizes)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="no oracle leg (for profiling runs): c_A estimated by the plan, data made on the device, "
                         "no cpu_baseline and no time-to-solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the operator is measured on one MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    from paper_2511_06627_amd import configs
    cfg = configs.REALISTIC_192
    small = configs.PARITY_32
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_leg(cfg, want_minimiser=not args.no_tts, sample_seconds=args.cpu_seconds,
                               small_cfg=None if args.skip_small else small)
        if not args.no_hdr:
            cpu["hdr"] = oracle_hdr_inputs()

    import numpy as np
    import torch
    from paper_2511_06627_amd.plan import Plan

    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.calib_copy_mib > 0:
        # a plain copy of known size: under rocprofv3 --pmc its FETCH_SIZE and
        # WRITE_SIZE calibrate the counters against known bytes
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if cpu is not None:
        plan = Plan.from_config(cfg, cpu["op_scale"], precisions=("fp32", "mixed"))
        x = torch.from_numpy(cpu["phantom"]).float().cuda()
        b = torch.from_numpy(cpu["b"]).cuda()
    else:
        plan = Plan.from_config(cfg, 0.0, precisions=("fp32", "mixed"))
        phantom = configs.make_phantom(cfg)
        x = torch.from_numpy(phantom).float().cuda()
        b = torch.from_numpy(device_data(torch, plan, phantom, cfg.noise, cfg.noise_seed)).cuda()
    yb = torch.empty(plan.data_shape, dtype=torch.complex64, device="cuda")
    xo = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    ws = plan.workspace("op")

    def step():
        plan.forward(x, out=yb, ws=ws)
        plan.adjoint(yb, out=xo, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    log("A^T A: %.3f ms/step" % ms_step)
    st32 = step_times(torch, step)

    # per-kernel device times (HIP events inside the library, on this stream)
    kt = {k: plan.time_kernel(k, repeats=10, x=x, b=b, ws=ws)
          for k in ("project", "signal_fwd", "signal_adj", "backproject")}
    log("kernels (ms): " + ", ".join("%s %.3f" % kv for kv in kt.items()))
    fl = signal_flops(cfg)
    dom = max(("signal_fwd", "signal_adj"), key=lambda k: kt[k])
    achieved = fl / (kt[dom] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dom), "flops_per_launch": fl}
    kernels = {}
    for k in ("signal_fwd", "signal_adj"):
        a = fl / (kt[k] * 1e-3) / 1e12
        kernels[k] = {"ms": round(kt[k], 4), "tflops": round(a, 2), "mfma_frac": round(a / FP32_PEAK_TFLOPS, 4)}
    pb = projection_bytes(cfg)
    for k in ("project", "backproject"):
        gbs = pb / (kt[k] * 1e-3) / 1e9
        kernels[k] = {"ms": round(kt[k], 4), "per_angle_stream_GBs": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}

    # mixed operator: A^T A rate and fp16 kernel times
    def step16():
        plan.forward(x, precision="mixed", out=yb, ws=ws)
        plan.adjoint(yb, precision="mixed", out=xo, ws=ws)

    for _ in range(args.warmup):
        step16()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step16()
    torch.cuda.synchronize()
    dt16 = time.perf_counter() - t0
    kt16 = {k: plan.time_kernel(k, repeats=10, precision="mixed", x=x, b=b, ws=ws)
            for k in ("project", "signal_fwd", "signal_adj")}
    mixed = {"applies_per_s": round(args.steps / dt16, 2), "ms_per_step": round(1e3 * dt16 / args.steps, 4),
             "step_ms": step_times(torch, step16)}
    for k, v in kt16.items():
        if k == "project":
            mixed["project_bf16"] = {"ms": round(v, 4), "per_angle_stream_GBs": round(pb / (v * 1e-3) / 1e9, 1)}
            continue
        a16 = fl / (v * 1e-3) / 1e12
        mixed[k] = {"ms": round(v, 4), "tflops": round(a16, 1), "mfma_frac_fp16": round(a16 / FP16_PEAK_TFLOPS, 4)}
    log("mixed A^T A: %.3f ms/step; kernels %s" % (1e3 * dt16 / args.steps, kt16))

    # the precomposed-line operator (same map, signal stage as two float32
    # GEMMs with G = F^T K): A^T A rate and the GEMM times
    planp = Plan.from_config(cfg, plan.op_scale, precisions=("fp32", "precomposed"))
    wsp = planp.workspace("op")

    def stepp():
        planp.forward(x, precision="precomposed", out=yb, ws=wsp)
        planp.adjoint(yb, precision="precomposed", out=xo, ws=wsp)

    for _ in range(args.warmup):
        stepp()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stepp()
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    gemm_flops = 2.0 * cfg.n_lines * cfg.n_u * 2 * cfg.n_bins
    ktp = {k: planp.time_kernel(k, repeats=10, precision="precomposed", x=x, b=b, ws=wsp)
           for k in ("signal_fwd", "signal_adj")}
    precomposed = {"applies_per_s": round(args.steps / dtp, 2), "ms_per_step": round(1e3 * dtp / args.steps, 4),
                   "gemm_flops": gemm_flops,
                   "gemm_fwd_ms": round(ktp["signal_fwd"], 4), "gemm_adj_ms": round(ktp["signal_adj"], 4)}
    log("precomposed A^T A: %.3f ms/step; GEMMs %s" % (1e3 * dtp / args.steps, ktp))
    del planp, wsp

    raster = tensor = dual = None
    if not args.no_variants:
        # the same scan under a zig-zag raster (two PSF tables, per-line sweep
        # direction): drive over a sixth of the fast axis, the focus field carrying
        # the line across two thirds of it
        ra, rs = cfg.n_u / 6.0, 2.0 * cfg.n_u / 3.0
        planr = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.n_angles, cfg.n_t, cfg.drive_cycles, cfg.psf_width, cfg.harm_lo,
                     cfg.harm_hi, cfg.half_band, 0.0, drive_amp=ra, raster_sweep=rs, precisions=("fp32", "mixed"))
        wsr = planr.workspace("op")
        raster = {"drive_amp": ra, "sweep": rs, "op_scale": planr.op_scale}
        for prec in ("fp32", "mixed"):
            def stepr():
                planr.forward(x, precision=prec, out=yb, ws=wsr)
                planr.adjoint(yb, precision=prec, out=xo, ws=wsr)

            for _ in range(args.warmup):
                stepr()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                stepr()
            torch.cuda.synchronize()
            dtr = time.perf_counter() - t0
            raster[prec] = {"applies_per_s": round(args.steps / dtr, 2), "ms_per_step": round(1e3 * dtr / args.steps, 4)}
        log("raster A^T A: %s" % raster)
        del planr, wsr

        # the same scan with the tensor PSF coupling each z-row to three rows on
        # either side (seven signal passes per application, FP32)
        plant = Plan.from_config(cfg, plan.op_scale, precisions=("fp32", "precomposed"), psf_rows=3)
        wst = plant.workspace("op")
        tensor = {"psf_rows": 3, "signal_passes": 7}
        for prec in ("fp32", "precomposed"):
            def stept():
                plant.forward(x, precision=prec, out=yb, ws=wst)
                plant.adjoint(yb, precision=prec, out=xo, ws=wst)

            for _ in range(args.warmup):
                stept()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                stept()
            torch.cuda.synchronize()
            dtt = time.perf_counter() - t0
            tensor[prec] = {"applies_per_s": round(args.steps / dtt, 2), "ms_per_step": round(1e3 * dtt / args.steps, 4)}
        log("tensor PSF (R = 3) A^T A: %s" % tensor)
        del plant, wst

        # the same scan acquired with both drive directions: 36 x 192 z-drive
        # lines (96 samples, padded to the x-drive lines' 192) after the x-drive ones
        pland = Plan.from_config(cfg, 0.0, precisions=("fp32", "mixed"), drive_axes=2)
        wsd = pland.workspace("op")
        ybd = torch.empty(pland.data_shape, dtype=torch.complex64, device="cuda")
        dual = {"z_lines": int(pland.info.n_lines) - cfg.n_lines, "op_scale": pland.op_scale}
        for prec in ("fp32", "mixed"):
            def stepd():
                pland.forward(x, precision=prec, out=ybd, ws=wsd)
                pland.adjoint(ybd, precision=prec, out=xo, ws=wsd)

            for _ in range(args.warmup):
                stepd()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                stepd()
            torch.cuda.synchronize()
            dtd = time.perf_counter() - t0
            dual[prec] = {"applies_per_s": round(args.steps / dtd, 2), "ms_per_step": round(1e3 * dtd / args.steps, 4)}
        log("dual drive A^T A: %s" % dual)
        del pland, wsd, ybd

    # CGLS iteration rate of the configured 50-iteration solve
    swk = plan.workspace("solve")
    plan.solve(b, cfg.lam, iters=2, ws=swk, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, rep = plan.solve(b, cfg.lam, iters=cfg.iters, ws=swk)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    log("CGLS %d iterations: %.3f s" % (cfg.iters, t_solve))

    # the paper's own solver (eq. iters): momentum gradient, finite-difference
    # T, projection onto x >= 0 every iteration, 150 iterations as in its
    # reconstructions; tau from power iteration on the device
    plan.solve(b, cfg.lam, iters=2, solver="momentum", reg="fd", clamp_every=1, ws=swk, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, repm_p = plan.solve(b, cfg.lam, iters=150, solver="momentum", reg="fd", clamp_every=1, ws=swk)
    torch.cuda.synchronize()
    t_paper = time.perf_counter() - t0
    paper_solver = {"iters": 150, "reg": "finite differences", "lambda": cfg.lam, "seconds_incl_tau": round(t_paper, 4),
                    "status": repm_p.status}
    log("paper solver (momentum, FD, 150 its): %.3f s" % t_paper)

    # mixed refinement solve (3 sweeps x 20 inner) against the 60-iteration FP32 solve
    m2 = configs.MIXED_192
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xm, repm = plan.solve(b, m2.lam, precision="mixed", refine_sweeps=m2.refine_sweeps, inner_iters=m2.inner_iters,
                          ws=swk)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    x60, _ = plan.solve(b, m2.lam, iters=m2.refine_sweeps * m2.inner_iters, ws=swk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve(b, m2.lam, iters=m2.refine_sweeps * m2.inner_iters, ws=swk, report=False)
    torch.cuda.synchronize()
    t_fp32_60 = time.perf_counter() - t0
    dm = float(torch.linalg.vector_norm(xm - x60) / torch.linalg.vector_norm(x60))
    mixed["solve_3x20"] = {"seconds": round(t_mixed, 4), "fp32_60_seconds": round(t_fp32_60, 4),
                           "rel_l2_vs_fp32_60": dm, "status": repm.status}
    log("mixed 3x20 solve %.4f s (fp32 60 its %.4f s), rel diff vs fp32 %.2e" % (t_mixed, t_fp32_60, dm))

    # time-to-solve at 1e-4 relative error against the FP64 minimiser
    tts = {}
    if cpu is not None and not args.skip_small:
        sm = cpu["small"]
        psmall = Plan.from_config(small, sm["op_scale"], precisions=("fp32", "mixed"))
        tts["parity_32cube"] = {p: time_to_solve(psmall, torch, sm["b"], sm["xstar"], small.lam, p)
                                for p in ("fp32", "mixed")}
    if cpu is not None and not args.no_tts:
        tts[cfg.name] = {p: time_to_solve(plan, torch, cpu["b"], cpu["xstar"], cfg.lam, p)
                         for p in ("fp32", "mixed")}

    hdr = None
    if cpu is not None and not args.no_hdr:
        hdr = hdr_leg(torch, cpu["hdr"])

    serve = None
    if not args.no_serve:
        serve = serve_leg(torch, args.serve_requests or None)

    value = args.steps / dt
    line = {
        "metric": "A^T A applies/s + time-to-solve at 1e-4 rel err vs FP64; p50/p99 latency",
        "value": round(value, 3),
        "unit": "A^T A applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "realistic_192x192x96: 36 angles, 96 lines x 8192 samples per angle, "
                               "harmonics 1-31 +/-3 bins, 40 blobs + ellipsoid phantom, 0.5% noise",
                   "step": "A then A^T, FP32 path", "global_batch": 1, "parallelism": "single GPU"},
        "step_ms": st32,
        "roofline": roofline,
        "cpu_baseline": cpu["cpu_baseline"] if cpu is not None else None,
        "kernels": kernels,
        "cgls": {"iters": cfg.iters, "seconds": round(t_solve, 4), "iters_per_s": round(cfg.iters / t_solve, 2),
                 "status": rep.status},
        "time_to_solve": tts,
        "paper_solver": paper_solver,
        "mixed": mixed,
        "precomposed": precomposed,
        "raster": raster,
        "tensor_psf": tensor,
        "dual_drive": dual,
        "serving": serve,
        "hdr": hdr,
        "oracle_small": cpu.get("oracle_small") if cpu is not None else None,
        "gpu_over_cpu": round(value / cpu["cpu_baseline"]["value"], 1) if cpu is not None else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

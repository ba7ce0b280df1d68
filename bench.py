"""Benchmark of the compressed 3D FFL operator on one MI355X.

Default run (python bench.py [--steps K] [--warmup W]):
  workload  the high-dynamic-range scan, the largest single-GPU workload:
            256 x 256 x 128 voxels, 60 FFL angles, 128 lines x 16384 time
            samples per angle, harmonics 1-47 +/- 3 bins, bright ellipsoid with
            30 faint satellite blobs
  step      one application of A followed by A^T (mpi3d_forward then
            mpi3d_adjoint), FP32 path, inputs resident in HBM
  value     A^T A applications per second (K steps timed between two device
            synchronisations)
Also reported: per-kernel device times from HIP events and the roofline of
the dominant kernel (with HBM traffic from the committed counter summary while
the kernel sources are unchanged), the mixed operator on the same scan, and
its nonnegative solves in both precisions against the oracle's clusters; then
the realistic 192 x 192 x 96 scan (FP32, mixed, precomposed-line operators;
raster, tensor-PSF and dual-drive variants; CGLS rate; the paper's own
solver; the configured mixed 3 x 20 schedule against x*; time-to-solve at 1e-4
relative error against the FP64 minimiser, also on 32^3); the serving stream
(p50/p99) and closed-loop capacity at 1e-4 against each request's
FP64-converged reference; and the FP64 CPU oracle timed on this host
(cpu_baseline leg: the time-domain oracle on a sample of the headline scan's
z-slices, scaled to the whole scan).

--headline-only runs only the headline scan's operator (profiling runs).
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
    while sample_seconds > 0:
        x = op.adjoint(op.forward(x))
        x /= np.linalg.norm(x)
        n += 1
        if n >= 2 and time.time() - t0 >= sample_seconds:
            break
    dt = time.time() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    if n:
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
        out["xstar_seconds"] = round(time.time() - t0, 2)
        log("oracle minimiser: %d CGLS iterations, %.1fs" % (it, time.time() - t0))
    return out


def hdr_cpu_leg(sample_slices=4, sample_seconds=15.0):
    """Oracle leg of the headline scan: c_A, phantom and data (the same recipe
    as the oracle's stored clusters in tests/golden/hdr_reference.json), and
    the timed oracle.  The cpu_baseline sample: A then A^T of the time-domain
    FP64 oracle (the form it defines) on `sample_slices` of the scan's 128
    z-slices -- A acts slice by slice, so the whole scan costs 128 /
    sample_slices times as much -- repeated for about `sample_seconds`, the
    rate scaled to whole-scan applications per second."""
    import numpy as np
    from oracle import operator as oop
    from oracle.geometry import Geometry
    from paper_2511_06627_amd import configs
    c = configs.HDR_256
    t0 = time.time()
    g = Geometry(nx=c.nx, ny=c.ny, nz=c.nz, n_angles=c.n_angles, n_t=c.n_t, drive_cycles=c.drive_cycles,
                 psf_width=c.psf_width, harm_lo=c.harm_lo, harm_hi=c.harm_hi, half_band=c.half_band)
    g = oop.normalised(g, iters_min=30, rtol=1e-9)
    phantom = configs.make_phantom(c)
    b, _ = oop.make_data(g, phantom, c.noise, c.noise_seed)
    log("oracle %s setup %.1fs" % (c.name, time.time() - t0))
    gs = Geometry(**{**{k: getattr(g, k) for k in g.__dataclass_fields__}, "nz": sample_slices})
    op = oop.Operator(gs)
    k0 = (c.nz - sample_slices) // 2
    x = phantom[k0:k0 + sample_slices].copy()
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
    value = n / dt * sample_slices / c.nz
    cpu = {"value": value, "unit": "A^T A applies/s", "cores": threads, "kind": "oracle",
           "sample": "%d applications of A then A^T of the FP64 time-domain oracle (C projector with OpenMP, BLAS "
                     "contractions) on %d of the %d z-slices of the %s scan in %.1f s; A is block diagonal over "
                     "z-slices, so the rate is scaled by %d/%d to whole-scan applications"
                     % (n, sample_slices, c.nz, c.name, dt, sample_slices, c.nz)}
    log("oracle A^T A (%s, %d-slice sample): %.4f whole-scan applies/s on %d threads"
        % (c.name, sample_slices, value, threads))
    return {"op_scale": g.op_scale, "b": b.astype(np.complex64), "phantom": phantom, "cpu_baseline": cpu}


# ---------------------------------------------------------------------------
# GPU leg
# ---------------------------------------------------------------------------
def signal_flops(cfg):
    """Algorithmic flops of one signal contraction (forward or adjoint) over all lines:
    2 L (Nu T + 2 nb T): the PSF contraction plus the band DFT, real arithmetic."""
    L = cfg.n_lines
    return 2.0 * L * (cfg.n_u * cfg.n_t + 2 * cfg.n_bins * cfg.n_t)


def fac_flops(cfg, plan, kernel):
    """Algorithmic flops of one launch of a kernel of the band DFT factored over
    drive cycles (t = n1 + P n2, T = C P, R residues of the kept bins mod C),
    real arithmetic over all L lines:
      fac_fwd / fac_adj       2 L T (Nu + 2R): the PSF contraction and the
                              C-point residue DFT (real signal, complex twiddles);
      fac_fwd_out / fac_adj_in 8 L P nb: each bin's P-point complex sum."""
    L, T = cfg.n_lines, cfg.n_t
    P = T // plan.dft_cycles
    if kernel in ("fac_fwd", "fac_adj"):
        return 2.0 * L * T * (cfg.n_u + 2 * plan.dft_residues)
    return 8.0 * L * P * cfg.n_bins


def fac_bytes(cfg, plan, kernel):
    """Algorithmic HBM bytes of one launch of a factored band-DFT kernel: its
    inputs and outputs once (lines 4 L Nu, phase sums 4 L P 2R, data 8 L nb)
    and its tables once (PSF table 4 T Nu and residue twiddles 8 C R for the
    contraction kernels; per-bin phase twiddles 8 P nb for the outer sums)."""
    L, T, C, R = cfg.n_lines, cfg.n_t, plan.dft_cycles, plan.dft_residues
    P = T // C
    phase = 4.0 * L * P * 2 * R
    if kernel in ("fac_fwd", "fac_adj"):
        return 4.0 * L * cfg.n_u + phase + 4.0 * T * cfg.n_u + 8.0 * C * R
    return phase + 8.0 * L * cfg.n_bins + 8.0 * P * cfg.n_bins


LDS_PEAK_GBS = 256 * 128 * 2.4      # 128 bytes per clock per CU, 256 CUs at 2.4 GHz (78.6 TB/s)


def projection_bytes(cfg):
    """Per-angle-stream byte model of one projection: every angle reads the whole
    volume once and writes its lines (fp32).  The kernels stage each slice in
    LDS once for many angles, so this is a model of a streaming design, not the
    kernels' traffic (see projection_report)."""
    nvox = cfg.nx * cfg.ny * cfg.nz
    return 4.0 * (cfg.n_angles * nvox + cfg.n_lines * cfg.n_u)


def projection_report(cfg, kernel, ms, measured_bytes, half=False):
    """Projection / backprojection against three references:
    * the per-angle-stream model (a design that streams the volume once per angle);
    * compulsory HBM bytes (the volume and the lines once) and, when the
      counter summary matches the sources, the measured HBM bytes;
    * LDS: the bytes the kernel's gathers read from LDS, one bilinear footprint
      of 4 texels per ray sample and slice (forward: 4 B per texel and slice in
      fp32, 2 B in bf16) or 3 staged ray values per voxel, angle and slice
      (backprojection: 4 B each in fp32, 2 B in the mixed operator's fp16),
      about n_angles * n_vox samples in all,
      against the LDS peak of 128 B per clock per CU."""
    nvox = cfg.nx * cfg.ny * cfg.nz
    samples = float(cfg.n_angles) * nvox
    if kernel == "project":
        lds = samples * 4 * (2 if half else 4)
    else:
        lds = samples * 3 * (2 if half else 4)
    pb = projection_bytes(cfg)
    vol_b = 2 if half and kernel == "project" else 4        # the mixed forward gathers a bf16 volume
    line_b = 2 if half and kernel == "backproject" else 4   # the mixed adjoint gathers fp16 lines
    compulsory = vol_b * nvox + line_b * cfg.n_lines * cfg.n_u
    t = ms * 1e-3
    out = {"ms": round(ms, 4),
           "model_stream_GBs": round(pb / t / 1e9, 1), "model_stream_frac": round(pb / t / 1e9 / HBM_PEAK_GBS, 4),
           "compulsory_bytes": compulsory,
           "lds_bytes": lds, "lds_GBs": round(lds / t / 1e9, 1), "lds_frac": round(lds / t / 1e9 / LDS_PEAK_GBS, 4)}
    if measured_bytes:
        out["hbm_bytes_measured"] = measured_bytes
        out["hbm_GBs_measured"] = round(measured_bytes / t / 1e9, 1)
        out["hbm_frac_measured"] = round(measured_bytes / t / 1e9 / HBM_PEAK_GBS, 4)
    return out


def signal_bytes(cfg, kernel):
    """Algorithmic HBM bytes of one signal contraction: its input lines, its
    output, the PSF table K (fp32, T x Nu) and a T-entry complex twiddle table
    (the band DFT's values), each once.  Forward: lines 4 L Nu in, data
    8 L nb out; adjoint the reverse."""
    L = cfg.n_lines
    return 4.0 * L * cfg.n_u + 8.0 * L * cfg.n_bins + 4.0 * cfg.n_t * cfg.n_u + 8.0 * cfg.n_t


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


# Library sources that do not take part in an operator application (the
# serving scheduler, the no-allocation entry point): outside the hash below.
HASH_EXCLUDED = ("serve.cpp", "noalloc.cpp")


def kernel_source_hash():
    """sha256 over the library's kernel and launch sources of the operator
    (kernels, launch configuration, line jobs): HBM traffic taken from
    counters is only valid for the code it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2511_06627_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".cpp", ".h")) and name not in HASH_EXCLUDED:
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain
    copy's readings), or None when the sources changed since the counters were
    taken or the summary has no such entry."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("workloads", {}).get(workload)
    if not rec or rec.get("source_sha256") != kernel_source_hash():
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


def hdr_leg(torch, plan, inputs):
    """The headline scan's nonnegative solves, FP32 (100 CGLS iterations, clamp
    + restart every 10) and mixed (10 sweeps of 10, clamp after each): solve
    time, and the iterate and the faint blobs' recovered amplitudes against the
    means of the oracle's clusters of the same schedule at the two ends of the
    path's operator error range (the solve is chaotic mid-run;
    tests/golden/make_hdr.py), with the exact oracle run's distance to those
    means beside them."""
    import numpy as np
    from paper_2511_06627_amd import configs, phantoms
    cfg = configs.HDR_256
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "hdr_reference.json")))
    bd = torch.from_numpy(inputs["b"]).cuda()
    idx = np.array(ref["sample_index"])
    amp_true = np.array([bl["amp_true"] for bl in ref["blobs"]])
    profiles = [phantoms._blob(cfg.shape, bl["centre_xyz"], bl["sigma"], 1.0) for bl in ref["blobs"]]
    out = {}
    schedules = {"fp32": dict(iters=cfg.iters, clamp_every=cfg.clamp_every),
                 "mixed": dict(precision="mixed", refine_sweeps=cfg.iters // cfg.clamp_every,
                               inner_iters=cfg.clamp_every, clamp_every=cfg.clamp_every)}
    ws = plan.workspace("solve")
    for prec, kw in schedules.items():
        plan.solve(bd, cfg.lam, report=False, ws=ws, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, rep = plan.solve(bd, cfg.lam, ws=ws, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xn = x.cpu().numpy().astype(np.float64)
        amp = np.array([float(np.vdot(xn, gb) / np.vdot(gb, gb)) for gb in profiles])
        if "cluster" not in ref:       # a reference file without clusters: times and amplitudes only
            out[prec] = {"schedule": kw, "seconds": round(dt, 4), "status": rep.status,
                         "faint_amp_recovered_over_true_median": float(np.median(amp / amp_true))}
            log("hdr %s: %s" % (prec, out[prec]))
            continue
        lo, hi = ref["cluster"][prec]
        xs = xn.ravel()[idx]
        alo, ahi = np.array(lo["amp_mean"]), np.array(hi["amp_mean"])
        out[prec] = {"schedule": kw, "seconds": round(dt, 4), "status": rep.status,
                     "samples_to_cluster_means": [float(np.linalg.norm(xs - np.array(c["sample_mean"]))
                                                        / np.linalg.norm(c["sample_mean"])) for c in (lo, hi)],
                     "cluster_radii": [lo["sample_radius"], hi["sample_radius"]],
                     "cluster_eps": [lo["eps"], hi["eps"]],
                     "exact_oracle_to_cluster_means": [lo["exact_sample_to_mean"], hi["exact_sample_to_mean"]],
                     "faint_amp_max_rel_to_cluster_means": [float(np.max(np.abs(amp - a) / np.abs(a)))
                                                            for a in (alo, ahi)],
                     "faint_amp_cluster_radii": [lo["amp_radius_rel"], hi["amp_radius_rel"]],
                     "faint_amp_recovered_over_true_median": float(np.median(amp / amp_true))}
        log("hdr %s: %s" % (prec, out[prec]))
    del ws
    return out


# ---------------------------------------------------------------------------
# Serving leg: the request stream, solved by the continuous batcher
# ---------------------------------------------------------------------------
# Refinement schedules (sweeps, inner iterations), in order of cost: a sweep's
# FP32 restart costs about two mixed iterations.
MIXED_CANDIDATES = ((2, 25), (2, 30), (3, 20), (2, 35), (3, 25), (4, 20), (3, 30), (4, 25), (3, 40), (5, 30),
                    (6, 30))
SERVE_REF_ITERS = 300      # FP32 CGLS iterations of a serving request's converged reference
SERVE_TARGET = 8e-5        # schedule target: every request of a class within this of its reference


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

    # every request's reference: FP32 CGLS run to convergence (REF_ITERS
    # iterations; tests/test_gpu_solve.py holds such solves within 1e-5 of
    # the FP64 minimiser on serving classes)
    ref = {}
    for r, k in reqs:
        bd = torch.from_numpy(r.b).cuda()
        x, _ = plans[k].solve(bd, r.lam, iters=SERVE_REF_ITERS, report=False)
        ref[r.rid] = x.cpu().numpy().astype(np.float64)

    def errors(res):
        return [float(np.linalg.norm(o.x - ref[o.rid]) / np.linalg.norm(ref[o.rid])) for o in res]

    # (1) the stream as configured: Poisson arrivals, mixed path, 2 sweeps x 20
    if stream:
        cfg_sched = {k: dict(precision="mixed", refine_sweeps=2, inner_iters=20) for _, k in reqs}
        res, summ = run(with_sched(cfg_sched))
        rec = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in summ.items()}
        e = errors(res)
        rec.update({"rel_err_max": max(e), "rel_err_median": float(np.median(e))})
        out["stream_mixed_2x20"] = rec
        log("serve stream (mixed 2x20): %s" % rec)

    # (2) per-class schedules that hold every request of the class within
    # SERVE_TARGET of its reference (the cheapest FP32 iteration count, found
    # by bisection on the class's worst request, and the cheapest refinement
    # schedule in MIXED_CANDIDATES order), then the closed loop of all requests
    by_class = {}
    for r, k in reqs:
        by_class.setdefault(k, []).append(r)

    def worst(p, rs, **kw):
        e = 0.0
        for r in rs:
            x, _ = p.solve(torch.from_numpy(r.b).cuda(), r.lam, report=False, **kw)
            xr = ref[r.rid]
            e = max(e, float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)))
        return e

    sched32, sched16 = {}, {}
    for k, rs in by_class.items():
        p = plans[k]
        lo, hi = 10, 200            # smallest FP32 iteration count within the target (bisection)
        while hi - lo > 2:
            mid = (lo + hi) // 2
            if worst(p, rs, iters=mid) <= SERVE_TARGET:
                hi = mid
            else:
                lo = mid
        sched32[k] = dict(precision="fp32", iters=hi)
        sched16[k] = dict(precision="mixed", refine_sweeps=8, inner_iters=30)
        for sw, inner in MIXED_CANDIDATES:
            if worst(p, rs, precision="mixed", refine_sweeps=sw, inner_iters=inner) <= SERVE_TARGET:
                sched16[k] = dict(precision="mixed", refine_sweeps=sw, inner_iters=inner)
                break
        log("serve schedule %s (%d requests): fp32 %d iterations, mixed %d x %d"
            % (k, len(rs), hi, sched16[k]["refine_sweeps"], sched16[k]["inner_iters"]))
    cap = {}
    for name, sched in (("fp32", sched32), ("mixed", sched16)):
        run(with_sched(sched, 0.0)[:8])
        res, summ = run(with_sched(sched, 0.0))
        errs = errors(res)
        iters = [sched[k].get("iters", sched[k].get("refine_sweeps", 0) * sched[k].get("inner_iters", 0))
                 for _, k in reqs]
        cap[name] = {"solves_per_s": round(summ["solves_per_s"], 2), "makespan_s": round(summ["span_s"], 4),
                     "p50_s": round(summ["p50_s"], 4), "p99_s": round(summ["p99_s"], 4),
                     "mean_iters": round(float(np.mean(iters)), 1),
                     "rel_err_max": float(max(errs)), "rel_err_median": float(np.median(errs))}
        log("serve closed loop %s: %s" % (name, cap[name]))
    out["closed_loop_at_1e-4"] = cap
    out["mixed_over_fp32"] = round(cap["mixed"]["solves_per_s"] / cap["fp32"]["solves_per_s"], 3)
    out["reference"] = "FP32 CGLS, %d iterations, per request (converged)" % SERVE_REF_ITERS
    out["schedule_target"] = SERVE_TARGET
    return out


def realistic_leg(torch, args, cfg, small, cpu, inputs):
    """The realistic 192 x 192 x 96 scan: FP32 and mixed operators, the
    precomposed-line operator, the raster / tensor-PSF / dual-drive variants,
    the CGLS rate, the paper's own solver, the configured mixed 3 x 20 solve
    (against x* and against 60 FP32 iterations), and time-to-solve at 1e-4."""
    import numpy as np
    from paper_2511_06627_amd import configs
    from paper_2511_06627_amd.plan import Plan
    plan, x, b = inputs(cfg, cpu)
    out = operator_leg(torch, plan, cfg, x, b, args.warmup, args.steps)
    out["applies_per_s"] = round(1.0 / out["seconds_per_step"], 2)
    yb = torch.empty(plan.data_shape, dtype=torch.complex64, device="cuda")
    xo = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    if args.realistic_only:
        return out

    # the precomposed-line operator (same map, signal stage as two float32
    # GEMMs with G = F^T K): A^T A rate and the GEMM times
    planp = Plan.from_config(cfg, plan.op_scale, precisions=("fp32", "precomposed"))
    wsp = planp.workspace("op")

    def stepp():
        planp.forward(x, precision="precomposed", out=yb, ws=wsp)
        planp.adjoint(yb, precision="precomposed", out=xo, ws=wsp)

    sec, _ = timed_rate(torch, stepp, args.warmup, args.steps)
    ktp = {k: planp.time_kernel(k, repeats=10, precision="precomposed", x=x, b=b, ws=wsp)
           for k in ("signal_fwd", "signal_adj")}
    out["precomposed"] = {"applies_per_s": round(1.0 / sec, 2), "ms_per_step": round(1e3 * sec, 4),
                          "gemm_flops": 2.0 * cfg.n_lines * cfg.n_u * 2 * cfg.n_bins,
                          "gemm_fwd_ms": round(ktp["signal_fwd"], 4), "gemm_adj_ms": round(ktp["signal_adj"], 4)}
    log("precomposed A^T A: %.3f ms/step; GEMMs %s" % (1e3 * sec, ktp))
    del planp, wsp

    def rate_of(p, prec, data_shape=None):
        yy = yb if data_shape is None else torch.empty(data_shape, dtype=torch.complex64, device="cuda")
        ws = p.workspace("op")

        def st():
            p.forward(x, precision=prec, out=yy, ws=ws)
            p.adjoint(yy, precision=prec, out=xo, ws=ws)

        sec, _ = timed_rate(torch, st, args.warmup, args.steps)
        return {"applies_per_s": round(1.0 / sec, 2), "ms_per_step": round(1e3 * sec, 4)}

    if not args.no_variants:
        # the same scan under a zig-zag raster (two PSF tables, per-line sweep
        # direction): drive over a sixth of the fast axis, the focus field carrying
        # the line across two thirds of it
        ra, rs = cfg.n_u / 6.0, 2.0 * cfg.n_u / 3.0
        planr = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.n_angles, cfg.n_t, cfg.drive_cycles, cfg.psf_width, cfg.harm_lo,
                     cfg.harm_hi, cfg.half_band, 0.0, drive_amp=ra, raster_sweep=rs, precisions=("fp32", "mixed"))
        out["raster"] = {"drive_amp": ra, "sweep": rs, "op_scale": planr.op_scale,
                         "fp32": rate_of(planr, "fp32"), "mixed": rate_of(planr, "mixed")}
        log("raster A^T A: %s" % out["raster"])
        del planr
        # the tensor PSF coupling each z-row to three rows on either side
        plant = Plan.from_config(cfg, plan.op_scale, precisions=("fp32", "mixed", "precomposed"), psf_rows=3)
        out["tensor_psf"] = {"psf_rows": 3, "fp32": rate_of(plant, "fp32"), "mixed": rate_of(plant, "mixed"),
                             "precomposed": rate_of(plant, "precomposed")}
        log("tensor PSF (R = 3) A^T A: %s" % out["tensor_psf"])
        del plant
        # both drive directions: 36 x 192 z-drive lines after the x-drive ones
        pland = Plan.from_config(cfg, 0.0, precisions=("fp32", "mixed"), drive_axes=2)
        out["dual_drive"] = {"z_lines": int(pland.info.n_lines) - cfg.n_lines, "op_scale": pland.op_scale,
                             "fp32": rate_of(pland, "fp32", pland.data_shape),
                             "mixed": rate_of(pland, "mixed", pland.data_shape)}
        log("dual drive A^T A: %s" % out["dual_drive"])
        del pland
        # both drives under the tensor PSF: x-drive lines coupled across three
        # z-rows on either side, z-drive lines across three detector columns
        plantd = Plan.from_config(cfg, 0.0, precisions=("fp32", "mixed"), drive_axes=2, psf_rows=3)
        out["tensor_dual"] = {"psf_rows": 3, "z_lines": int(plantd.info.n_lines) - cfg.n_lines,
                              "fp32": rate_of(plantd, "fp32", plantd.data_shape),
                              "mixed": rate_of(plantd, "mixed", plantd.data_shape)}
        log("tensor PSF + dual drive A^T A: %s" % out["tensor_dual"])
        del plantd

    # CGLS iteration rate of the configured 50-iteration solve
    swk = plan.workspace("solve")
    plan.solve(b, cfg.lam, iters=2, ws=swk, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = plan.solve(b, cfg.lam, iters=cfg.iters, ws=swk)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    out["cgls"] = {"iters": cfg.iters, "seconds": round(t_solve, 4), "iters_per_s": round(cfg.iters / t_solve, 2),
                   "status": rep.status}
    log("CGLS %d iterations: %.3f s" % (cfg.iters, t_solve))

    # the paper's own solver (eq. iters): momentum gradient, finite-difference
    # T, projection onto x >= 0 every iteration, 150 iterations; tau from
    # power iteration on the device
    plan.solve(b, cfg.lam, iters=2, solver="momentum", reg="fd", clamp_every=1, ws=swk, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, repm_p = plan.solve(b, cfg.lam, iters=150, solver="momentum", reg="fd", clamp_every=1, ws=swk)
    torch.cuda.synchronize()
    out["paper_solver"] = {"iters": 150, "reg": "finite differences", "lambda": cfg.lam,
                           "seconds_incl_tau": round(time.perf_counter() - t0, 4), "status": repm_p.status}

    # the configured mixed schedule (3 sweeps x 20 inner): against x* (when the
    # oracle leg ran) and against 60 FP32 iterations
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
    rec = {"seconds": round(t_mixed, 4), "fp32_60_seconds": round(t_fp32_60, 4), "status": repm.status,
           "rel_l2_vs_fp32_60": float(torch.linalg.vector_norm(xm - x60) / torch.linalg.vector_norm(x60))}
    if cpu is not None and "xstar" in cpu:
        xs = cpu["xstar"]
        xn = np.linalg.norm(xs)
        rec["rel_l2_vs_xstar"] = float(np.linalg.norm(xm.cpu().numpy() - xs) / xn)
        rec["fp32_60_rel_l2_vs_xstar"] = float(np.linalg.norm(x60.cpu().numpy() - xs) / xn)
    out["mixed"]["solve_3x20"] = rec
    log("mixed 3x20 solve: %s" % rec)
    del swk

    tts = {}
    if cpu is not None and not args.skip_small and "small" in cpu:
        sm = cpu["small"]
        psmall = Plan.from_config(small, sm["op_scale"], precisions=("fp32", "mixed"))
        tts["parity_32cube"] = {p: time_to_solve(psmall, torch, sm["b"], sm["xstar"], small.lam, p)
                                for p in ("fp32", "mixed")}
    if cpu is not None and "xstar" in cpu:
        tts[cfg.name] = {p: time_to_solve(plan, torch, cpu["b"], cpu["xstar"], cfg.lam, p)
                         for p in ("fp32", "mixed")}
    out["time_to_solve"] = tts
    if cpu is not None:
        out["oracle_small"] = cpu.get("oracle_small")
        # the oracle beside it on this scan: its A then A^T rate (time-domain
        # form, a few applications) and its minimiser solve (CGLS to 1e-9)
        out["oracle"] = {"AtA": cpu.get("cpu_baseline"), "minimiser_cgls_iters": cpu.get("xstar_iters"),
                         "minimiser_seconds": cpu.get("xstar_seconds")}
    return out


def timed_rate(torch, step, warmup, steps):
    """Wall time per step of `steps` steps after `warmup`, bracketed by device
    synchronisations; returns (seconds per step, total seconds)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt / steps, dt


def operator_leg(torch, plan, cfg, x, b, warmup, steps, with_mixed=True):
    """A then A^T on one scan: FP32 rate (the step of the headline), per-kernel
    device times, the dominant kernel's roofline, and the same for the mixed
    operator."""
    yb = torch.empty(plan.data_shape, dtype=torch.complex64, device="cuda")
    xo = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    ws = plan.workspace("op")

    def step():
        plan.forward(x, out=yb, ws=ws)
        plan.adjoint(yb, out=xo, ws=ws)

    sec, dt = timed_rate(torch, step, warmup, steps)
    log("%s A^T A: %.3f ms/step" % (cfg.name, 1e3 * sec))
    out = {"seconds_per_step": sec, "total_s": dt, "step_ms": step_times(torch, step)}
    kt = {k: plan.time_kernel(k, repeats=10, x=x, b=b, ws=ws)
          for k in ("project", "signal_fwd", "signal_adj", "backproject")}
    log("%s kernels (ms): %s" % (cfg.name, ", ".join("%s %.3f" % kv for kv in kt.items())))
    fl = signal_flops(cfg)
    kernels = {}
    if plan.dft_cycles:
        # the band DFT factored over drive cycles: two kernels a stage; the
        # roofline is that of the dominant one, on its own algorithmic flops
        facs = ("fac_fwd", "fac_fwd_out", "fac_adj_in", "fac_adj")
        kf = {k: plan.time_kernel(k, repeats=10, x=x, b=b, ws=ws) for k in facs}
        log("%s factored band DFT (C = %d, %d residues) kernels (ms): %s"
            % (cfg.name, plan.dft_cycles, plan.dft_residues, ", ".join("%s %.3f" % kv for kv in kf.items())))
        dom = max(("fac_fwd", "fac_adj"), key=lambda k: kf[k])
        fd = fac_flops(cfg, plan, dom)
        achieved = fd / (kf[dom] * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2),
                           "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                           "traffic": measured_traffic(cfg.name, dom), "flops_per_launch": fd,
                           "algorithmic_bytes_per_launch": fac_bytes(cfg, plan, dom)}
        for k in facs:
            fk = fac_flops(cfg, plan, k)
            a = fk / (kf[k] * 1e-3) / 1e12
            kernels[k] = {"ms": round(kf[k], 4), "flops": fk, "tflops": round(a, 2),
                          "mfma_frac": round(a / FP32_PEAK_TFLOPS, 4),
                          "hbm_bytes_measured": measured_traffic(cfg.name, k),
                          "hbm_bytes_algorithmic": fac_bytes(cfg, plan, k)}
        stage = {"signal_fwd": ("fac_fwd", "fac_fwd_out"), "signal_adj": ("fac_adj_in", "fac_adj")}
        for k, parts in stage.items():
            fs = sum(fac_flops(cfg, plan, p) for p in parts)
            kernels[k] = {"ms": round(kt[k], 4), "kernels": list(parts), "flops": fs,
                          "tflops": round(fs / (kt[k] * 1e-3) / 1e12, 2),
                          "dense_equivalent_tflops": round(fl / (kt[k] * 1e-3) / 1e12, 2),
                          "dft_cycles": plan.dft_cycles, "dft_residues": plan.dft_residues}
    else:
        dom = max(("signal_fwd", "signal_adj"), key=lambda k: kt[k])
        achieved = fl / (kt[dom] * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2),
                           "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                           "traffic": measured_traffic(cfg.name, dom), "flops_per_launch": fl,
                           "algorithmic_bytes_per_launch": signal_bytes(cfg, dom)}
        for k in ("signal_fwd", "signal_adj"):
            a = fl / (kt[k] * 1e-3) / 1e12
            kernels[k] = {"ms": round(kt[k], 4), "tflops": round(a, 2), "mfma_frac": round(a / FP32_PEAK_TFLOPS, 4),
                          "hbm_bytes_measured": measured_traffic(cfg.name, k),
                          "hbm_bytes_algorithmic": signal_bytes(cfg, k)}
    for k in ("project", "backproject"):
        kernels[k] = projection_report(cfg, k, kt[k], measured_traffic(cfg.name, k))
    out["kernels"] = kernels
    if not with_mixed:
        return out

    def step16():
        plan.forward(x, precision="mixed", out=yb, ws=ws)
        plan.adjoint(yb, precision="mixed", out=xo, ws=ws)

    sec16, _ = timed_rate(torch, step16, warmup, steps)
    kt16 = {k: plan.time_kernel(k, repeats=10, precision="mixed", x=x, b=b, ws=ws)
            for k in ("project", "signal_fwd", "signal_adj", "backproject")}
    mixed = {"applies_per_s": round(1.0 / sec16, 2), "ms_per_step": round(1e3 * sec16, 4),
             "step_ms": step_times(torch, step16)}
    for k, v in kt16.items():
        if k in ("project", "backproject"):
            # 16-bit gathers: a bf16 volume forward, fp16 lines backward
            mixed[k + ("_bf16" if k == "project" else "_f16")] = projection_report(
                cfg, k, v, measured_traffic(cfg.name, k + "_mixed"), half=True)
            continue
        a16 = fl / (v * 1e-3) / 1e12
        mixed[k] = {"ms": round(v, 4), "tflops": round(a16, 1), "mfma_frac_fp16": round(a16 / FP16_PEAK_TFLOPS, 4),
                    "hbm_bytes_measured": measured_traffic(cfg.name, k + "_mixed")}
    log("%s mixed A^T A: %.3f ms/step; kernels %s" % (cfg.name, 1e3 * sec16, kt16))
    out["mixed"] = mixed
    del ws
    return out


# ---------------------------------------------------------------------------
# Profile summaries: rocprofv3 output directories -> profiles/
# ---------------------------------------------------------------------------
KERNEL_KEYS = (("fac_fwd_kernel", "fac_fwd"), ("fac_fwd_out_kernel", "fac_fwd_out"), ("fac_adj_in_kernel", "fac_adj_in"),
               ("fac_adj_kernel", "fac_adj"),
               ("sig_fwd_f32", "signal_fwd"), ("sig_adj_f32", "signal_adj"), ("sig_fwd_f16", "signal_fwd_mixed"),
               ("sig_adj_f16", "signal_adj_mixed"), ("proj_fwd_kernel<unsigned int>", "project_mixed"),
               ("proj_fwd_kernel", "project"), ("proj_adj_f16", "backproject_mixed"),
               ("proj_adj_kernel", "backproject"))


def kernel_key(name):
    for frag, key in KERNEL_KEYS:
        if frag in name:
            return key
    return None


def _csv_rows(directory, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path) as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit("no %s under %s" % (suffix, directory))
    return rows


def summarize_kernel_stats(directory, workload, command):
    """profiles/kernel_stats_<workload>.md from a rocprofv3 --kernel-trace --stats run."""
    rows = _csv_rows(directory, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# Kernel statistics: %s" % workload, "", "Command (from the repository root, on one MI355X):", "",
           "    " + command, "", "| kernel | calls | average (us) | min (us) | max (us) | share |",
           "|---|---|---|---|---|---|"]
    for r in rows[:25]:
        name = r["Name"] if len(r["Name"]) < 110 else r["Name"][:107] + "..."
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.1f%% |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    path = os.path.join(ROOT, "profiles", "kernel_stats_%s.md" % workload)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("wrote", path)


def summarize_hbm(fetch_dir, write_dir, workload, commands, copy_mib=512):
    """profiles/hbm_traffic.json (entry `workload`) and
    profiles/hbm_traffic_<workload>.md from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE; KiB per dispatch).  Both are scaled by what they read for
    the plain device copy of copy_mib MiB that bench.py runs first (read and
    written once), so the result is HBM bytes per launch."""
    import numpy as np

    def per_kernel(directory, counter):
        rows = [r for r in _csv_rows(directory, "counter_collection.csv") if r["Counter_Name"].startswith(counter)]
        by = {}
        for r in rows:
            by.setdefault((r["Dispatch_Id"], r["Kernel_Name"]), 0.0)
            by[(r["Dispatch_Id"], r["Kernel_Name"])] += float(r["Counter_Value"])
        return by

    f = per_kernel(fetch_dir, "FETCH_SIZE")
    w = per_kernel(write_dir, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    cf = max(v for (d, n), v in f.items() if "copy" in n.lower())
    cw = max(v for (d, n), v in w.items() if "copy" in n.lower())
    fs, wsc = copy_kib / cf, copy_kib / cw
    kern = {}
    for src, key in ((f, "fetch"), (w, "write")):
        for (d, n), v in src.items():
            k = kernel_key(n)
            if k is None:
                continue
            kern.setdefault(k, {"kernel": n, "fetch": [], "write": []})[key].append(v)
    out = {}
    for k, v in kern.items():
        if not v["fetch"] or not v["write"]:
            continue
        fk, wk = float(np.mean(v["fetch"])), float(np.mean(v["write"]))
        rb, wb = int(round(fk * 1024 * fs)), int(round(wk * 1024 * wsc))
        out[k] = {"kernel": v["kernel"], "dispatches": len(v["fetch"]), "fetch_kib": round(fk, 1),
                  "write_kib": round(wk, 1), "hbm_read_bytes": rb, "hbm_write_bytes": wb,
                  "hbm_bytes_per_launch": rb + wb}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec.setdefault("workloads", {})
    rec.pop("kernels", None)
    rec["workloads"][workload] = {"commands": commands, "source_sha256": kernel_source_hash(),
                                  "calibration": {"copy_kib": copy_kib, "fetch_kib": cf, "write_kib": cw,
                                                  "fetch_scale": fs, "write_scale": wsc},
                                  "kernels": out}
    for k in ("workload", "commands", "calibration", "source_sha256"):
        rec.pop(k, None)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    lines = ["# HBM traffic per launch: %s" % workload, "",
             "Two rocprofv3 counter runs (from the repository root, on one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Calibration: a plain device copy of %d MiB read FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB, so "
              "fetch counts are scaled by %.4f and write counts by %.4f." % (copy_mib, cf, cw, fs, wsc), "",
              "| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM read (MB) | HBM write (MB) | total (MB) |",
              "|---|---|---|---|---|---|---|"]
    for k, v in sorted(out.items()):
        lines.append("| %s (`%s`) | %d | %.1f | %.1f | %.2f | %.2f | %.2f |" % (
            k, v["kernel"][:80], v["dispatches"], v["fetch_kib"], v["write_kib"], v["hbm_read_bytes"] / 1e6,
            v["hbm_write_bytes"] / 1e6, v["hbm_bytes_per_launch"] / 1e6))
    md = os.path.join(ROOT, "profiles", "hbm_traffic_%s.md" % workload)
    with open(md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", path, md)


def summarize_sq(directory, workload, command):
    """profiles/mfma_lds_counters_<workload>.md from a rocprofv3 --pmc run of
    SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA SQ_INSTS_LDS SQ_ACTIVE_INST_LDS
    SQ_LDS_BANK_CONFLICT SQ_INSTS_VALU GRBM_GUI_ACTIVE: per dispatch, averaged
    over each kernel's dispatches.  GRBM_GUI_ACTIVE is summed over the 8 XCDs,
    so its per-XCD value is the kernel's duration in GPU cycles; MFMA
    utilisation = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x 1024 SIMDs); the
    bank-conflict ratio = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS."""
    import numpy as np
    rows = _csv_rows(directory, "counter_collection.csv")
    per = {}
    for r in rows:
        k = kernel_key(r["Kernel_Name"])
        if k is None:
            continue
        d = per.setdefault(k, {}).setdefault(r["Dispatch_Id"], {})
        name = r["Counter_Name"]
        d[name] = d.get(name, 0.0) + float(r["Counter_Value"])
    names = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS",
             "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_VALU", "GRBM_GUI_ACTIVE")
    out = ["# MFMA and LDS counters: %s" % workload, "", "Command (from the repository root, on one MI355X):", "",
           "    " + command, "", summarize_sq.__doc__.split("\n\n")[0].replace("\n    ", "\n"), "",
           "| kernel | dispatches | GPU cycles | MFMA instr | MFMA util | LDS instr | LDS active cycles | "
           "bank-conflict cycles | conflict / active | VALU instr |", "|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(per):
        ds = list(per[k].values())
        m = {n: float(np.mean([d.get(n, 0.0) for d in ds])) for n in names}
        cyc = m["GRBM_GUI_ACTIVE"] / 8.0
        util = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * 1024) if cyc else 0.0
        ratio = m["SQ_LDS_BANK_CONFLICT"] / m["SQ_ACTIVE_INST_LDS"] if m["SQ_ACTIVE_INST_LDS"] else 0.0
        out.append("| %s | %d | %.0f | %.0f | %.1f%% | %.0f | %.0f | %.0f | %.2f | %.0f |" % (
            k, len(ds), cyc, m["SQ_INSTS_MFMA"], 100 * util, m["SQ_INSTS_LDS"], m["SQ_ACTIVE_INST_LDS"],
            m["SQ_LDS_BANK_CONFLICT"], ratio, m["SQ_INSTS_VALU"]))
    path = os.path.join(ROOT, "profiles", "mfma_lds_counters_%s.md" % workload)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("wrote", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-tts", action="store_true", help="skip time-to-solve on the realistic scan")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy-mib", type=int, default=512,
                    help="size of a plain device copy run once, the reference for HBM byte counters")
    ap.add_argument("--skip-small", action="store_true", help="skip the 32^3 time-to-solve")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream and closed-loop capacity")
    ap.add_argument("--serve-requests", type=int, default=0, help="requests in the serving stream (default 64)")
    ap.add_argument("--no-hdr-solve", action="store_true", help="skip the headline scan's nonnegative solves")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the raster, tensor-PSF and dual-drive legs (their kernels run at other sizes)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline scan's A then A^T (FP32 and mixed): for profiling runs")
    ap.add_argument("--realistic-only", action="store_true",
                    help="only the realistic scan's operator legs (profiling runs of its kernels)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="no oracle leg (for profiling runs): c_A estimated by the plan, data made on the device, "
                         "no cpu_baseline, no time-to-solve and no solve comparisons")
    ap.add_argument("--summarize-kernel-stats", metavar="DIR",
                    help="write profiles/kernel_stats_<workload>.md from a rocprofv3 --stats output folder")
    ap.add_argument("--summarize-hbm", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/hbm_traffic* from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output folders")
    ap.add_argument("--summarize-sq", metavar="DIR",
                    help="write profiles/mfma_lds_counters_<workload>.md from a rocprofv3 --pmc SQ counter folder")
    ap.add_argument("--workload", default="hdr_256x256x128", help="workload name for --summarize-*")
    ap.add_argument("--command", action="append", default=[], help="profiling command(s) for --summarize-*")
    args = ap.parse_args()
    if args.summarize_kernel_stats:
        summarize_kernel_stats(args.summarize_kernel_stats, args.workload, " && ".join(args.command))
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq, args.workload, " && ".join(args.command))
        return
    if args.summarize_hbm:
        summarize_hbm(args.summarize_hbm[0], args.summarize_hbm[1], args.workload, args.command)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the operator is measured on one MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    from paper_2511_06627_amd import configs
    head = configs.HDR_256
    real = configs.REALISTIC_192
    small = configs.PARITY_32
    do_head = not args.realistic_only
    do_extras = not args.headline_only
    cpu_head = cpu_real = None
    if not args.no_cpu:
        if do_head:
            cpu_head = hdr_cpu_leg(sample_seconds=args.cpu_seconds)
        if do_extras:
            cpu_real = cpu_baseline_leg(real, want_minimiser=not args.no_tts, sample_seconds=5.0,
                                        small_cfg=None if args.skip_small else small)

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

    def inputs(cfg, cpu):
        if cpu is not None:
            plan = Plan.from_config(cfg, cpu["op_scale"], precisions=("fp32", "mixed"))
            return plan, torch.from_numpy(cpu["phantom"]).float().cuda(), torch.from_numpy(cpu["b"]).cuda()
        plan = Plan.from_config(cfg, 0.0, precisions=("fp32", "mixed"))
        phantom = configs.make_phantom(cfg)
        return (plan, torch.from_numpy(phantom).float().cuda(),
                torch.from_numpy(device_data(torch, plan, phantom, cfg.noise, cfg.noise_seed)).cuda())

    # ---- headline: the 256 x 256 x 128 scan, FP32 A then A^T ----------------
    head_out = hdr = None
    if do_head:
        plan_h, x_h, b_h = inputs(head, cpu_head)
        head_out = operator_leg(torch, plan_h, head, x_h, b_h, args.warmup, args.steps)
        if cpu_head is not None and do_extras and not args.no_hdr_solve:
            hdr = hdr_leg(torch, plan_h, cpu_head)
        del plan_h, x_h, b_h
        torch.cuda.empty_cache()

    # ---- the realistic 192 x 192 x 96 scan -----------------------------------
    realistic = None
    if do_extras:
        realistic = realistic_leg(torch, args, real, small, cpu_real, inputs)

    serve = None
    if do_extras and not args.no_serve and not args.realistic_only:
        serve = serve_leg(torch, args.serve_requests or None)

    if do_head:
        value = 1.0 / head_out["seconds_per_step"]
        workload = ("hdr_256x256x128: 60 angles, 128 lines x 16384 samples per angle, harmonics 1-47 +/-3 bins, "
                    "bright ellipsoid + 30 faint blobs (1e-4..1e-2), 0.1% noise")
        ms_step = 1e3 * head_out["seconds_per_step"]
        roofline = head_out["roofline"]
        cpu_b = cpu_head["cpu_baseline"] if cpu_head is not None else None
    else:
        value = 1.0 / realistic["seconds_per_step"]
        workload = "realistic_192x192x96 (headline scan skipped)"
        ms_step = 1e3 * realistic["seconds_per_step"]
        roofline = realistic["roofline"]
        cpu_b = None
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
        "config": {"workload": workload, "step": "A then A^T, FP32 path", "global_batch": 1,
                   "parallelism": "single GPU"},
        "step_ms": head_out["step_ms"] if head_out else None,
        "roofline": roofline,
        "cpu_baseline": cpu_b,
        "kernels": head_out["kernels"] if head_out else None,
        "mixed": head_out["mixed"] if head_out else None,
        "hdr_solve": hdr,
        "realistic": realistic,
        "serving": serve,
        "gpu_over_cpu": round(value / cpu_b["value"], 1) if cpu_b else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Write tests/golden/hdr_reference.json: the FP64 oracle's solve of the
high-dynamic-range scan (256 x 256 x 128 voxels, 60 angles, T = 16384,
harmonics 1-47 +/- 3, bright ellipsoid with 30 faint satellite blobs, 0.1%
noise): CGLS, 100 iterations, clamped at zero and restarted every 10 (the
nonnegativity of Sec. 3.3 after eq. iters).

Calls only the oracle (and the seeded phantom generator).  Stores what a GPU
test can compare without the 33 MB volume:
  * the exact (unperturbed) iterate on 4096 seeded sample voxels and its norm;
  * each faint blob's recovered amplitude <x, g_b> / <g_b, g_b> (g_b the
    blob's unit-amplitude profile) next to its true amplitude;
  * clusters (tests/helpers.py, ``ClusterPath``): the solve is chaotic
    mid-run, so a GPU iterate is compared with clusters of oracle runs whose
    operator outputs carry independent random relative errors at the low and
    the high end of the GPU path's per-call error range, within a few radii of
    the segment between the two cluster means --
      fp32   the FP32 schedule (CGLS 100, clamp and restart every 10) with
             operator errors of 1e-7 and 1e-6, 3 runs each;
      mixed  the mixed schedule (10 refinement sweeps of 10 in correction
             form, clamped after each) with sweep residuals at 1e-6 and the
             inner operator at 5e-5 and 3e-4, 3 runs each;
    each level with the mean and radius on the sample voxels and of every
    faint blob's amplitude (radius: the largest relative distance of a run
    from the mean, over runs and, for amplitudes, over blobs).

Usage: python tests/golden/make_hdr.py   (about 2.5 hours on 8 cores)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

from oracle import operator as oop, solvers  # noqa: E402
from paper_2511_06627_amd import configs, phantoms  # noqa: E402
from helpers import (config_geometry, Cluster, PerturbedOperator, FP32_OP_EPS, FP32_EPS_RANGE,  # noqa: E402
                     MIXED_EPS_RANGE, CLUSTER_BAR)

N_SAMPLES = 4096
SAMPLE_SEED = 4242
SEEDS_FP32 = tuple(range(111, 114))
SEEDS_MIXED = tuple(range(211, 214))


def blob_profiles(cfg):
    _, blobs = phantoms.organ_with_satellites(cfg.shape, 30, (1.0, 2.0), (-4.0, -2.0), (2.0, 5.0), cfg.phantom_seed)
    return blobs


def amplitudes(x, blobs, shape):
    out = []
    for c, sigma, _ in blobs:
        g = phantoms._blob(shape, c, sigma, 1.0)
        out.append(float(np.vdot(x, g) / np.vdot(g, g)))
    return np.array(out)


def main(cfg=configs.HDR_256, dest=os.path.join(HERE, "hdr_reference.json")):
    t0 = time.time()
    g = config_geometry(cfg)
    ph = configs.make_phantom(cfg)
    b, _ = oop.make_data(g, ph, cfg.noise, cfg.noise_seed)
    b = b.astype(np.complex64).astype(np.complex128)
    op = oop.Operator(g, precomposed=True)
    blobs = blob_profiles(cfg)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(int(np.prod(cfg.shape)), N_SAMPLES, replace=False))
    print("setup %.1fs" % (time.time() - t0), flush=True)

    def timed(fn, what):
        t = time.time()
        x = fn()
        print("  %s %.1fs" % (what, time.time() - t), flush=True)
        return x

    run32 = lambda o: solvers.cgls_restarted(o, b, cfg.lam, cfg.iters, cfg.clamp_every, clamp=True)  # noqa: E731
    sweeps = cfg.iters // cfg.clamp_every
    run16 = lambda o, oi: solvers.refine(o, oi, b, cfg.lam, sweeps, cfg.clamp_every, clamp=True)  # noqa: E731

    x = timed(lambda: run32(op), "fp32 exact")
    amp = amplitudes(x, blobs, cfg.shape)
    xs = x.ravel()[idx]

    def cluster(runs, eps):
        smp = Cluster(runs, select=lambda v: np.asarray(v).ravel()[idx])
        amps = np.array([amplitudes(r, blobs, cfg.shape) for r in runs])
        amean = amps.mean(axis=0)
        arad = float(np.max(np.abs(amps - amean) / np.abs(amean)))
        return {"eps": eps, "runs": len(runs), "sample_mean": smp.mean.tolist(), "sample_radius": smp.radius,
                "sample_pairwise": smp.pairwise, "amp_mean": amean.tolist(), "amp_radius_rel": arad,
                "exact_sample_to_mean": smp.distance(xs),
                "exact_amp_to_mean_rel": float(np.max(np.abs(amp - amean) / np.abs(amean)))}

    def show(name, rec):
        print(name, {k: v for k, v in rec.items() if k not in ("sample_mean", "amp_mean")}, flush=True)

    clusters = {"bar_radii": CLUSTER_BAR}
    for eps in FP32_EPS_RANGE:
        runs = [timed(lambda: run32(PerturbedOperator(op, eps, s)), "fp32 eps %.0e seed %d" % (eps, s))
                for s in SEEDS_FP32]
        clusters.setdefault("fp32", []).append(cluster(runs, eps))
        show("fp32", clusters["fp32"][-1])
        del runs
    for eps in MIXED_EPS_RANGE:
        runs = [timed(lambda: run16(PerturbedOperator(op, FP32_OP_EPS, s), PerturbedOperator(op, eps, s + 5000)),
                      "mixed eps %.0e seed %d" % (eps, s)) for s in SEEDS_MIXED]
        clusters.setdefault("mixed", []).append(cluster(runs, eps))
        show("mixed", clusters["mixed"][-1])
        del runs
    clusters["mixed_schedule"] = "%d refinement sweeps of %d, clamped after each" % (sweeps, cfg.clamp_every)
    rec = {
        "workload": cfg.name,
        "schedule": "CGLS, %d iterations, clamped at 0 and restarted every %d" % (cfg.iters, cfg.clamp_every),
        "lambda": cfg.lam,
        "op_scale": g.op_scale,
        "x_norm": float(np.linalg.norm(x)),
        "sample_seed": SAMPLE_SEED,
        "sample_index": idx.tolist(),
        "sample_value": xs.tolist(),
        "blobs": [{"centre_xyz": [float(v) for v in c], "sigma": float(sg), "amp_true": float(a),
                   "amp_oracle": float(ao)} for (c, sg, a), ao in zip(blobs, amp)],
        "cluster": clusters,
    }
    with open(dest, "w") as f:
        json.dump(rec, f)
    print("done %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()

"""Write tests/golden/cgls_clusters.json: perturbed-oracle clusters of the
same-schedule solves on the realistic 192 x 192 x 96 scan.

Calls only the oracle (and the seeded phantom generator).  CGLS is chaotic
mid-run (see tests/helpers.py, ``Cluster``), so a GPU iterate is compared with
the mean of oracle runs whose operator outputs carry independent random
relative errors at the GPU path's error level, and the bar is a multiple of the
runs' spread around that mean.  For each schedule the file holds, on a seeded
sample of voxels (the volume itself is 14 MB): the sample indices, the
cluster mean, its radius (largest run-to-mean distance, relative to the mean)
and largest pairwise distance, the radius over the whole volume, and the exact
(unperturbed) run's distance from the mean.

Schedules:
  cgls50     FP32 path: CGLS, 50 iterations; operator errors 1e-6 (the FP32
             operator's level), 6 runs.
  mixed3x20  mixed path: 3 refinement sweeps of 20 inner iterations in
             correction form; sweep residuals at 1e-6, inner operator at 2e-4
             (the mixed operator's level), 6 runs.  Also stored: the FP64
             minimiser x* on the same sample (CGLS to |s| <= 1e-12 |s_0|), so a
             test can state the schedule's error against x*.

Usage: python tests/golden/make_clusters.py   (about 20 minutes on 8 cores)
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
from paper_2511_06627_amd import configs  # noqa: E402
from helpers import (config_geometry, Cluster, PerturbedOperator, FP32_OP_EPS, MIXED_OP_EPS,  # noqa: E402
                     CLUSTER_BAR)

N_SAMPLES = 16384
SAMPLE_SEED = 1919
SEEDS_FP32 = tuple(range(101, 107))
SEEDS_MIXED = tuple(range(201, 207))


def record(runs, exact, idx, eps):
    full = Cluster(runs)
    smp = Cluster(runs, select=lambda v: np.asarray(v).ravel()[idx])
    return {"eps": eps, "runs": len(runs), "sample_mean": smp.mean.tolist(), "radius": smp.radius,
            "pairwise": smp.pairwise, "radius_full": full.radius, "bar_radii": CLUSTER_BAR,
            "exact_to_mean_full": full.distance(exact)}


def main():
    cfg = configs.REALISTIC_192
    m2 = configs.MIXED_192
    t0 = time.time()
    g = config_geometry(cfg)
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    b = b.astype(np.complex64).astype(np.complex128)
    op = oop.Operator(g, precomposed=True)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(int(np.prod(cfg.shape)), N_SAMPLES, replace=False))
    out = {"workload": cfg.name, "op_scale": g.op_scale, "lambda": cfg.lam, "sample_seed": SAMPLE_SEED,
           "sample_index": idx.tolist()}
    print("setup %.1fs" % (time.time() - t0), flush=True)

    def timed(fn, what):
        t = time.time()
        x = fn()
        print("  %s %.1fs" % (what, time.time() - t), flush=True)
        return x

    cg = lambda o: solvers.cgls(o, b, cfg.lam, cfg.iters)  # noqa: E731
    exact = timed(lambda: cg(op), "cgls50 exact")
    runs = [timed(lambda: cg(PerturbedOperator(op, FP32_OP_EPS, s)), "cgls50 seed %d" % s) for s in SEEDS_FP32]
    out["cgls50"] = record(runs, exact, idx, FP32_OP_EPS)
    print("cgls50", {k: v for k, v in out["cgls50"].items() if k != "sample_mean"}, flush=True)

    rf = lambda o, oi: solvers.refine(o, oi, b, m2.lam, m2.refine_sweeps, m2.inner_iters)  # noqa: E731
    exact = timed(lambda: rf(op, op), "mixed3x20 exact")
    runs = [timed(lambda: rf(PerturbedOperator(op, FP32_OP_EPS, s), PerturbedOperator(op, MIXED_OP_EPS, s + 5000)),
                  "mixed3x20 seed %d" % s) for s in SEEDS_MIXED]
    out["mixed3x20"] = record(runs, exact, idx, MIXED_OP_EPS)
    print("mixed3x20", {k: v for k, v in out["mixed3x20"].items() if k != "sample_mean"}, flush=True)

    xs, its = timed(lambda: solvers.reference_minimiser(op, b, cfg.lam, tol=1e-12), "minimiser")
    out["xstar"] = {"tol": 1e-12, "iters": its, "sample": xs.ravel()[idx].tolist(),
                    "norm": float(np.linalg.norm(xs))}
    mean_full = np.mean(runs, axis=0)
    out["mixed3x20"]["mean_to_xstar_full"] = float(np.linalg.norm(mean_full - xs) / np.linalg.norm(xs))
    print("mixed 3x20 cluster mean vs x*: %.3e" % out["mixed3x20"]["mean_to_xstar_full"], flush=True)
    with open(os.path.join(HERE, "cgls_clusters.json"), "w") as f:
        json.dump(out, f)
    print("done %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()

"""Write tests/golden/cgls_clusters.json: perturbed-oracle clusters of the
same-schedule solves on the realistic 192 x 192 x 96 scan.

Calls only the oracle (and the seeded phantom generator).  CGLS is chaotic
mid-run (see tests/helpers.py, ``Cluster`` and ``ClusterPath``), so a GPU
iterate is compared with clusters of oracle runs whose operator outputs carry
independent random relative errors at the low and the high end of the GPU
path's per-call error range: within a bar of a few radii of the segment
between the two cluster means.  For each schedule and level the file holds, on
a seeded sample of voxels (the volume itself is 14 MB): the cluster mean, its
radius (largest run-to-mean distance, relative to the mean) and largest
pairwise distance, the radius over the whole volume, and the exact
(unperturbed) run's distance from the mean; and the distance between the two
means.

Schedules:
  cgls50     FP32 path: CGLS, 50 iterations; operator errors 1e-7 and 1e-6
             (the FP32 operator's range), 6 runs each.
  mixed3x20  mixed path: 3 refinement sweeps of 20 inner iterations in
             correction form; sweep residuals at 1e-6, inner operator at 5e-5
             and 3e-4 (the mixed operator's range), 6 runs each.  Also stored:
             the FP64 minimiser x* on the same sample (CGLS to
             |s| <= 1e-12 |s_0|), so a test can state the schedule's error
             against x*.

Usage: python tests/golden/make_clusters.py   (about 80 minutes on 8 cores)
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
from helpers import (config_geometry, Cluster, PerturbedOperator, FP32_OP_EPS, FP32_EPS_RANGE,  # noqa: E402
                     MIXED_EPS_RANGE, CLUSTER_BAR)

N_SAMPLES = 16384
SAMPLE_SEED = 1919
SEEDS_FP32 = tuple(range(101, 107))
SEEDS_MIXED = tuple(range(201, 207))


def record(runs, exact, idx, eps):
    full = Cluster(runs)
    smp = Cluster(runs, select=lambda v: np.asarray(v).ravel()[idx])
    return {"eps": eps, "runs": len(runs), "sample_mean": smp.mean.tolist(), "radius": smp.radius,
            "pairwise": smp.pairwise, "radius_full": full.radius, "exact_to_mean_full": full.distance(exact)}, full.mean


def path(lo, hi):
    (rlo, mlo), (rhi, mhi) = lo, hi
    return {"lo": rlo, "hi": rhi, "bar_radii": CLUSTER_BAR,
            "span": float(np.linalg.norm(mhi - mlo) / np.linalg.norm(mhi))}


def main(cfg=configs.REALISTIC_192, m2=configs.MIXED_192, dest=os.path.join(HERE, "cgls_clusters.json")):
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

    def show(name, rec):
        print(name, {k: (v if k not in ("lo", "hi") else {kk: vv for kk, vv in v.items() if kk != "sample_mean"})
                     for k, v in rec.items()}, flush=True)

    cg = lambda o: solvers.cgls(o, b, cfg.lam, cfg.iters)  # noqa: E731
    exact = timed(lambda: cg(op), "cgls50 exact")
    levels = []
    for eps in FP32_EPS_RANGE:
        runs = [timed(lambda: cg(PerturbedOperator(op, eps, s)), "cgls50 eps %.0e seed %d" % (eps, s))
                for s in SEEDS_FP32]
        levels.append(record(runs, exact, idx, eps))
        del runs
    out["cgls50"] = path(*levels)
    show("cgls50", out["cgls50"])

    rf = lambda o, oi: solvers.refine(o, oi, b, m2.lam, m2.refine_sweeps, m2.inner_iters)  # noqa: E731
    exact = timed(lambda: rf(op, op), "mixed3x20 exact")
    levels = []
    for eps in MIXED_EPS_RANGE:
        runs = [timed(lambda: rf(PerturbedOperator(op, FP32_OP_EPS, s), PerturbedOperator(op, eps, s + 5000)),
                      "mixed3x20 eps %.0e seed %d" % (eps, s)) for s in SEEDS_MIXED]
        levels.append(record(runs, exact, idx, eps))
        del runs
    out["mixed3x20"] = path(*levels)
    show("mixed3x20", out["mixed3x20"])

    xs, its = timed(lambda: solvers.reference_minimiser(op, b, cfg.lam, tol=1e-12), "minimiser")
    out["xstar"] = {"tol": 1e-12, "iters": its, "sample": xs.ravel()[idx].tolist(),
                    "norm": float(np.linalg.norm(xs))}
    xsf = xs.ravel()
    for name, (_, m) in zip(("lo", "hi"), levels):
        out["mixed3x20"][name]["mean_to_xstar_full"] = float(np.linalg.norm(m.ravel() - xsf) / np.linalg.norm(xsf))
    print("mixed 3x20 cluster means vs x*: %.3e / %.3e" % (out["mixed3x20"]["lo"]["mean_to_xstar_full"],
                                                            out["mixed3x20"]["hi"]["mean_to_xstar_full"]), flush=True)
    with open(dest, "w") as f:
        json.dump(out, f)
    print("done %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()

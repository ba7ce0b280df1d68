"""Write tests/golden/cgls_envelopes.json: FP32 drift envelopes of CGLS schedules.

Calls only the oracle.  For each (workload, schedule) it runs the FP64 CGLS
and three runs whose operator outputs carry independent random relative
errors of size 1e-6 (the FP32 operator's error level, see tests/helpers.py)
and records the largest relative L2 deviation of the final iterate.  GPU tests compare their FP32
iterate against the FP64 one with max(1e-5, 4 x envelope).

Usage: python tests/golden/make_envelopes.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

from oracle import operator as oop, solvers  # noqa: E402
from paper_2511_06627_amd import configs  # noqa: E402
from helpers import config_geometry, fp32_envelope  # noqa: E402


def main():
    out = {}
    cfg = configs.REALISTIC_192
    g = config_geometry(cfg)
    ph = configs.make_phantom(cfg)
    b, _ = oop.make_data(g, ph, cfg.noise, cfg.noise_seed)
    b = b.astype(np.complex64).astype(np.complex128)
    op = oop.Operator(g, precomposed=True)
    _, env = fp32_envelope(lambda o: solvers.cgls(o, b, cfg.lam, cfg.iters), op)
    out["%s/cgls%d" % (cfg.name, cfg.iters)] = env
    print(cfg.name, env, flush=True)
    with open(os.path.join(HERE, "cgls_envelopes.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

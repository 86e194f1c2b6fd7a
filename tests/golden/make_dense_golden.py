"""Writes the dense-oracle reference values for the n = 65536 log-likelihood +
score workload (Matern 3/2, theta = (0.05, 1, 1e-4), points uniform in
[0,1]^2 with seed 31, z = N(0, I) draws with seed 32) into
c3_matern32_n65536_dense.json.

Calls only oracle.dense (dense FP64 Cholesky, about 35 GB of host memory and
tens of minutes on 8 cores).  Usage:  python tests/golden/make_dense_golden.py [n]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import dense  # noqa: E402
import workloads as W  # noqa: E402


def main():
    spec = W.WORKLOADS["c3_matern32_n65536"]
    n = int(sys.argv[1]) if len(sys.argv) > 1 else spec["n"]
    P = W.workload_points("c3_matern32_n65536", n)
    z = W.gaussian(n, spec["w_seed"])
    t0 = time.time()
    o = dense.loglik_and_grad(P, z, spec["theta"], spec["kernel"], spec["alpha"], block=2048, want_terms=True)
    secs = time.time() - t0
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    out = {
        "workload": "c3_matern32_n65536" if n == spec["n"] else "c3_recipe_n%d" % n,
        "n": n, "kernel": spec["kernel"], "theta": list(spec["theta"]), "points_seed": spec["points"][1],
        "z": "workloads.gaussian(n, %d)" % spec["w_seed"],
        "ell": o["ell"], "logdet": o["logdet"], "ztSinvz": float(z @ o["alpha"]),
        "g": list(map(float, o["g"])), "q": list(map(float, o["q"])), "t": list(map(float, o["t"])),
        "alpha_index": sample.tolist(), "alpha_value": [float(o["alpha"][i]) for i in sample],
        "oracle_seconds": secs,
        "generator": "tests/golden/make_dense_golden.py (oracle.dense only)",
    }
    name = "c3_matern32_n65536_dense.json" if n == spec["n"] else "c3_recipe_n%d_dense.json" % n
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", name, "in %.1f s" % secs)


if __name__ == "__main__":
    main()

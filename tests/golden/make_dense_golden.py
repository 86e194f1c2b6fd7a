"""Writes dense-oracle reference values for the named workloads into
tests/golden/<workload>_dense.json.  Calls only oracle.dense (dense FP64
Cholesky).  The n = 65536 workload needs about 35 GB of host memory and tens
of minutes on 8 cores.

  python tests/golden/make_dense_golden.py c3_matern32_n65536
  python tests/golden/make_dense_golden.py c2_rq_n16384

Observations z are N(0, I) draws (workloads.gaussian(n, w_seed)); the
log-likelihood and its score are defined for any z.
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
    name = sys.argv[1] if len(sys.argv) > 1 else "c3_matern32_n65536"
    spec = W.WORKLOADS[name]
    n = int(sys.argv[2]) if len(sys.argv) > 2 else spec["n"]
    P = W.workload_points(name, n)
    nrhs = spec.get("nrhs", 1)
    Z = W.gaussian((n, nrhs), spec["w_seed"]) if nrhs > 1 else W.gaussian(n, spec["w_seed"])
    z = Z if nrhs == 1 else Z[:, 0]
    t0 = time.time()
    o = dense.loglik_and_grad(P, z, spec["theta"], spec["kernel"], spec["alpha"], block=2048, want_terms=True)
    secs = time.time() - t0
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    out = {
        "workload": name if n == spec["n"] else "%s_recipe_n%d" % (name, n),
        "n": n, "kernel": spec["kernel"], "theta": list(spec["theta"]), "alpha_rq": spec["alpha"],
        "z": "workloads.gaussian(n, %d) (first column when several)" % spec["w_seed"],
        "ell": o["ell"], "logdet": o["logdet"], "ztSinvz": float(z @ o["alpha"]),
        "g": list(map(float, o["g"])), "q": list(map(float, o["q"])), "t": list(map(float, o["t"])),
        "alpha_index": sample.tolist(), "alpha_value": [float(o["alpha"][i]) for i in sample],
        "oracle_seconds": secs,
        "generator": "tests/golden/make_dense_golden.py (oracle.dense only)",
    }
    fname = ("%s_dense.json" % name) if n == spec["n"] else ("%s_recipe_n%d_dense.json" % (name, n))
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", fname, "in %.1f s" % secs)


if __name__ == "__main__":
    main()

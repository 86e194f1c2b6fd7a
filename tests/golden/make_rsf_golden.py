"""Writes the oracle RSF + peeling reference for the n = 65536 log-likelihood
+ score workload (Matern 3/2, theta = (0.05, 1, 1e-4), eps = eps_peel = 1e-6,
leaf 64, 256 proxies on 4 rings, peeling seed 33; z = workloads.gaussian(n, 32))
into c3_matern32_n65536_rsf.json.  Calls only oracle.rsf / oracle.peel (plain
numpy; about an hour on 8 cores).

  python tests/golden/make_rsf_golden.py [n]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import rsf  # noqa: E402
import workloads as W  # noqa: E402


def main():
    name = "c3_matern32_n65536"
    spec = W.WORKLOADS[name]
    n = int(sys.argv[1]) if len(sys.argv) > 1 else spec["n"]
    P = W.workload_points(name, n)
    z = W.gaussian(n, spec["w_seed"])
    t0 = time.time()
    o = rsf.loglik_grad(P, z, spec["theta"], spec["kernel"], spec["eps"], spec["leaf"], eps_peel=spec["eps"],
                        seed=spec["peel_seed"], n_prox=spec["n_prox"], prox_rings=spec["prox_rings"])
    secs = time.time() - t0
    F = o["factor"]
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    ranks = {int(d): [int(F.rank[int(b)]) for b in F.tree.levels[d]] for d in range(1, F.tree.max_depth + 1)}
    out = {
        "workload": name if n == spec["n"] else "%s_recipe_n%d" % (name, n),
        "n": n, "eps": spec["eps"], "eps_peel": spec["eps"], "peel_seed": spec["peel_seed"],
        "z": "workloads.gaussian(n, %d)" % spec["w_seed"],
        "ell": o["ell"], "logdet": o["logdet"], "q": list(map(float, o["q"])), "t": list(map(float, o["t"])),
        "g": list(map(float, o["g"])),
        "peel_cols": {str(k): int(v) for k, v in o["peel_cols"].items()},
        "peel_ranks": {str(k): int(v) for k, v in o["peel_ranks"].items()},
        "root_size": int(F.Iroot.shape[0]),
        "skeleton_total_per_level": {str(d): int(sum(r)) for d, r in ranks.items()},
        "alpha_index": sample.tolist(), "alpha_value": [float(o["alpha"][i]) for i in sample],
        "oracle_seconds": secs,
        "generator": "tests/golden/make_rsf_golden.py (oracle.rsf and oracle.peel only)",
    }
    fname = "%s_rsf.json" % out["workload"]
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", fname, "in %.1f s" % secs)


if __name__ == "__main__":
    main()

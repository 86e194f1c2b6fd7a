"""Writes dense-oracle reference values for the named workloads into
tests/golden/<workload>_dense.json.  Calls only oracle.dense (dense FP64
Cholesky; for n > 20000 the blocked in-place route of one n x n buffer:
factor, triangular inverse and Sigma^-1 in place, then the score terms).  The
n = 65536 workload needs about 36 GB of host memory and most of an hour on 8
cores.

  python tests/golden/make_dense_golden.py c3_matern32_n65536
  python tests/golden/make_dense_golden.py c2_rq_n16384
  python tests/golden/make_dense_golden.py c3_matern32_n65536 model

With "model", z is a draw from the model itself, z = L w with the dense
Cholesky factor L of Sigma and w = workloads.gaussian(n, w_seed); z and
Sigma^-1 z are written next to the reference as <workload>_model_z.npy and
<workload>_model_alpha.npy (the log-likelihood is then exact for that z:
z^T Sigma^-1 z = w^T w), with the score terms q, t and g.

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
    if len(sys.argv) > 2 and sys.argv[2] == "model":
        return model(name, spec)
    n = int(sys.argv[2]) if len(sys.argv) > 2 else spec["n"]
    P = W.workload_points(name, n)
    nrhs = spec.get("nrhs", 1)
    Z = W.gaussian((n, nrhs), spec["w_seed"]) if nrhs > 1 else W.gaussian(n, spec["w_seed"])
    z = Z if nrhs == 1 else Z[:, 0]
    t0 = time.time()
    if n <= 20000:
        o = dense.loglik_and_grad(P, z, spec["theta"], spec["kernel"], spec["alpha"], block=2048, want_terms=True)
    else:
        o = dense.score_large(P, spec["theta"], spec["kernel"], spec["alpha"], bs=8192, z=z,
                              log=lambda m: print(m, flush=True))
    secs = time.time() - t0
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    out = {
        "workload": name if n == spec["n"] else "%s_recipe_n%d" % (name, n),
        "n": n, "kernel": spec["kernel"], "theta": list(spec["theta"]), "alpha_rq": spec["alpha"],
        "z": "workloads.gaussian(n, %d) (first column when several)" % spec["w_seed"],
        "ell": o["ell"], "logdet": o["logdet"], "ztSinvz": float(z @ o["alpha"]),
        "g": list(map(float, o["g"])) if "g" in o else None,
        "q": list(map(float, o["q"])) if "q" in o else None,
        "t": list(map(float, o["t"])) if "t" in o else None,
        "alpha_index": sample.tolist(), "alpha_value": [float(o["alpha"][i]) for i in sample],
        "oracle_seconds": secs,
        "generator": "tests/golden/make_dense_golden.py (oracle.dense only)",
    }
    fname = ("%s_dense.json" % name) if n == spec["n"] else ("%s_recipe_n%d_dense.json" % (name, n))
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", fname, "in %.1f s" % secs)


def model(name, spec):
    """z = L w (a draw from the model, Sigma = L L^T by the blocked dense
    Cholesky) and, for that z, the exact l, log|Sigma|, Sigma^-1 z = L^-T w and
    the score terms q, t, g from Sigma^-1 = L^-T L^-1 formed in place."""
    n = spec["n"]
    P = W.workload_points(name, n)
    w = W.gaussian(n, spec["w_seed"])
    t0 = time.time()
    o = dense.score_large(P, spec["theta"], spec["kernel"], spec["alpha"], bs=8192, w=w,
                          log=lambda m: print(m, flush=True))
    secs = time.time() - t0
    z, a = o["z"], o["alpha"]
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    np.save(os.path.join(HERE, "%s_model_z.npy" % name), z)
    np.save(os.path.join(HERE, "%s_model_alpha.npy" % name), a)
    out = {
        "workload": name, "n": n, "kernel": spec["kernel"], "theta": list(spec["theta"]),
        "z": "%s_model_z.npy: z = L w, Sigma = L L^T (dense), w = workloads.gaussian(n, %d)" % (name, spec["w_seed"]),
        "alpha": "%s_model_alpha.npy: Sigma^-1 z = L^-T w" % name,
        "ell": o["ell"], "logdet": o["logdet"], "ztSinvz": float(w @ w),
        "q": list(map(float, o["q"])), "t": list(map(float, o["t"])), "g": list(map(float, o["g"])),
        "alpha_index": sample.tolist(), "alpha_value": [float(a[i]) for i in sample],
        "oracle_seconds": secs,
        "generator": "tests/golden/make_dense_golden.py %s model (oracle.dense only)" % name,
    }
    with open(os.path.join(HERE, "%s_model_dense.json" % name), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %s_model_dense.json in %.1f s" % (name, secs))


if __name__ == "__main__":
    main()

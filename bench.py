"""Benchmark: log-likelihood + score evaluations per second on one MI355X.

One step = one evaluation of Algorithm 1 for a parameter vector theta on fixed
observation sites: build F ~= Sigma(theta) (quadtree, near fields, IDs,
elimination, root), l(theta) from one solve and log|F|, then the score:
F_rho (multiply-only skeletonization of dSigma/drho), the quadratic terms and
the peeled traces of B B^T = Tr F^-1 and B F_rho B^T = Tr F^-1 F_rho
(F^-1 = B^T B).  Inputs are
resident on the device before the timed region.

Workload (default): n = 65536 sites uniform in [0,1]^2 (seed 31), Matern 3/2,
theta = (0.05, 1.0, 1e-4), eps = 1e-6, leaf 64, 256 proxies on 4 rings,
eps_peel = eps; z = L w, the draw from the model by the dense Cholesky factor
(w ~ N(0, I), seed 32; committed with the dense oracle's l, log-det and score
for it, so the line carries the errors against the dense definitions); other
sizes draw z = F^(1/2) w once before timing.  The default run also times the
64-instance batch (one warm-up batch, one timed) against its instances one by
one.

Prints one JSON line (see the repository's design notes for the fields).
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
DEFAULT = "c3_matern32_n65536"
TRAFFIC = os.path.join(HERE, "profiles", "gemm_family_c3_matern32_n65536_traffic.json")
# every library source: the kernels and the host code that sets the launch mix
FAMILY_SOURCES = ["paper_1603_08057_amd/csrc/" + f for f in
                  ("capi.cpp", "common.h", "factor.hip", "gemm.hip", "grad.hip", "rsf.h", "sweep.hip", "tree.cpp")]


def measured_traffic(launches_per_step):
    """HBM bytes per launch of the kernel family from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by the copy-kernel calibration), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in FAMILY_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("sources_sha256") or "family_hbm_bytes_per_step" not in rec:
        return None
    # two counted runs of one and of two steps: their difference is one
    # steady-state step (the setup and the first step's autotuning cancel)
    return rec["family_hbm_bytes_per_step"] / launches_per_step


def bench_mle(args, spec, name, P, z, kw, eps_peel):
    """The MLE loop: L-BFGS-B over log theta (the nugget held fixed) from the
    workload's theta0, every l and g from the library."""
    import torch
    import paper_1603_08057_amd as R
    kw = dict(kw)
    kernel, eps = kw.pop("kernel"), kw.pop("eps")
    leaf = kw.pop("leaf")
    t0 = time.time()
    r = R.fit(P, z, spec["theta0"], kernel, eps=eps, eps_peel=eps_peel, leaf=leaf, seed=spec.get("peel_seed", 0),
              log=sys.stderr, **kw)
    torch.cuda.synchronize()
    el = time.time() - t0
    print(json.dumps({
        "metric": "MLE fit (L-BFGS-B over log theta, nugget fixed)", "seconds": el, "unit": "s",
        "objective_calls": r.nfev, "iterations": r.nit, "success": r.success, "message": r.message,
        "theta_true": list(spec["theta"]), "theta0": list(spec["theta0"]), "theta_hat": [float(v) for v in r.theta],
        "ell_hat": r.ell, "grad_hat": [float(v) for v in r.grad],
        "seconds_per_call": el / max(r.nfev, 1), "n": int(P.shape[0]), "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "eps": eps, "eps_peel": eps_peel, "leaf": leaf}}))


KERNEL_NAMES = {0: "matern12", 1: "matern32", 2: "matern52", 3: "rq", 4: "matern32_aniso", 5: "rq_aniso"}


def cpu_baseline(spec, name, budget_s=35.0):
    """The dense oracle (l and g by FP64 Cholesky) timed on the host on a
    sample n of the same recipe: a 4096-point calibration run, then the
    largest power-of-two n whose O(n^3) extrapolation stays within budget_s;
    scaled to the workload's n by (n / m)^3."""
    import numpy as np
    from oracle import dense
    import workloads as W
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass

    def run(m):
        P = W.workload_points(name, m)
        z = W.gaussian(m, spec["w_seed"])
        t0 = time.time()
        dense.loglik_and_grad(P, z, spec["theta"], spec["kernel"], spec["alpha"], block=2048)
        return time.time() - t0

    m = 4096
    t = run(m)
    while t * 8 <= budget_s and m * 2 <= spec["n"]:
        m *= 2
        t *= 8
    if m > 4096:
        t = run(m)
    scale = (spec["n"] / m) ** 3
    return {"value": 1.0 / (t * scale), "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "dense FP64 oracle l+grad at n=%d (same recipe), %.2f s, scaled by (%d/%d)^3"
                      % (m, t, spec["n"], m),
            "host": host_description()}


def host_description():
    """CPU model and memory of the host (for the CPU baseline record)."""
    out = {}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                out["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                out["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    out["logical_cpus"] = os.cpu_count()
    return out


def dense_errors(spec, P, theta, kw, z, gold, eps_fact, eps_peel, seed):
    """Errors of l, log|F|, the sampled F^-1 z and the score against the dense
    oracle's reference for the same model draw z (committed golden values)."""
    import numpy as np
    import torch
    import paper_1603_08057_amd as R
    kw = dict(kw)
    kw["eps"] = eps_fact
    F = R.Factor(P, theta, with_score=True, **kw)
    ell, alpha = F.loglik(z, want_alpha=True)
    g, info = F.grad(z, eps_peel, seed)
    logdet = F.logdet
    F.close()
    a = alpha.cpu().numpy()
    idx = np.array(gold["alpha_index"])
    ref = np.array(gold["alpha_value"])
    gd, qd, td = np.array(gold["g"]), np.array(gold["q"]), np.array(gold["t"])
    scale = np.abs(qd) + 0.5 * np.abs(td)
    return {"eps_fact": eps_fact, "eps_peel": eps_peel,
            "loglik": abs(ell - gold["ell"]) / abs(gold["ell"]),
            "logdet": abs(logdet - gold["logdet"]) / abs(gold["logdet"]),
            "solve_sampled_max": float(np.max(np.abs(a[idx] - ref)) / np.max(np.abs(ref))),
            "grad_l2": float(np.linalg.norm(np.array(g) - gd) / np.linalg.norm(gd)),
            "grad_over_q_plus_half_t": (np.abs(np.array(g) - gd) / scale).tolist(),
            "traces": (np.abs(np.array(list(info.t)) - td) / np.abs(td)).tolist()}


def measure_batch(args, name, steps, warmup):
    """Independent instances: one batched handle per step (every level of all
    instances in one launch set) against the same instances one by one.
    Returns (seconds per batch, one-by-one seconds, record)."""
    import numpy as np
    import torch
    import paper_1603_08057_amd as R
    import workloads as W
    spec = W.BATCHES[name]
    inst = W.batch_instances(spec["count"], spec["master_seed"])
    dev = torch.device("cuda:0")
    pts = [torch.tensor(p, dtype=torch.float64, device=dev) for p, _ in inst]
    thetas = [th for _, th in inst]
    kw = dict(kernel=spec["kernel"], eps=spec["eps"], leaf=spec["leaf"], n_prox=spec["n_prox"],
              prox_rings=spec["prox_rings"], rq_alpha=spec["alpha"])
    rng = np.random.default_rng(spec["w_seed"])
    B0 = R.BatchedFactor(pts, thetas, **kw)
    zs = B0.apply_sqrt([torch.tensor(rng.standard_normal(len(p)), device=dev) for p in pts])
    B0.close()
    torch.cuda.synchronize()
    ntot = sum(len(p) for p in pts)
    print("setup done: %d instances, %d points" % (len(pts), ntot), file=sys.stderr, flush=True)

    def step_batched():
        B = R.BatchedFactor(pts, thetas, with_score=True, precision=args.precision, **kw)
        ls = B.loglik(zs)
        gs, info = B.grad(zs, spec["eps"], spec["peel_seed"])
        B.close()
        return ls, gs

    def step_single():
        out = []
        for P, th, z in zip(pts, thetas, zs):
            F = R.Factor(P, th, precision=args.precision, **kw)
            ell = F.loglik(z)
            g, _ = F.grad(z, spec["eps"], spec["peel_seed"])
            F.close()
            out.append((ell, g))
        return out

    for i in range(warmup):
        step_batched()
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(steps):
        ls, gs = step_batched()
        print("batched step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb = (time.time() - t0) / steps
    t0 = time.time()
    single = step_single()
    torch.cuda.synchronize()
    ts = time.time() - t0
    print("one by one: %.3f s" % ts, file=sys.stderr, flush=True)
    rel_l = max(abs(a - b[0]) / abs(b[0]) for a, b in zip(ls, single))
    rec = {"workload": name, "instances": len(pts), "points": ntot,
           "n_range": [min(len(p) for p in pts), max(len(p) for p in pts)], "eps": spec["eps"], "leaf": spec["leaf"],
           "seconds_per_batch": tb, "batch_evals_per_s": 1.0 / tb, "steps": steps, "warmup": warmup,
           "one_by_one": {"seconds": ts, "speedup_of_batching": ts / tb, "max_rel_diff_loglik": rel_l}}
    return tb, ts, rec


def bench_batch(args):
    tb, ts, rec = measure_batch(args, args.workload, args.steps, args.warmup)
    out = {
        "metric": "loglik+grad evals/sec of a %d-instance batch (eps=%g)" % (rec["instances"], rec["eps"]),
        "value": 1.0 / tb, "unit": "batch evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * tb, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"precision": args.precision, "workload": args.workload, "instances": rec["instances"],
                   "points": rec["points"], "n_range": rec["n_range"], "eps": rec["eps"], "leaf": rec["leaf"],
                   "parallelism": "single GPU"},
        "one_by_one": rec["one_by_one"],
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT)
    ap.add_argument("--n", type=int, default=None, help="override n (same recipe)")
    ap.add_argument("--eps", type=float, default=None, help="override the factorization tolerance")
    ap.add_argument("--eps-peel", type=float, default=None, help="override the peeling tolerance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-instance batch measurement that the default run appends")
    ap.add_argument("--hutch", type=int, default=0,
                    help="score traces by Hutchinson's estimator with this many probes instead of peeling")
    ap.add_argument("--peeling", choices=["weak", "strong"], default="weak",
                    help="the format the score's traces are peeled in (weakly or strongly admissible)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="arithmetic of the timed factorizations (mixed: FP32 kernel entries and Schur products; "
                         "the data z is drawn in FP64 either way)")
    ap.add_argument("--mle", action="store_true",
                    help="fit theta by the MLE driver from the workload's theta0 (data drawn at its theta) "
                         "and print one JSON line with the fit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device (the known-size run that scales the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1603_08057_amd as R
    import workloads as W

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("copied %d bytes" % (8 * a.numel()))
        return
    if args.workload in W.BATCHES:
        return bench_batch(args)
    spec = dict(W.WORKLOADS[args.workload])
    name = args.workload
    if args.n:
        spec["n"] = args.n
    if args.eps:
        spec["eps"] = args.eps
    if args.eps_peel:
        spec["eps_peel"] = args.eps_peel
    n = spec["n"]
    dev = torch.device("cuda:0")
    P = torch.tensor(W.workload_points(name, n), dtype=torch.float64, device=dev)
    w = torch.tensor(W.gaussian(n, spec["w_seed"]), dtype=torch.float64, device=dev)
    theta = spec["theta"]
    eps_peel = spec.get("eps_peel", spec["eps"])
    kw = dict(kernel=spec["kernel"], eps=spec["eps"], leaf=spec["leaf"], n_prox=spec["n_prox"],
              prox_rings=spec["prox_rings"], rq_alpha=spec["alpha"])
    gold = None
    gpath = os.path.join(HERE, "tests", "golden", "%s_model_dense.json" % name)
    zpath = os.path.join(HERE, "tests", "golden", "%s_model_z.npy" % name)
    if not (args.n or args.eps) and os.path.exists(gpath) and os.path.exists(zpath):
        # the draw from the model by the dense Cholesky factor whose l, log-det
        # and score the dense oracle wrote: the errors below are against it
        gold = json.load(open(gpath))
        z = torch.tensor(np.load(zpath), dtype=torch.float64, device=dev)
    else:
        F0 = R.Factor(P, theta, **kw)
        z = F0.apply_sqrt(w)
        F0.close()
    torch.cuda.synchronize()
    print("setup done: n=%d" % n, file=sys.stderr, flush=True)
    if args.mle:
        return bench_mle(args, spec, name, P, z, kw, eps_peel)

    def step(precision=args.precision):
        # Sigma_rho is factored beside Sigma (second stream), as the score needs it
        F = R.Factor(P, theta, with_score=True, precision=precision, peeling=args.peeling, **kw)
        ell = F.loglik(z)
        if args.hutch > 0:
            g, info = F.grad_hutch(z, args.hutch, spec.get("peel_seed", 0))
        else:
            g, info = F.grad(z, eps_peel, spec.get("peel_seed", 0))
        F.close()
        return ell, g, info

    for i in range(args.warmup):
        t0 = time.time()
        ell, g, info = step()
        print("warmup %d: %.3f s  l=%.6e g=%s  phases=%s" % (i, time.time() - t0, ell, g, list(info.seconds)),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    R.trace_read(reset=True)
    R.trace_enable(True)
    t0 = time.time()
    for i in range(args.steps):
        t1 = time.time()
        ell, g, info = step()
        print("step %d done: %.3f s  peel %.3f s" % (i, time.time() - t1, info.seconds[2]), file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    R.trace_enable(False)
    ms, flops, nbytes, launches, phases = R.trace_read(reset=False, phases=True)
    busy = R.trace_busy_ms()
    R.trace_read(reset=True)
    ms_per_step = 1000.0 * elapsed / args.steps
    # phases are "<phase>" or "<phase>/<sweep direction><depth>": the JSON line
    # carries the phase totals, stderr the per-level split
    totals = {}
    for k, v in sorted(phases.items()):
        top = k.split("/")[0]
        a = totals.setdefault(top, [0.0, 0.0])
        a[0] += v[0]
        a[1] += v[1]
        if "/" in k:
            print("  %-24s %9.2f ms/step %7.2f TFLOP/s" % (k, v[0] / args.steps,
                  (v[1] / (v[0] * 1e-3) / 1e12) if v[0] > 0 else 0.0), file=sys.stderr)
    phases = totals
    achieved = (flops / (ms * 1e-3)) / 1e12 if ms > 0 else 0.0
    out = {
        "metric": ("loglik+grad evals/sec at n=%d (eps=%g)" % (n, spec["eps"]) if args.hutch <= 0 else
                   "loglik+grad (Hutchinson traces, %d probes) evals/sec at n=%d (eps=%g)" % (args.hutch, n, spec["eps"])),
        "value": args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"precision": args.precision, "peeling": args.peeling,
                   "workload": name if not (args.n or args.eps or args.eps_peel) else
                   "%s_recipe_n%d_eps%g_peel%g" % (name, n, spec["eps"], eps_peel), "n": n,
                   "kernel": KERNEL_NAMES.get(spec["kernel"], spec["kernel"]), "theta": list(theta),
                   "eps": spec["eps"], "eps_peel": eps_peel, "leaf": spec["leaf"], "n_prox": spec["n_prox"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma",
                     "kernel": "batched FP64 matrix-core products (gemm_big_kernel, gemm_tiles_kernel, "
                               "box_sweep_kernel)",
                     "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
                     "traffic": (measured_traffic(launches / args.steps)
                                 if not (args.n or args.eps or args.eps_peel) and name == DEFAULT and args.hutch <= 0
                                 else None),
                     "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
                     "launches": launches, "kernel_ms_per_step": ms / args.steps,
                     "flops_per_launch": flops / max(launches, 1),
                     "avg_launch_us": 1000.0 * ms / max(launches, 1),
                     # launches on the two streams overlap: the family's busy time
                     # (union of the launch intervals) and the rate over it
                     "busy_ms_per_step": busy / args.steps,
                     "achieved_over_busy_time": (flops / (busy * 1e-3) / 1e12) if busy > 0 else 0.0,
                     "phases": {k: {"ms_per_step": v[0] / args.steps,
                                    "tflops": (v[1] / (v[0] * 1e-3) / 1e12) if v[0] > 0 else 0.0}
                                for k, v in sorted(phases.items())}},
        "result": {"loglik": ell, "grad": g, "peel_cols": list(info.peel_cols)[:12],
                   "peel_rank": list(info.peel_rank)[:12]},
    }
    if gold is not None and gold.get("g") is not None and args.precision == "fp64" and args.hutch <= 0:
        # untimed: errors against the dense oracle at the benchmark's eps_fact
        # and at eps_fact = eps / 1000 (the paper pairs eps_fact = eps_peel / 1000)
        out["rel_err"] = {
            "reference": "dense FP64 oracle on the model draw z = L w (tests/golden/%s_model_dense.json)" % name,
            "at_benchmark_eps": dense_errors(spec, P, theta, kw, z, gold, spec["eps"], eps_peel,
                                             spec.get("peel_seed", 0)),
            "at_eps_over_1000": dense_errors(spec, P, theta, kw, z, gold, spec["eps"] / 1000, eps_peel,
                                             spec.get("peel_seed", 0))}
    if not args.no_batch and name == DEFAULT and not (args.n or args.eps or args.eps_peel) and args.hutch <= 0:
        print("timing the 64-instance batch", file=sys.stderr, flush=True)
        tb, ts, rec = measure_batch(args, "c4_batch64_matern32", 1, 1)
        out["batch"] = rec
    if args.precision != "fp64":
        # the same evaluation in FP64, untimed: the mixed form's error against it
        ell64, g64, info64 = step("fp64")
        scale = [abs(a) + 0.5 * abs(b) for a, b in zip(info64.q, info64.t)]
        out["vs_fp64"] = {"rel_err_loglik": abs(ell - ell64) / abs(ell64),
                          "grad_err_over_scale": [abs(a - b) / s for a, b, s in zip(g, g64, scale)],
                          "fp64_grad": list(g64)}
    if not args.no_cpu_baseline:
        print("timing the CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spec, name)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

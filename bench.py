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
# every library source (the kernels and the host code that sets the launch mix
# and the probe rule) and the workload recipe: the counters are void once any
# of them changes
FAMILY_SOURCES = ["paper_1603_08057_amd/csrc/" + f for f in
                  ("capi.cpp", "common.h", "factor.hip", "gemm.hip", "grad.hip", "rsf.h", "sweep.hip", "tree.cpp")]
FAMILY_SOURCES.append("workloads/__init__.py")
# the kernels whose launches the library's own trace counts (the roofline's family)
FAMILY_KERNELS = ("gemm_big_kernel", "gemm_tiles_kernel", "box_sweep_kernel")
PMC_COMMAND = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 400 rocprofv3 --pmc {ctr} --output-format csv "
               "-d <out>/{run} -o run -- python3 <repo>/bench.py {args}")
PMC_BENCH_ARGS = "--steps {s} --warmup 0 --no-cpu-baseline --no-batch --no-rel-err"


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in FAMILY_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pmc_rows(d):
    """(kernel name, counter value) per dispatch from a rocprofv3 --pmc csv run
    directory (one counter per run)."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit("%s: expected one counter_collection.csv, found %d" % (d, len(files)))
    per = {}
    with open(files[0]) as fh:
        for row in csv.DictReader(fh):
            key = row["Dispatch_Id"]
            name = row["Kernel_Name"]
            per[key] = (name, per.get(key, (name, 0.0))[1] + float(row["Counter_Value"]))
    return list(per.values())


def traffic_record(root):
    """Write the family's HBM traffic record and the per-kernel FETCH_SIZE /
    WRITE_SIZE summaries from the counter runs under root: fetch_1, fetch_2,
    write_1, write_2 (the benchmark at one and at two steps) and cal_fetch,
    cal_write (the 1 GiB copy)."""
    def fam(name):
        return any(k in name for k in FAMILY_KERNELS)

    def per_kernel(rows):
        out = {}
        for name, v in rows:
            a = out.setdefault(name, [0, 0.0])
            a[0] += 1
            a[1] += v
        return out

    runs = {k: per_kernel(_pmc_rows(os.path.join(root, k)))
            for k in ("fetch_1", "fetch_2", "write_1", "write_2", "cal_fetch", "cal_write")}

    def copy_kib(r):
        return sum(v for name, (c, v) in runs[r].items() if "copyBuffer" in name)

    copy_bytes = 1 << 30
    cal = {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": copy_kib("cal_fetch"), "WRITE_SIZE_KiB": copy_kib("cal_write")}
    cal["fetch_scale"] = copy_bytes / 1024.0 / cal["FETCH_SIZE_KiB"]
    cal["write_scale"] = copy_bytes / 1024.0 / cal["WRITE_SIZE_KiB"]
    rec = {"kernel_family": "batched FP64 matrix-core products: " + ", ".join(k + "<...>" for k in FAMILY_KERNELS),
           "workload": "%s, one steady-state step (difference of a two-step and a one-step run)" % DEFAULT,
           "commands": [PMC_COMMAND.format(ctr=c, run=c.split("_")[0].lower() + "_S",
                                           args=PMC_BENCH_ARGS.format(s="S")) + "   (S = 1 and S = 2)"
                        for c in ("FETCH_SIZE", "WRITE_SIZE")] + [
               "one steady-state step = the S = 2 run minus the S = 1 run (the setup and the first step's "
               "autotuning cancel)",
               "calibration: " + PMC_COMMAND.format(ctr="FETCH_SIZE (then WRITE_SIZE)", run="cal_fetch",
                                                    args="--copy-calibration") + " (a 1 GiB device-to-device copy)",
               "record: python3 bench.py --traffic-record <out>"],
           "calibration": cal, "runs": {}}
    step = {}
    for ctr in ("fetch", "write"):
        a, b = runs[ctr + "_1"], runs[ctr + "_2"]
        rec["runs"][ctr + "_1"] = [sum(c for n, (c, v) in a.items() if fam(n)), sum(v for n, (c, v) in a.items() if fam(n))]
        rec["runs"][ctr + "_2"] = [sum(c for n, (c, v) in b.items() if fam(n)), sum(v for n, (c, v) in b.items() if fam(n))]
        diff = {n: (b[n][0] - a.get(n, (0, 0.0))[0], b[n][1] - a.get(n, (0, 0.0))[1]) for n in b}
        step[ctr] = diff
        label = "FETCH_SIZE" if ctr == "fetch" else "WRITE_SIZE"
        lines = ["%s (KiB) per kernel for one steady-state step: dispatches, KiB, kernel, as the difference of two "
                 "runs: %s, with S = 2 minus S = 1; ×%.4f gives bytes of HBM traffic by the copy calibration"
                 % (label, PMC_COMMAND.format(ctr=label, run=ctr + "_S", args=PMC_BENCH_ARGS.format(s="S")),
                    1024.0 * cal[ctr + "_scale"])]
        for n, (c, v) in sorted(diff.items(), key=lambda kv: -kv[1][1]):
            if c > 0 and v > 0:
                lines.append("%10d %16.1f %s" % (c, v, n[:140]))
        with open(os.path.join(HERE, "profiles", "gemm_family_%s_%s.txt" % (DEFAULT, label.lower())), "w") as fh:
            fh.write("\n".join(lines[:40]) + "\n")
    rec["family_dispatches_per_step"] = sum(c for n, (c, v) in step["fetch"].items() if fam(n))
    rec["family_dispatches_per_step_write_runs"] = sum(c for n, (c, v) in step["write"].items() if fam(n))
    rec["family_FETCH_SIZE_KiB_per_step"] = sum(v for n, (c, v) in step["fetch"].items() if fam(n))
    rec["family_WRITE_SIZE_KiB_per_step"] = sum(v for n, (c, v) in step["write"].items() if fam(n))
    rec["sources_sha256"] = sources_sha256()
    rec["family_hbm_bytes_per_step"] = 1024.0 * (rec["family_FETCH_SIZE_KiB_per_step"] * cal["fetch_scale"] +
                                                 rec["family_WRITE_SIZE_KiB_per_step"] * cal["write_scale"])
    with open(TRAFFIC, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: rec[k] for k in ("family_dispatches_per_step", "family_hbm_bytes_per_step")}))


def _pmc_by_kernel(d):
    """{kernel: {"n": dispatches, "ns": summed durations, counter: summed value}}
    from a rocprofv3 --pmc csv run directory."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit("%s: expected one counter_collection.csv, found %d" % (d, len(files)))
    disp = {}
    with open(files[0]) as fh:
        for row in csv.DictReader(fh):
            e = disp.setdefault(row["Dispatch_Id"], {"name": row["Kernel_Name"],
                                                     "ns": float(row["End_Timestamp"]) - float(row["Start_Timestamp"])})
            e[row["Counter_Name"]] = e.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    out = {}
    for e in disp.values():
        if "MfmaUtil" in e:
            e["MfmaUtil_ns"] = e["MfmaUtil"] * e["ns"]  # the busy share, weighted by duration
        a = out.setdefault(e["name"], {"n": 0})
        a["n"] += 1
        for k, v in e.items():
            if k != "name":
                a[k] = a.get(k, 0.0) + v
    return out


def _step_diff(a, b):
    """Per-kernel difference of the two-step and the one-step run."""
    out = {}
    for name, eb in b.items():
        ea = a.get(name, {})
        out[name] = {k: v - ea.get(k, 0.0) for k, v in eb.items()}
    return out


def _short(name):
    base = name.split("(")[0].replace("void ", "").replace("rsf::", "")
    return base


def frac_record(root):
    """Per-kernel fraction of peak for one steady-state step, from the counter
    runs under root: mfma_1, mfma_2 (MfmaFlopsF64, MfmaUtil and
    SQ_INSTS_VALU_FLOPS_FP64 at one and two steps), the FETCH_SIZE / WRITE_SIZE
    runs and their copy calibration (as for the traffic record)."""
    mf = _step_diff(_pmc_by_kernel(os.path.join(root, "mfma_1")), _pmc_by_kernel(os.path.join(root, "mfma_2")))
    fe = _step_diff(_pmc_by_kernel(os.path.join(root, "fetch_1")), _pmc_by_kernel(os.path.join(root, "fetch_2")))
    wr = _step_diff(_pmc_by_kernel(os.path.join(root, "write_1")), _pmc_by_kernel(os.path.join(root, "write_2")))
    cal_f = sum(e.get("FETCH_SIZE", 0.0) for n, e in _pmc_by_kernel(os.path.join(root, "cal_fetch")).items()
                if "copyBuffer" in n)
    cal_w = sum(e.get("WRITE_SIZE", 0.0) for n, e in _pmc_by_kernel(os.path.join(root, "cal_write")).items()
                if "copyBuffer" in n)
    fscale, wscale = (1 << 30) / cal_f, (1 << 30) / cal_w  # bytes per counted KiB
    # algorithmic work per kernel and step, booked by the library during the
    # two-step counter run
    work = {}
    try:
        with open(os.path.join(root, "mfma_2.json")) as fh:
            line = [l for l in fh.read().splitlines() if l.startswith("{")][-1]
        work = json.loads(line)["roofline"].get("kernel_work_per_step", {})
    except (OSError, IndexError, ValueError, KeyError):
        pass
    cmd = PMC_COMMAND.format(ctr="MfmaFlopsF64 MfmaUtil SQ_INSTS_VALU_FLOPS_FP64", run="mfma_S",
                             args=PMC_BENCH_ARGS.format(s="S"))
    lines = ["# Per-kernel fraction of peak: %s, one steady-state step" % DEFAULT, "",
             "Commands (S = 1 and S = 2; one step = the S = 2 run minus the S = 1 run):", "", "```", cmd,
             PMC_COMMAND.format(ctr="FETCH_SIZE", run="fetch_S", args=PMC_BENCH_ARGS.format(s="S")),
             PMC_COMMAND.format(ctr="WRITE_SIZE", run="write_S", args=PMC_BENCH_ARGS.format(s="S")),
             PMC_COMMAND.format(ctr="FETCH_SIZE", run="cal_fetch", args="--copy-calibration") +
             "   (and WRITE_SIZE into cal_write)",
             "python3 bench.py --frac-record <out>", "```", "",
             "Durations are the counter runs' dispatch timestamps: under --pmc every dispatch runs alone, so "
             "they are the kernels' own times without the second stream beside them.  MFMA flops are the "
             "hardware's count (MfmaFlopsF64 = 512 x SQ_INSTS_VALU_MFMA_MOPS_F64), padding and skipped "
             "triangles included; MFMA util is the busy share of the matrix cores over the dispatch "
             "(MfmaUtil, weighted by duration).  HBM bytes are FETCH_SIZE and WRITE_SIZE scaled by what "
             "they read for a 1 GiB copy (x%.3f and x%.3f).  Peaks: FP64 matrix 78.6 TFLOP/s, HBM 8 TB/s, "
             "FP64 vector 78.6 TFLOP/s." % (fscale / 1024, wscale / 1024), "",
             "Algorithmic columns: the work the library books per kernel (2 M N K flops per product, M N K "
             "for a lower-triangle or triangular-operand product, so no zero triangle and no unused quadrant "
             "counts; 2 c r (2 k + r) per box and column for the fused level steps; for the pivoting steps of "
             "the interpolative decompositions 16 bytes per entry of the trailing block each step reads and "
             "writes) over the kernel's own time; the same rate against the peak of the kernel's bound "
             "(FP64 matrix for the products, HBM for the pivoting steps) is the frac.", "",
             "| kernel | dispatches | ms | alg. TFLOP/s | alg. GB/s | frac (alg.) | MFMA TFLOP/s (hw) | "
             "MFMA util % | VALU FP64 TFLOP/s | HBM GB | HBM TB/s |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    # kernels booked under their name without template arguments (the ID's
    # update kernel, one instantiation per register bucket) are summed over
    # their instantiations
    def merge(d):
        out = {}
        for name, e in d.items():
            short = _short(name)
            base = short.split("<")[0]
            key = base if (short not in work and base in work) else name
            a = out.setdefault(key, {})
            for k, v in e.items():
                a[k] = a.get(k, 0.0) + v
        return out

    mf, fe, wr = merge(mf), merge(fe), merge(wr)
    rows = []
    for name, e in mf.items():
        if e["n"] <= 0 or e["ns"] <= 0:
            continue
        hb = fe.get(name, {}).get("FETCH_SIZE", 0.0) * fscale + wr.get(name, {}).get("WRITE_SIZE", 0.0) * wscale
        rows.append((e["ns"], name, e, hb))
    rows.sort(key=lambda r: -r[0])
    tot = {"ns": 0.0, "fl": 0.0, "hb": 0.0}
    fam = {"ns": 0.0, "fl": 0.0, "hb": 0.0, "util": 0.0, "n": 0}
    alg = {"fl": 0.0}
    for ns, name, e, hb in rows[:28]:
        s = ns * 1e-9
        util = e.get("MfmaUtil_ns", 0.0) / ns
        w = work.get(_short(name))
        afl = w["gflop"] * 1e9 / s / 1e12 if w else None
        aby = w["gbyte"] * 1e9 / s / 1e9 if w else None
        if w is None:
            frac = "-"
        elif "cpqr" in name:
            frac = "%.3f" % (aby / 8000.0)
        else:
            frac = "%.3f" % (afl / FP64_MFMA_PEAK_TFLOPS)
        lines.append("| `%s` | %d | %.2f | %s | %s | %s | %.2f | %.1f | %.3f | %.2f | %.2f |" % (
            _short(name), int(e["n"]), ns * 1e-6, "%.2f" % afl if w else "-", "%.0f" % aby if w else "-", frac,
            e.get("MfmaFlopsF64", 0.0) / s / 1e12, util, e.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) / s / 1e12,
            hb / 1e9, hb / s / 1e12))
    for ns, name, e, hb in rows:
        tot["ns"] += ns
        tot["fl"] += e.get("MfmaFlopsF64", 0.0)
        tot["hb"] += hb
        if any(k in name for k in FAMILY_KERNELS):
            fam["ns"] += ns
            fam["fl"] += e.get("MfmaFlopsF64", 0.0)
            fam["hb"] += hb
            w = work.get(_short(name))
            alg["fl"] += w["gflop"] * 1e9 if w else 0.0
    fs = fam["ns"] * 1e-9
    lines += ["", "Matrix-core family (%s): %.1f ms of dispatch time per step; algorithmic %.3e flops, %.2f TFLOP/s "
              "(frac %.3f of the FP64 matrix peak); the hardware's MFMA count %.3e flops, %.2f TFLOP/s (%.3f); "
              "%.1f GB of HBM traffic (%.2f TB/s).  All kernels: %.1f ms."
              % (", ".join(FAMILY_KERNELS), fam["ns"] * 1e-6, alg["fl"], alg["fl"] / fs / 1e12,
                 alg["fl"] / fs / 1e12 / FP64_MFMA_PEAK_TFLOPS, fam["fl"], fam["fl"] / fs / 1e12,
                 fam["fl"] / fs / 1e12 / FP64_MFMA_PEAK_TFLOPS, fam["hb"] / 1e9, fam["hb"] / fs / 1e12,
                 tot["ns"] * 1e-6)]
    path = os.path.join(HERE, "profiles", "kernel_frac_%s.md" % DEFAULT)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", path)


def measured_traffic(launches_per_step):
    """HBM bytes per launch of the kernel family from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by the copy-kernel calibration), or None
    when the kernel sources changed since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC))
    except (OSError, ValueError):
        return None
    if sources_sha256() != rec.get("sources_sha256") or "family_hbm_bytes_per_step" not in rec:
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

    # both forms are warmed up: their first calls time the autotuners' trials
    # for launch shapes not seen before (the instances alone have shapes of
    # their own)
    for i in range(warmup):
        step_batched()
    if warmup > 0:
        step_single()
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
    ap.add_argument("--no-rel-err", action="store_true",
                    help="skip the untimed evaluations that measure the error against the dense oracle")
    ap.add_argument("--traffic-record", metavar="DIR", default=None,
                    help="(no GPU) write the family's HBM traffic record from the FETCH_SIZE / WRITE_SIZE counter "
                         "runs under DIR (fetch_1, fetch_2, write_1, write_2, cal_fetch, cal_write)")
    ap.add_argument("--frac-record", metavar="DIR", default=None,
                    help="(no GPU) write the per-kernel fraction-of-peak table from the counter runs under DIR "
                         "(mfma_1, mfma_2 and the traffic runs)")
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
    if args.traffic_record:
        return traffic_record(args.traffic_record)
    if args.frac_record:
        return frac_record(args.frac_record)
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
    kern = R.trace_kernels()
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
                     # algorithmic work per kernel (host counts; the counter runs
                     # divide it by each kernel's own time)
                     "kernel_work_per_step": {k: {"gflop": v[0] / args.steps / 1e9, "gbyte": v[1] / args.steps / 1e9,
                                                  "dispatches": v[2] / args.steps}
                                              for k, v in sorted(kern.items())},
                     "phases": {k: {"ms_per_step": v[0] / args.steps,
                                    "tflops": (v[1] / (v[0] * 1e-3) / 1e12) if v[0] > 0 else 0.0}
                                for k, v in sorted(phases.items())}},
        "result": {"loglik": ell, "grad": g, "peel_cols": list(info.peel_cols)[:12],
                   "peel_rank": list(info.peel_rank)[:12]},
    }
    if (gold is not None and gold.get("g") is not None and args.precision == "fp64" and args.hutch <= 0
            and not args.no_rel_err):
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

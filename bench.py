"""Benchmark of the H^2-ULV factorization (+ refined solve) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--form fp64|mixed|predicted|mixed+predicted]
                    [--refine gmres|classical] [--no-reference] [--no-cpu-baseline]

One step = factorize the workload's kernel matrix, then solve its right-hand
sides with iterative refinement (exact float64 matvec) down to a relative
residual of 1e-10; by default the correction equation is solved by GMRES
preconditioned with the ULV solve (--refine classical: x += solve(b - A x)).
Points and right-hand sides are resident on the GPU before the timed region.
Prints one JSON line.

Forms: fp64 (the plain method), mixed (FP32 products where the method allows),
predicted (bases from sketches sized by the learned rank model), and both
combined.  A rank model is trained first (outside the timed steps) on the
ranks of factorizations of two other point sets of the same family.

value = algorithmic flops of the plain FP64 factorization of the workload (the
paper's step costs from its actual ranks) / wall time of one step of the timed
form: an effective rate, so that forms that skip work are compared at equal
delivered accuracy.  The plain FP64 form is also timed (the reference) unless
--no-reference; without it the form's own flop count is used.
roofline = the dominant kernel (by time) of the timed steps measured with HIP
events on its launch stream: summed algorithmic flops / summed duration.
roofline.traffic = HBM bytes per launch of that kernel in the timed step, from
the rocprofv3 FETCH_SIZE / WRITE_SIZE counters recorded in
profiles/gemm_f64_traffic_ellipsoids262144.md (scaled by the same counters'
reading for a plain copy of known size, --copy-probe); null when the library
sources differ from those the counters were taken with (source hash).
cpu_baseline = the CPU oracle timed on a bounded sample of leaf boxes of the
same workload (GFLOP/s of the oracle's own flop count).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H² ULV factorize time + GFLOP/s, N=1M Laplace, mixed vs FP64 at 1e-10 resid"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f64_traffic_ellipsoids262144.md")


def library_source_hash() -> str:
    """sha256 over the library's device and host sources (sorted by name): the
    launch mix and the GEMM kernel both come from them."""
    import hashlib
    d = os.path.join(ROOT, "paper_2208_10907_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(d, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str):
    """HBM bytes per launch of the FP64 GEMM recorded for this workload, if the
    record was taken with the current library sources."""
    if workload != "ellipsoids262144" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            line = line.strip().strip("`")
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("library_source_sha256") != library_source_hash():
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
PEAK_TFLOPS = {"gemm_f64": 78.6, "gemm_f32": 157.3}


def workloads():
    import workloads as W
    return {
        "cube2048": lambda: W.small_cube(),
        "sphere65536": lambda: W.sphere65k(),
        "ellipsoids262144": lambda: W.ellipsoids(),
        "cube1048576": lambda: W.cube1m(),
    }


def training_sets(name):
    """Point sets the rank model learns from: the same family, other seeds."""
    import workloads as W
    if name.startswith("ellipsoids"):
        # two smaller sets and one of the workload's size (its upper levels are
        # larger than any box of the smaller sets)
        return ([(f"ellipsoids65536 seed {s}", lambda s=s: W.ellipsoid_points(65536, s))
                 for s in (501, 502)]
                + [("ellipsoids262144 seed 503", lambda: W.ellipsoid_points(262144, 503))])
    if name.startswith("sphere"):
        return [(f"sphere16384 seed {s}", lambda s=s: W.sphere_points(16384, s))
                for s in (501, 502)]
    return [(f"cube32768 seed {s}", lambda s=s: W.cube_points(32768, s)) for s in (501, 502)]


def describe(prob):
    kern = "laplace" if prob.kernel == 0 else f"yukawa(alpha={prob.alpha})"
    return (f"{prob.name}: N={prob.n}, kernel {kern}, diag {prob.diag:g}, leaf {prob.leaf}, "
            f"eta {prob.eta:g}, tol {prob.tol:g}, rank cap {prob.rank_cap or 'none'}, "
            f"far samples {prob.far_sample}, {prob.nrhs} Gaussian RHS")


def cpu_baseline(prob, budget_s=20.0):
    """Time the oracle on leaf boxes of the same workload (restricted to what the
    sample depends on); report its flops / time."""
    import numpy as np
    from oracle import h2ulv_ref as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    op = O.params_from_problem(prob)
    tree_L = O.tree_depth(prob.n, prob.leaf)
    nb = 1 << tree_L
    rng = np.random.default_rng(0)
    total_fl, total_t, boxes = 0.0, 0.0, []
    for _ in range(64):
        box = int(rng.integers(nb))
        t0 = time.perf_counter()
        f = O.factorize(prob.points, op, level_stop=tree_L, boxes={box})
        dt = time.perf_counter() - t0
        total_fl += sum(f.stats["flops"].values())
        total_t += dt
        boxes.append(box)
        if total_t > budget_s:
            break
    return {"value": round(total_fl / total_t / 1e9, 3), "unit": "GFLOP/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"leaf-level basis step (dense blocks, fill-ins, row ID, complement) of "
                       f"{len(boxes)} leaf boxes of {prob.name}, each with the near blocks it "
                       f"depends on; {total_t:.1f} s of CPU time; oracle flop count")}


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def train_model(H, torch, prob, name):
    """Factorize the training point sets (plain FP64), collect the per-box
    features and ranks, train the rank MLP on the GPU."""
    import numpy as np
    t0 = time.perf_counter()
    base = H.params_from_problem(prob)
    F, T, names = [], [], []
    for label, mk in training_sets(name):
        f = H.factorize(mk(), base)
        for lev in range(1, f.levels() + 1):
            a, b = f.features(lev)
            F.append(a)
            T.append(b)
        names.append(label)
        del f
        log(f"training factorization {label} done")
    F = np.concatenate(F)
    T = np.concatenate(T)
    model = H.RankModel(seed=1)
    t1 = time.perf_counter()
    loss = model.train(torch.tensor(F, device="cuda"), torch.tensor(T, device="cuda"), 3000, 3e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"rank model trained: {F.shape[0]} boxes, loss {loss:.4f}")
    return model, {"train_sets": names, "samples": int(F.shape[0]),
                   "factorize_s": round(t1 - t0, 3), "train_s": round(t2 - t1, 3),
                   "steps": 3000, "final_loss": round(loss, 5)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoids262144", choices=sorted(workloads()))
    ap.add_argument("--form", default="mixed+predicted",
                    choices=["fp64", "mixed", "predicted", "mixed+predicted"])
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--refine", default="gmres", choices=["gmres", "classical"],
                    help="correction solver of the refinement (both forms use the same)")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--window-file", default=None,
                    help="write the timed region's start and end (time.monotonic_ns) here, "
                         "to match a profiler trace to the timed steps")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB from one device buffer to another (the known-size "
                         "calibration kernel for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe << 20}))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (the distributed process tree of the paper "
              "is a design note, not built); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2208_10907_amd import h2ulv as H

    prob = workloads()[args.workload]()
    pts = torch.tensor(prob.points, device="cuda")
    b = torch.tensor(prob.rhs(), device="cuda")
    torch.cuda.synchronize()

    model, model_info = None, None
    if "predicted" in args.form:
        model, model_info = train_model(H, torch, prob, args.workload)

    def params_of(form):
        prec = H.MIXED if "mixed" in form else H.FP64
        return H.params_from_problem(prob, precision=prec,
                                     rank_model=model if "predicted" in form else None,
                                     sketch_seed=5)

    def step(params):
        t0 = time.perf_counter()
        f = H.factorize(pts, params)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if args.refine == "gmres":
            x, iters, rel = f.refine_gmres(b, rtol=args.rtol, max_iter=60, restart=30)
        else:
            x, iters, rel = f.refine(b, rtol=args.rtol, max_iter=60)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = f.stats()
        sk = [0, 0, 0, 0]  # outcome per box: not sketched, accepted, rejected, retried and accepted
        for lev in range(1, f.levels() + 1):
            s = f.sketch_info(lev)[2]
            for o in range(4):
                sk[o] += int((s == o).sum())
        del f
        return {"factor_s": t1 - t0, "refine_s": t2 - t1, "iters": iters, "rel": rel, "st": st,
                "sketches": {"accepted": sk[1], "retried_accepted": sk[3],
                             "rejected_full_qr": sk[2], "not_sketched": sk[0]}}

    form_params = params_of(args.form)
    for w in range(args.warmup):
        r = step(form_params)
        log(f"warmup step {w + 1}/{args.warmup} done ({r['factor_s']:.2f} s factorize, "
            f"{r['refine_s']:.2f} s refine)")
    torch.cuda.synchronize()
    H.profile_enable(True)
    w_start = time.monotonic_ns()
    t_start = time.perf_counter()
    res = []
    for i in range(args.steps):
        res.append(step(form_params))
        log(f"timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    if args.window_file:
        with open(args.window_file, "w") as fh:
            fh.write(f"{w_start} {time.monotonic_ns()}\n")
    prof = H.profile_read()
    H.profile_enable(False)
    ms = 1e3 * t_total / args.steps
    last = res[-1]
    st = last["st"]

    ref = None
    if not args.no_reference and args.form != "fp64":
        r = step(params_of("fp64"))
        log(f"reference fp64 step done ({r['factor_s']:.2f} s factorize)")
        ref = {"form": "fp64", "step_s": round(r["factor_s"] + r["refine_s"], 4),
               "factor_s": round(r["factor_s"], 4), "refine_s": round(r["refine_s"], 4),
               "refine_iters": r["iters"], "relres": r["rel"], "flops": r["st"]["flops"],
               "max_rank": r["st"]["max_rank"], "device_gb": round(r["st"]["device_bytes"] / 1e9, 2)}
    work = ref["flops"] if ref else st["flops"]
    value = work / (ms / 1e3) / 1e9

    # the GEMM profile is split by call site ("gemm_f64:<site>"): one kernel, summed
    gemms = {}
    for k, v in prof.items():
        base = k.split(":")[0]
        if base in PEAK_TFLOPS:
            a = gemms.setdefault(base, {"launches": 0, "time_ms": 0.0, "flops": 0.0,
                                        "bytes": 0.0})
            a["launches"] += v["launches"]
            a["time_ms"] += v["time_ms"]
            a["flops"] += v["flops"]
            a["bytes"] += v["bytes"]
    dom = max(gemms, key=lambda k: gemms[k]["time_ms"]) if gemms else None
    roof = None
    if dom:
        g = gemms[dom]
        ach = g["flops"] / (g["time_ms"] / 1e3) / 1e12
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(ach, 3),
                "peak": PEAK_TFLOPS[dom], "unit": "TFLOP/s",
                "frac": round(ach / PEAK_TFLOPS[dom], 4),
                "traffic": recorded_traffic(args.workload) if dom == "gemm_f64" else None,
                "launches": g["launches"],
                "avg_launch_ms": round(g["time_ms"] / g["launches"], 4),
                "flops_per_launch": g["flops"] / g["launches"],
                # operands read once and results written once, per launch
                "algorithmic_bytes_per_launch": g["bytes"] / g["launches"]}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if "mixed" in args.form else "f64",
        "data": "synthetic",
        "config": {"workload": describe(prob), "form": args.form, "refine_rtol": args.rtol,
                   "refine": args.refine,
                   "value_flops": "plain FP64 method" if ref else "this form"},
        "factor_s": round(last["factor_s"], 4),
        "refine_s": round(last["refine_s"], 4),
        "refine_iters": last["iters"],
        "relres": last["rel"],
        "flops": st["flops"],
        "max_rank": st["max_rank"],
        "root_size": st["root_size"],
        "device_gb": round(st["device_bytes"] / 1e9, 2),
        "sketches": last["sketches"],
        "reference": ref,
        "speedup_vs_fp64": round(ref["step_s"] / (ms / 1e3), 3) if ref else None,
        "rank_model": model_info,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["time_ms"], 2),
                        "tflops": round(v["flops"] / max(v["time_ms"], 1e-9) / 1e9, 3)}
                    for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

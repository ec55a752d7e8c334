"""Benchmark: SP-SVM training time on one MI355X, with roofline and CPU-oracle baseline.

One step = one complete greedy SP-SVM training run (basis selection + Newton re-optimisation to |J| = J_max,
every row of the hot path) on a fixed synthetic workload already resident in HBM. Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload binary-100k] [--precision f32]

The default workload is the 100 000 x 123 binary one (|J| = 1000, C = 1, gamma = 0.05). With
--workload mnist-60k a step is instead one batched call: 160 one-vs-rest x (C, gamma) Newton solves on a shared
basis of 2000 rows of a 60 000 x 784 matrix. The dominant kernel
(largest GPU time among kernel block, SYRK, score passes, Cholesky, found on the first warm-up run) is timed
with HIP events on the training stream during the timed steps, for the roofline entry. Parity of the first
timed run is checked against the FP64 oracle (objective at the GPU's basis, sampled decision values), and the
oracle itself is timed on a bounded sample of the same workload (the CPU baseline).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train sec to oracle objective (rel 1e-6), mixed vs FP32; K-block TFLOP/s"
PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_mfma_TFLOPs": 78.6,
    "fp32_mfma_TFLOPs": 157.3,
}
# Timed steps bracket every 8th launch of the profiled kernels with HIP events (each bracket delays the stream
# a few microseconds, so timing every launch would slow the steps being measured).
PROFILE_STRIDE = 8 << 8
CATS = {  # profile bit -> (stats prefix, unit of work, bound)
    1: ("kblock", "flops", "mfma"),
    2: ("syrk", "flops", "mfma"),
    4: ("score", "bytes", "hbm"),
    8: ("chol", "flops", "mfma"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="binary-100k")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=12)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 256 MiB device buffer 3 times (a plain copy kernel of known size, to calibrate "
                         "hardware byte counters)")
    return ap.parse_args()


def copy_probe():
    import torch

    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 256 MiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


KERNEL_OF = {"kblock": "k_kblock_store", "syrk": "k_syrk", "score": "k_score_pass", "chol": "k_potrf_diag"}


def measured_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed byte-counter summary of this workload, or None when
    there is none or the kernel's source file changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{KERNEL_OF.get(kernel, kernel)}_{workload}.txt")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.loads(fh.read().strip().splitlines()[-1])
        with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["bytes_per_dispatch"]
    except (OSError, ValueError, KeyError, TypeError):
        return None


def roofline_entry(stats, bit, precision):
    pre, unit, bound = CATS[bit]
    sec = stats[f"{pre}_seconds"]
    work = stats[f"{pre}_{'bytes' if unit == 'bytes' else 'flops'}"]
    launches = stats[f"{pre}_launches" if pre != "chol" else "chol_calls"]
    if sec <= 0:
        return None
    if bound == "hbm":
        achieved = work / sec / 1e9
        peak, u = PEAKS["hbm_GBps"], "GB/s"
    else:
        achieved = work / sec / 1e12
        fp64 = pre in ("syrk", "chol") or precision == "f64"
        peak = PEAKS["fp64_mfma_TFLOPs"] if fp64 else PEAKS["fp32_mfma_TFLOPs"]
        u = "TFLOP/s"
    return {"kernel": pre, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": u,
            "frac": round(achieved / peak, 4), "traffic": None, "launches": launches,
            "avg_launch_us": round(1e6 * sec / max(launches, 1), 3),
            "work_per_launch": work / max(launches, 1)}


def run_batch(args):
    """The batched workload: 160 one-vs-rest x (C, gamma) Newton solves on one shared basis; one step is one
    spsvm_train_batch call over all of them."""
    import numpy as np
    import torch

    import datagen
    import paper_1404_1066_amd as lib

    p = datagen.make_config(args.workload)
    n, d = p.X.shape
    P, m = p.Y.shape[0], len(p.J)
    dt = torch.float64 if args.precision == "f64" else torch.float32
    Xg = torch.tensor(p.X, dtype=dt, device="cuda")
    Yg = torch.tensor(p.Y, dtype=torch.float32, device="cuda")
    ws = torch.empty(lib.workspace_bytes(n, d, m, batch=True, problems=P, dtype=dt, precision=args.precision),
                     dtype=torch.uint8, device="cuda")
    common = dict(precision=args.precision, workspace=ws, stream=torch.cuda.current_stream())
    warm = None
    for w in range(max(args.warmup, 1)):
        ms = lib.train_batch(Xg, Yg, p.C, p.gamma, p.J, profile=15 if w == 0 else 0, **common)
        if w == 0:
            warm = ms[-1].stats()  # kernel timings cover the whole batch
    dominant = max(CATS, key=lambda b: warm[f"{CATS[b][0]}_seconds"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    runs = []
    for k in range(args.steps):
        runs.append(lib.train_batch(Xg, Yg, p.C, p.gamma, p.J, profile=(dominant | 1) | PROFILE_STRIDE, **common))
    torch.cuda.synchronize()
    per_run = (time.perf_counter() - t1) / args.steps
    agg = {}
    for key in warm:
        agg[key] = sum(r[-1].stats()[key] for r in runs)
    out = {
        "metric": METRIC,
        "value": round(per_run, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * per_run, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "problems": P, "m": m,
                   "C": sorted(set(float(c) for c in p.C)), "gamma": sorted(set(float(g) for g in p.gamma)),
                   "precision": args.precision},
        "roofline": roofline_entry(agg, dominant, args.precision),
        "kblock": roofline_entry(agg, 1, args.precision),
        "kernels_warmup": {CATS[b][0]: roofline_entry(warm, b, args.precision) for b in CATS},
    }
    if out["roofline"] is not None:
        out["roofline"]["traffic"] = measured_traffic(args.workload, out["roofline"]["kernel"])
    from oracle import spsvm as osp

    if not args.no_parity:
        par = []
        for q in (0, P - 1):
            _, beta, _ = runs[0][q].get()
            tq = time.perf_counter()
            b_or, F_or, _ = osp.solve_fixed_J(p.X, p.Y[q], p.C[q], p.gamma[q], p.J)
            oracle_s = time.perf_counter() - tq
            Fo = osp.objective_at(p.X, p.Y[q], p.C[q], p.gamma[q], p.J, beta)
            par.append({"problem": q, "objective_rel": (Fo - F_or) / F_or, "objective_ok": bool((Fo - F_or) / F_or <= 1e-6)})
        out["parity"] = par
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {
                "value": round(oracle_s * P, 3), "unit": "s", "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                "sample": f"FP64 oracle fixed-basis Newton solve of problem {P - 1} ({oracle_s:.2f} s), times {P} problems"}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
    if args.workload == "mnist-60k":
        run_batch(args)
        return
    import numpy as np
    import torch

    import datagen
    import paper_1404_1066_amd as lib

    t0 = time.time()
    p = datagen.make_config(args.workload)
    gen_s = time.time() - t0
    n, d = p.X.shape
    dt = torch.float64 if args.precision == "f64" else torch.float32
    Xg = torch.tensor(p.X, dtype=dt, device="cuda")
    yg = torch.tensor(p.y, dtype=torch.float32, device="cuda")
    # sized for the mixed-precision runs too (they also hold the split-BF16 copies of X)
    ws_prec = "mixed" if (args.precision == "f32" and not args.no_mixed) else args.precision
    ws = torch.empty(lib.workspace_bytes(n, d, p.J_max, dtype=dt, precision=ws_prec), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    common = dict(precision=args.precision, workspace=ws, stream=stream)

    # warm-up; the first one is profiled on every kernel class to find the dominant kernel
    dominant, warm_stats = 2, None
    for w in range(max(args.warmup, 1)):
        m = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=1000 + w, profile=15 if w == 0 else 0, **common)
        if w == 0:
            warm_stats = m.stats()
            dominant = max(CATS, key=lambda b: warm_stats[f"{CATS[b][0]}_seconds"])
        del m
    torch.cuda.synchronize()

    models, stats = [], []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):  # the kernel block is timed too (the metric's K-block TFLOP/s); every 8th launch
        models.append(lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=k, profile=(dominant | 1) | PROFILE_STRIDE,
                                **common))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    per_run = (t2 - t1) / args.steps
    for m in models:
        stats.append(m.stats())

    # roofline of the dominant kernel over the timed region (sum of the timed runs' event timings)
    agg = {}
    for key in stats[0]:
        agg[key] = sum(s[key] for s in stats)
    roof = roofline_entry(agg, dominant, args.precision)
    if roof is not None:
        roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    kblock_timed = roofline_entry(agg, 1, args.precision)
    others = {CATS[b][0]: roofline_entry(warm_stats, b, args.precision) for b in CATS}

    out = {
        "metric": METRIC,
        "value": round(per_run, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * per_run, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "J_max": p.J_max, "C": p.C, "gamma": p.gamma,
                   "kappa": 59, "precision": args.precision, "seeds": list(range(args.steps))},
        "roofline": roof,
        "kblock_tflops": kblock_timed["achieved"] if kblock_timed else None,
        "kblock": kblock_timed,
        "kernels_warmup": others,
        "train_stats_seed0": {k: stats[0][k] for k in ("stages", "newton_iters", "factorizations", "score_passes",
                                                        "ls_passes", "n_sv", "grad_norm", "seconds_select",
                                                        "seconds_newton")},
    }

    # the same runs with split-BF16 distances (SPSVM_MIXED), for the "mixed vs FP32" part of the metric
    mixed_models = []
    if not args.no_mixed and args.precision == "f32":
        mcommon = dict(common, precision="mixed")
        lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=1000, **mcommon)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for k in range(args.steps):
            mixed_models.append(lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=k, **mcommon))
        torch.cuda.synchronize()
        per_mixed = (time.perf_counter() - t3) / args.steps
        out["mixed"] = {"value": round(per_mixed, 6), "unit": "s", "ratio_fp32_over_mixed": round(per_run / per_mixed, 4)}

    J, beta, F = models[0].get()
    if not args.no_parity or not args.no_cpu_baseline:
        from oracle import spsvm as osp
        import oracle

    if not args.no_parity:
        tq = time.perf_counter()
        b_or, F_or, info = osp.solve_fixed_J(p.X, p.y, p.C, p.gamma, J)
        newton_oracle_s = time.perf_counter() - tq
        Fo = osp.objective_at(p.X, p.y, p.C, p.gamma, J, beta)
        rows = np.random.default_rng(0).choice(n, 2000, replace=False)
        dg = models[0].predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
        do = oracle.predict(p.X[J], b_or, p.gamma, p.X[rows])
        derr = float(np.max(np.abs(dg - do) / np.maximum(1.0, np.abs(do))))
        rel = (Fo - F_or) / F_or
        out["parity"] = {"objective_rel": rel, "objective_ok": bool(rel <= 1e-6), "decision_max_rel": derr,
                         "decision_ok": bool(derr <= 1e-4), "F_gpu": Fo, "F_oracle": F_or, "m": int(len(J))}
        if mixed_models:
            Jm, bm, _ = mixed_models[0].get()
            _, F_orm, _ = osp.solve_fixed_J(p.X, p.y, p.C, p.gamma, Jm) if not np.array_equal(Jm, J) else (None, F_or, None)
            Fm = osp.objective_at(p.X, p.y, p.C, p.gamma, Jm, bm)
            out["mixed"]["objective_rel"] = (Fm - F_orm) / F_orm
            out["mixed"]["objective_ok"] = bool((Fm - F_orm) / F_orm <= 1e-6)
    else:
        newton_oracle_s = None

    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        try:
            from threadpoolctl import threadpool_limits
            ctx = threadpool_limits(cores)
        except Exception:  # noqa: BLE001
            ctx = None
        os.environ.setdefault("OMP_NUM_THREADS", str(cores))
        S = args.cpu_sample_steps
        tq = time.perf_counter()
        osp.train(p.X, p.y, p.C, p.gamma, p.J_max, seed=0, max_steps=S)
        sample_s = time.perf_counter() - tq
        steps_full = int(stats[0]["additions"])
        est = sample_s / S * steps_full + (newton_oracle_s or 0.0)
        out["cpu_baseline"] = {
            "value": round(est, 3),
            "unit": "s",
            "cores": cores,
            "kind": "oracle",
            "sample": (f"FP64 oracle greedy training, first {S} addition steps on the full {n} x {d} data "
                       f"({sample_s:.2f} s, scaled to {steps_full} steps) plus one oracle Newton re-solve at "
                       f"the GPU's final basis ({newton_oracle_s:.2f} s); a lower bound on the full oracle run"
                       if newton_oracle_s is not None else f"first {S} addition steps scaled to {steps_full}"),
        }
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    print(json.dumps(out))


if __name__ == "__main__":
    main()

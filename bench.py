#!/usr/bin/env python3
"""Benchmark of the NeuRLP-PDE solve on one MI355X.

Workload: 64 instances of the 2D-space + time variable-coefficient
diffusion-advection-reaction PDE on a 32(t) x 64(x) x 64(y) grid, periodic in
space, Fourier-mode coefficient fields, Gaussian-random-field initial data,
FP32, solved to a normal-equation relative residual of 1e-6 for every
instance.  A step is one full pass of the hot path over the batch: build
(coefficient coarsening, operator diagonals, Chebyshev intervals, dense
coarsest inverses) plus the refined multigrid-PCG solve, with the inputs
already resident in HBM.

Prints one JSON line: solves/s, milliseconds per step, the roofline of the
dominant kernel (the finest-grid operator pass in its Chebyshev-smoothing
form: algorithmic bytes per launch / mean launch duration, timed with HIP
events over back-to-back launches on the library's stream right after the
timed steps, against 8 TB/s), the HBM traffic of that kernel from committed
rocprofv3 counter runs (null if the kernel source has changed since), and
the FP64 oracle timed on the host CPU on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDE solves/sec to 1e-6 rel. residual, learned vs plain MG; stencil HBM GB/s"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2502_18377_amd", "csrc")
KERNEL_SRC = {"apply3": "mpde_fused.hip", "gamma": "mpde_kernels.hip", "gather": "mpde_kernels.hip"}
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_rd2d_64x32x64x64.json")


def kernel_source_sha(kernel):
    with open(os.path.join(CSRC, KERNEL_SRC[kernel]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel, mode):
    """Counter-measured HBM bytes per launch of `kernel` in operator `mode`
    on the finest grid, from a committed summary of rocprofv3
    FETCH_SIZE/WRITE_SIZE runs; null when absent or when the kernel source
    differs from the one the counters were taken on."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("source_sha") != kernel_source_sha(kernel):
        return None
    m = k.get("modes", {}).get(str(mode))
    return None if m is None else m.get("bytes_per_launch")


def cpu_baseline(seconds=12.0, max_instances=8):
    """FP64 oracle (saddle-point sparse LU, single-threaded SuperLU) on
    instances of the same generator at 8x8x8 points: a direct factorisation
    of a full 32x64x64 instance does not fit in host memory."""
    import numpy as np
    import workloads as W
    from oracle.system import OracleProblem, assemble
    from oracle.solve import solve_kkt
    n, t0 = 0, time.perf_counter()
    unknowns = 0
    while n < max_instances and (time.perf_counter() - t0) < seconds:
        inst = W.reaction_diffusion_2d(1000 + n, shape=(8, 8, 8))
        op = OracleProblem(**{k: inst[k] for k in ("shape", "step", "bc", "mset", "coeff", "rhs", "bc_values")})
        A, d, _ = assemble(op)
        solve_kkt(A, d)
        unknowns += A.shape[1]
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} instances of the same generator at 8x8x8 points ({unknowns // n} unknowns each), "
                      f"FP64 saddle-point SuperLU, {dt:.1f} s; host has {os.cpu_count()} cores",
            "unknowns_per_s": unknowns / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="also time every finest-grid operator launch of the solves with events (diagnostic; slows them)")
    ap.add_argument("--no-single", action="store_true", help="ragged: skip the one-problem-per-instance baseline")
    ap.add_argument("--workload", choices=["rd2d", "ragged"], default="rd2d",
                    help="rd2d: 64 x 32x64x64 reaction-diffusion (default); ragged: 256 ragged 1D+time instances, "
                         "batched vs one problem per instance")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); instances of a batch are "
              "independent, so a multi-GPU run would shard the batch with no communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2502_18377_amd.api import Problem, pack

    dev = torch.device("cuda:0")
    if args.workload == "ragged":
        return bench_ragged(args, np, torch, W, Problem, pack, dev)
    B = args.batch
    insts = [W.reaction_diffusion_2d(i) for i in range(B)]
    pk = pack(insts, dtype=torch.float32, device=dev)
    del insts
    torch.cuda.synchronize()
    prof = 1 if args.profile else 0

    def step():
        prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"],
                       profile=prof)
        z, info = prob.solve()
        ks = prob.kernel_stats() if prof else {}
        prob.close()
        return z, info, ks

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kstat, iters, relres, outer, solve_s = {}, [], [], [], 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z, info, ks = step()
        iters.append(info["iters"].mean())
        outer.append(info["outer"].mean())
        relres.append(float(info["relres"].max()))
        solve_s += info["seconds"]
        if info["code"] != 0:
            raise SystemExit(f"solve did not converge: {info}")
        for k, v in ks.items():
            if v["launches"] == 0:
                continue
            a = kstat.setdefault(k, dict(launches=0, ms=0.0, bytes=0.0))
            for f in a:
                a[f] += v[f]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1000 / args.steps
    value = B * args.steps / (t1 - t0)

    # Roofline of the dominant kernel: the finest-grid operator pass, timed
    # over back-to-back launches with HIP events on the library's stream.
    prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])
    modes = {}
    for mode, label in ((2, "chebyshev"), (1, "residual"), (3, "apply_dot")):
        us, by = prob.time_operator(mode, reps=30)
        modes[label] = {"us_per_launch": round(us, 2), "bytes_per_launch": by,
                        "GB/s": round(by / (us * 1e-6) / 1e9, 1)}
    prob.close()
    ch = modes["chebyshev"]
    achieved = ch["bytes_per_launch"] / (ch["us_per_launch"] * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": "k_apply3 (finest grid 64x32x64x64, Chebyshev step, FP32)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for("apply3", 2),
            "bytes_per_launch": ch["bytes_per_launch"], "us_per_launch": ch["us_per_launch"],
            "timing": "HIP events around 30 back-to-back launches on the library stream", "modes": modes}
    if kstat:
        roof["solve_launches"] = {n: {"launches_per_step": v["launches"] / args.steps,
                                      "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1),
                                      "ms_per_step": round(v["ms"] / args.steps, 3)} for n, v in kstat.items()}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 instances of 2D-space+time diffusion-advection-reaction, 32(t)x64x64 "
                                  "periodic, FP32, build+solve to 1e-6 normal-equation relative residual",
                      "batch": B, "grid": [32, 64, 64], "solver": "plain multigrid-PCG"},
           "solve_only_ms_per_step": round(solve_s * 1000 / args.steps, 3),
           "mean_pcg_iters": round(float(np.mean(iters)), 2), "mean_outer_steps": round(float(np.mean(outer)), 2),
           "max_relres": max(relres), "roofline": roof}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def bench_ragged(args, np, torch, W, Problem, pack, dev):
    """Batching form: 256 instances of the 1D+time workload with each axis
    drawn from {16,24,32,48,64}, FP32, solved in one batch (one launch per
    stage for all instances) vs one problem per instance."""
    from paper_2502_18377_amd import autotune
    B = 256 if args.batch == 64 else args.batch
    shapes = W.ragged_shapes(B)
    insts = [W.reaction_diffusion_1d_ragged(i, s) for i, s in enumerate(shapes)]
    pk = pack(insts, dtype=torch.float32, device=dev)
    singles = [pack([inst], dtype=torch.float32, device=dev) for inst in insts]
    torch.cuda.synchronize()
    # autotuned settings for this shape class (searched once, outside the timed region)
    tp = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])
    tuned = autotune.run(tp)
    tp.close()
    topts = {k: tuned[k] for k in ("nu", "check_every", "inner_tol")}

    def batched():
        prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"],
                       **topts)
        z, info = prob.solve()
        prob.close()
        if info["code"] != 0:
            raise SystemExit(f"batched solve did not converge: {info}")
        return info

    def one_by_one():
        its = []
        for q in singles:
            prob = Problem(q["coeff"], q["rhs"], q["bc_values"], q["shapes"], q["steps"], q["bc"], q["mset"])
            z, info = prob.solve()
            prob.close()
            its.append(info["iters"][0])
        return its

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = batched()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.no_single:
        t2, its1, t3 = 0.0, [0], 1.0
    else:
        one_by_one()                    # warm
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        its1 = one_by_one()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    value = B * args.steps / (t1 - t0)
    single = B / (t3 - t2) if not args.no_single else None
    out = {"metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round((t1 - t0) * 1000 / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 ragged 1D+time reaction-advection-diffusion instances, each axis in "
                                  "{16,24,32,48,64}, FP32, build+solve to 1e-6, one batch",
                      "batch": B, "solver": "plain multigrid-PCG, captured HIP graphs", "autotuned": tuned},
           "one_problem_per_instance": None if single is None else
           {"value": round(single, 3), "unit": "solves/s", "mean_pcg_iters": round(float(np.mean(its1)), 2)},
           "batched_over_single": None if single is None else round(value / single, 2),
           "mean_pcg_iters": round(float(info["iters"].mean()), 2), "max_relres": float(info["relres"].max())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
    ap.add_argument("--workload", choices=["rd2d", "ragged", "learned", "adjoint"], default="rd2d",
                    help="rd2d: 64 x 32x64x64 reaction-diffusion (default); ragged: 256 ragged 1D+time instances, "
                         "batched vs one problem per instance; learned: network trained on 32x64x64 systems, "
                         "evaluated on held-out 64x128x128 instances against plain multigrid; adjoint: 32 x "
                         "32x128x128 advection-diffusion, solve + adjoint gradient per step")
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
    if args.workload == "learned":
        return bench_learned(args, np, torch, W, Problem, pack, dev)
    if args.workload == "adjoint":
        return bench_adjoint(args, np, torch, W, Problem, pack, dev)
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
    for mode, label in ((2, "chebyshev"), (1, "residual"), (3, "apply_dot"), (4, "residual_fp64")):
        us, by = prob.time_operator(mode, reps=30)
        modes[label] = {"us_per_launch": round(us, 2), "bytes_per_launch": by,
                        "GB/s": round(by / (us * 1e-6) / 1e9, 1),
                        "traffic": traffic_for("apply3", mode)}
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


def bench_learned(args, np, torch, W, Problem, pack, dev):
    """Learned-preconditioner form: a network trained on the GPU on systems
    of the 32x64x64 reaction-diffusion generator (the correction at grid
    level 1), evaluated on held-out instances at 64x128x128 (seeds from
    10^6) solved to 1e-6 with flexible CG + learned correction against
    plain multigrid-PCG on the same instances."""
    from paper_2502_18377_amd.learned import Net, train
    B = 128 if args.batch == 64 else args.batch
    n_train, per_batch, steps = 8, 8, 300
    probs = []
    for k in range(n_train):
        pk = pack([W.reaction_diffusion_2d(100 + per_batch * k + i) for i in range(per_batch)],
                  dtype=torch.float32, device=dev)
        probs.append(Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"],
                             pk["mset"]))
    net = Net(2 + 6, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, probs, 1, steps, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for q in probs:
        q.close()
    loss = np.array([h[1] for h in hist])
    plain = np.array([h[2] for h in hist])
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        insts = list(ex.map(W.reaction_diffusion_2d_large, range(10**6, 10**6 + B)))
    pk = pack(insts, dtype=torch.float32, device=dev)
    del insts
    prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])

    def timed(reps):
        z, info = prob.solve()               # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            z, info = prob.solve()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, info

    reps = max(1, args.steps // 2)
    t_plain, i_plain = timed(reps)
    net.attach(prob, 1)
    t_learn, i_learn = timed(reps)
    Net.detach(prob)
    prob.close()
    for inf in (i_plain, i_learn):
        if inf["code"] != 0:
            raise SystemExit(f"solve did not converge: {inf}")
    out = {"metric": METRIC, "value": round(B / t_learn, 3), "unit": "solves/s", "n_gpus": 1, "steps": reps,
           "warmup": 1, "ms_per_step": round(t_learn * 1e3, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{B} held-out instances of 2D-space+time reaction-diffusion, 64(t)x128x128 "
                                  "periodic, FP32, solve to 1e-6; network trained on 32x64x64 systems",
                      "batch": B, "grid": [64, 128, 128], "solver": "flexible CG + learned coarse correction"},
           "plain_multigrid": {"value": round(B / t_plain, 3), "unit": "solves/s",
                               "ms_per_solve_batch": round(t_plain * 1e3, 3),
                               "mean_pcg_iters": round(float(i_plain["iters"].mean()), 2)},
           "learned": {"mean_iters": round(float(i_learn["iters"].mean()), 2),
                       "max_relres": float(i_learn["relres"].max())},
           "learned_over_plain": round(t_plain / t_learn, 3),
           "training": {"systems": n_train * per_batch, "steps": steps, "seconds": round(t_train, 2),
                        "loss_first10": float(loss[:10].mean()), "loss_last10": float(loss[-10:].mean()),
                        "plain_vcycle_loss_last10": float(plain[-10:].mean())}}
    net.close()
    print(json.dumps(out), flush=True)


def bench_adjoint(args, np, torch, W, Problem, pack, dev):
    """Differentiation form: 32 instances of the 2D+time advection-diffusion
    workload at 32x128x128, FP32.  A step is build + forward solve + the
    adjoint solve and gradients of the loss mean((u - target)^2) with
    respect to the coefficient fields, the source and the boundary data."""
    B = 32 if args.batch == 64 else args.batch
    shape = (32, 128, 128)
    pairs = [W.advection_diffusion_2d(i, shape=shape) for i in range(B)]
    pk = pack([p[0] for p in pairs], dtype=torch.float32, device=dev)
    N = int(np.prod(shape))
    V = 7
    target = torch.tensor(np.concatenate([p[1].ravel() for p in pairs]), dtype=torch.float32, device=dev)
    del pairs

    def step():
        prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])
        z, info = prob.solve()
        zz = z.view(B, V, N)
        u = zz[:, 0, :].reshape(-1)
        g = torch.zeros_like(zz)
        g[:, 0, :] = (2.0 / (B * N)) * (u - target).view(B, N)
        gc, gf, gw, ainfo = prob.adjoint(g.reshape(-1))
        prob.close()
        return info, ainfo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, ainfo = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for inf in (info, ainfo):
        if inf["code"] != 0:
            raise SystemExit(f"solve did not converge: {inf}")
    out = {"metric": METRIC, "value": round(B / dt, 3), "unit": "gradient solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{B} instances of 2D-space+time advection-diffusion, 32(t)x128x128 periodic, "
                                  "FP32: build + solve + adjoint solve + gradients w.r.t. c, f, omega",
                      "batch": B, "grid": list(shape)},
           "forward_pcg_iters": round(float(info["iters"].mean()), 2),
           "adjoint_pcg_iters": round(float(ainfo["iters"].mean()), 2),
           "adjoint_max_relres": float(ainfo["relres"].max())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""HBM traffic of the finest-grid operator kernel from rocprofv3 counters.

Two steps, each under rocprofv3 with one counter (FETCH_SIZE, then
WRITE_SIZE; both count KiB per dispatch):

    rocprofv3 --pmc FETCH_SIZE -d D1 -o run --output-format csv -- \
        python -m paper_2502_18377_amd.traffic run
    rocprofv3 --pmc WRITE_SIZE -d D2 -o run --output-format csv -- \
        python -m paper_2502_18377_amd.traffic run
    python -m paper_2502_18377_amd.traffic summarize D1 D2 OUT.json

`run` performs a plain device-to-device copy of a known size (the
calibration: counter KiB per copied byte), then what bench.py does: one
build + solve of the benchmark workload (64 instances of 32x64x64, FP32)
and the timing loops of the finest-grid operator (30 back-to-back passes
per mode after one warm-up pass; mode 4 is the FP64 residual pass).  `summarize` averages the counters over
the timing-loop dispatches of each mode (the launches the benchmark's
roofline times), scales them by the copy's bytes-per-counter ratio and
records the hash of the kernel source, so that bench.py reports the
traffic only while the kernel is unchanged.

    python -m paper_2502_18377_amd.traffic trace KERNEL_TRACE.csv > summary.txt

summarises a `rocprofv3 --kernel-trace` run: per-kernel calls and average
duration, and the same for the operator kernel's finest-grid dispatches
(the largest grid among its launches), the set bench.py's roofline times.
"""
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20
KERNELS = {"apply3": ("k_apply3", "mpde_fused.hip")}
LOOP_MODES = (2, 1, 3, 4)   # the modes bench.py times, in its order (4: the FP64 residual)
LOOP_REPS = 30


def source_sha(fname):
    with open(os.path.join(HERE, "csrc", fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def run():
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as W
    from paper_2502_18377_amd.api import Problem, pack
    dev = torch.device("cuda:0")
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copy done", flush=True)
    pk = pack([W.reaction_diffusion_2d(i) for i in range(64)], dtype=torch.float32, device=dev)
    prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])
    z, info = prob.solve()
    torch.cuda.synchronize()
    print("solve done", info["code"], float(info["iters"].mean()), flush=True)
    prob.close()
    prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"])
    for mode in LOOP_MODES:
        print("mode", mode, prob.time_operator(mode, reps=LOOP_REPS), flush=True)
    prob.close()


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _mode(kernel_name):
    """Key of a k_apply3 instantiation: its operator mode (fourth template
    argument) as in Problem.time_operator, i.e. "4" for the FP64 residual
    pass (arithmetic type double); "fp64_<mode>" for other FP64 passes;
    None for other kernels."""
    if "k_apply3<" not in kernel_name:
        return None
    args = [a.strip() for a in kernel_name.split("k_apply3<")[1].split(">")[0].split(",")]
    if args[0] == "double":   # FP64: the outer residual is mode 4; other FP64 passes (probing) apart
        return "4" if args[3] == "1" else "fp64_" + args[3]
    return args[3]


def _per_dispatch(rows, match):
    """{dispatch id: (counter value summed over its rows, grid size, mode)} for kernels containing `match`."""
    out = {}
    for r in rows:
        if match not in r["Kernel_Name"]:
            continue
        k = r["Dispatch_Id"]
        v = float(r["Counter_Value"])
        g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
        prev = out.get(k, (0.0, g, _mode(r["Kernel_Name"])))
        out[k] = (prev[0] + v, g, prev[2])
    return out


def summarize(d_fetch, d_write, out_path):
    res = {"command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python -m paper_2502_18377_amd.traffic run",
           "copy_bytes": COPY_BYTES, "kernels": {}}
    scale = {}
    for name, d in (("FETCH_SIZE", d_fetch), ("WRITE_SIZE", d_write)):
        rows = _rows(d)
        cp = _per_dispatch(rows, "copyBuffer")
        big = [v for v, g, _m in cp.values() if v > 0.5 * COPY_BYTES / 1024]
        if not big:
            raise SystemExit(f"{name}: no calibration copy dispatch found")
        kib = sum(big) / len(big)
        scale[name] = COPY_BYTES / (kib * 1024.0)
        res[f"copy_{name}_KiB"] = kib
        res[f"{name}_bytes_per_KiB"] = scale[name]
        for key, (kname, src) in KERNELS.items():
            disp = _per_dispatch(rows, kname)
            if not disp:
                continue
            ent = res["kernels"].setdefault(key, {"source_sha": source_sha(src), "modes": {}})
            for mode in sorted({m for _, _, m in disp.values()}):
                # the timing loop: the last LOOP_REPS finest-grid dispatches of the mode
                gmax = max(g for _, g, m in disp.values() if m == mode)
                seq = [v for d, (v, g, m) in sorted(disp.items(), key=lambda kv: int(kv[0]))
                       if g == gmax and m == mode]
                fin = seq[-LOOP_REPS:]
                if not fin:
                    continue
                e = ent["modes"].setdefault(mode, {"loop_dispatches": len(fin)})
                e[f"{name}_KiB_per_dispatch"] = sum(fin) / len(fin)
                e[f"{name}_bytes_per_dispatch"] = sum(fin) / len(fin) * 1024.0 * scale[name]
    for ent in res["kernels"].values():
        for e in ent["modes"].values():
            if "FETCH_SIZE_bytes_per_dispatch" in e and "WRITE_SIZE_bytes_per_dispatch" in e:
                e["bytes_per_launch"] = e["FETCH_SIZE_bytes_per_dispatch"] + e["WRITE_SIZE_bytes_per_dispatch"]
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def trace(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))

    def name_of(r):
        return r["Kernel_Name"].split("(")[0].replace("void ", "")

    def grid(r):
        return int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)

    def dur(r):
        return (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3

    agg = {}
    gmax = {}   # finest grid of each k_apply3 instantiation: its largest launch
    for r in rows:
        name = name_of(r)
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += dur(r)
        if "k_apply3" in name:
            gmax[name] = max(gmax.get(name, 0), grid(r))
    fin, loops = {}, {}
    for r in rows:
        name = name_of(r)
        if "k_apply3" in name and grid(r) == gmax[name]:
            b = fin.setdefault(name, [0, 0.0])
            b[0] += 1
            b[1] += dur(r)
            loops.setdefault(name, []).append((int(r["Dispatch_Id"]), dur(r)))
    tot = sum(v[1] for v in agg.values())
    print(f"# total kernel time {tot / 1e3:.2f} ms")
    print("kernel | calls | total_ms | avg_us | pct")
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{k} | {n} | {t / 1e3:.2f} | {t / n:.2f} | {100 * t / tot:.2f}")
    print(f"# timing loops of bench.py (last {LOOP_REPS} finest-grid dispatches of each k_apply3 instantiation)")
    for k, v in sorted(loops.items()):
        d = [t for _, t in sorted(v)][-LOOP_REPS:]
        print(f"{k} | {len(d)} | {sum(d) / 1e3:.2f} | {sum(d) / len(d):.2f}")
    print("# finest-grid dispatches of each k_apply3 instantiation, whole run")
    for k, (n, t) in sorted(fin.items()):
        print(f"{k} | grid {gmax[k]} | {n} | {t / 1e3:.2f} | {t / n:.2f}")
    # multigrid level of each operator launch, from the dispatch order:
    # k_restrict moves one level down, k_prolong_add one level up (launches
    # outside a V-cycle count as level 0)
    print("# k_apply3 by multigrid level (from restrict/prolong order), whole run")
    lev, per = 0, {}
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        name = name_of(r)
        if "k_restrict" in name:
            lev += 1
        elif "k_prolong_add" in name:
            lev = max(0, lev - 1)
        elif "k_apply3" in name:
            c = per.setdefault((name, lev), [0, 0.0])
            c[0] += 1
            c[1] += dur(r)
    for (k, l), (n, t) in sorted(per.items()):
        print(f"{k} | level {l} | {n} | {t / 1e3:.2f} | {t / n:.2f}")


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run()
    elif len(sys.argv) == 5 and sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) == 3 and sys.argv[1] == "trace":
        trace(sys.argv[2])
    else:
        raise SystemExit(__doc__)

"""HBM traffic of the finest-grid operator kernel from rocprofv3 counters.

Two steps, each under rocprofv3 with one counter (FETCH_SIZE, then
WRITE_SIZE; both count KiB per dispatch):

    rocprofv3 --pmc FETCH_SIZE -d D1 -o run --output-format csv -- \
        python -m paper_2502_18377_amd.traffic run
    rocprofv3 --pmc WRITE_SIZE -d D2 -o run --output-format csv -- \
        python -m paper_2502_18377_amd.traffic run
    python -m paper_2502_18377_amd.traffic summarize D1 D2 OUT.json

`run` performs a plain device-to-device copy of a known size (the
calibration: counter KiB per copied byte), then one build + solve of the
benchmark workload (64 instances of 32x64x64, FP32).  `summarize` averages
the counters over the dispatches of the operator kernel on the finest grid
(the launches the benchmark's roofline times), scales them by the copy's
bytes-per-counter ratio and records the hash of the kernel source, so that
bench.py reports the traffic only while the kernel is unchanged.
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


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, match):
    """{dispatch id: (counter value summed over its rows, grid size)} for kernels containing `match`."""
    out = {}
    for r in rows:
        if match not in r["Kernel_Name"]:
            continue
        k = r["Dispatch_Id"]
        v = float(r["Counter_Value"])
        g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
        prev = out.get(k, (0.0, g))
        out[k] = (prev[0] + v, g)
    return out


def summarize(d_fetch, d_write, out_path):
    res = {"command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python -m paper_2502_18377_amd.traffic run",
           "copy_bytes": COPY_BYTES, "kernels": {}}
    scale = {}
    for name, d in (("FETCH_SIZE", d_fetch), ("WRITE_SIZE", d_write)):
        rows = _rows(d)
        cp = _per_dispatch(rows, "copyBuffer")
        big = [v for v, g in cp.values() if v > 0.5 * COPY_BYTES / 1024]
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
            gmax = max(g for _, g in disp.values())
            fin = [v for v, g in disp.values() if g == gmax]      # finest grid: the largest launches
            ent = res["kernels"].setdefault(key, {"source_sha": source_sha(src), "finest_dispatches": len(fin)})
            ent[f"{name}_KiB_per_dispatch"] = sum(fin) / len(fin)
            ent[f"{name}_bytes_per_dispatch"] = sum(fin) / len(fin) * 1024.0 * scale[name]
    for ent in res["kernels"].values():
        if "FETCH_SIZE_bytes_per_dispatch" in ent and "WRITE_SIZE_bytes_per_dispatch" in ent:
            ent["bytes_per_launch"] = ent["FETCH_SIZE_bytes_per_dispatch"] + ent["WRITE_SIZE_bytes_per_dispatch"]
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run()
    elif len(sys.argv) == 5 and sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)

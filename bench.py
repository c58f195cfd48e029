#!/usr/bin/env python3
"""Benchmark of the Hierarchy-Scan hot path on one MI355X.

Default workload: the deep-skeleton forward scan, 4096 characters x 1024
joints (a 64-joint humanoid plus four 240-joint chains, depth 246), fp32.
A step is one hs_scan_forward over the whole batch with every input already
resident in HBM.  Two input/output sets alternate between steps so that the
256 MB last-level cache never holds the next step's data.

Prints one JSON line with the throughput in joint transforms per second, the
roofline of the scan kernel (algorithmic bytes / measured kernel time against
8 TB/s HBM), and the FP64 CPU oracle timed on the host as a baseline.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "joint transforms/sec fwd + fwd/bwd on 1 GPU; % HBM roofline; err vs FP64"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2505_06703_amd", "csrc", f)
                  for f in ("hs_kernels.hip", "hs_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch from committed PMC counters, if they were taken
    on the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="deep_forward",
                    choices=["deep_forward", "plain_scan", "heterogeneous", "fused_sample"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape at plan time")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE run, WRITE_SIZE run) "
                         "into profiles/traffic.json for --workload and exit")
    return ap.parse_args()


# algorithmic HBM bytes per joint that one step must move (read + write)
BYTES_PER_JOINT = {
    # quat 16 + trans 12 + scale 12 + parent 4 read, global 64 written
    "deep_forward": 108,
    "heterogeneous": 108,
    # + inverse bind 64 read, skin 64 written
    "plain_scan": 236,
    # parent 4 + inverse bind 64 read, skin 64 written (+ clip library once)
    "fused_sample": 132,
}


COPY_BYTES = 256 << 20


def summarize_pmc(workload, fetch_csv, write_csv):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the scan kernel,
    scaled by what the same counters read for the plain copy of COPY_BYTES."""
    import csv

    def per_kernel(path, counter):
        vals = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name = row["Kernel_Name"]
                key = "scan" if "fwd_tile_kernel" in name else ("copy" if "copy" in name.lower() else None)
                if key:
                    vals.setdefault(key, []).append(float(row["Counter_Value"]))
        # the calibration copy is the largest copy of the run
        return {"scan": sum(vals["scan"]) / len(vals["scan"]), "copy": max(vals["copy"])}

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (fetch["copy"] * 1024.0)
    w_scale = COPY_BYTES / (write["copy"] * 1024.0)
    rec = {"kernel": "fwd_tile_kernel", "source_sha": kernel_source_sha(),
           "fetch_bytes_per_launch": fetch["scan"] * 1024.0 * f_scale,
           "write_bytes_per_launch": write["scan"] * 1024.0 * w_scale,
           "copy_fetch_scale": f_scale, "copy_write_scale": w_scale}
    rec["hbm_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    try:
        with open(TRAFFIC_FILE) as f:
            allrec = json.load(f)
    except (OSError, ValueError):
        allrec = {}
    allrec[workload] = rec
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
    print(json.dumps({workload: rec}))


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.workload, *args.summarize_pmc)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; characters are independent, "
                                   "so a multi-GPU run would split them with no exchange (see DESIGN.md)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2505_06703_amd import hs
    from paper_2505_06703_amd import workloads as wl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    b = wl.make(args.workload)
    N, C = b.num_joints, b.num_characters
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    plan = hs.Plan(b.offsets, b.parents, autotune=args.autotune)
    info = plan.info

    clips = None
    inv = None
    if args.workload in ("plain_scan", "fused_sample"):
        # inverse binds from the rest pose: scan it on the GPU, invert on the host
        Grest, _ = hs.hs_scan_forward(plan, up(b.rest_quat), up(b.rest_trans), up(b.rest_scale))
        inv = up(np.linalg.inv(Grest.cpu().numpy().astype(np.float64)).astype(np.float32))
        del Grest
    if args.workload == "fused_sample":
        clips = hs.ClipLibrary(up(b.extra["key_quat"]), up(b.extra["key_trans"]), b.extra["fps"])
        cp = dict(clip_a=up(b.extra["clip_a"]), clip_b=up(b.extra["clip_b"]), time=up(b.extra["time"]),
                  weight=up(b.extra["weight"]))

    nsets = 2
    sets = []
    for k in range(nsets):
        s = {}
        if clips is None:
            s["q"], s["t"], s["s"] = up(b.quat), up(b.trans), up(b.scale)
        s["inv"] = None if inv is None else (inv if k == 0 else inv.clone())
        if args.workload in ("deep_forward", "heterogeneous"):
            s["G"] = torch.empty((N, 4, 4), device=dev)
        else:
            s["S"] = torch.empty((N, 4, 4), device=dev)
        sets.append(s)

    def step(k):
        s = sets[k % nsets]
        if args.workload == "fused_sample":
            hs.hs_scan_forward(plan, clips=clips, **cp, want_global=False, inv_bind=s["inv"], skin_out=s["S"])
        elif args.workload == "plain_scan":
            hs.hs_scan_forward(plan, s["q"], s["t"], s["s"], want_global=False, inv_bind=s["inv"],
                               skin_out=s["S"])
        else:
            hs.hs_scan_forward(plan, s["q"], s["t"], s["s"], global_out=s["G"])

    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(e) for a, e in ev]))

    value = N * args.steps / elapsed
    bytes_per_launch = N * BYTES_PER_JOINT[args.workload]
    if args.workload == "fused_sample":
        bytes_per_launch += b.extra["key_quat"].nbytes + b.extra["key_trans"].nbytes + 16 * C
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "joint transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "characters": C, "joints": N,
                   "max_depth": info["max_depth"], "tile_joints": info["tile_joints"],
                   "waves_per_tile": info["waves_per_tile"], "tiles": info["num_tiles"],
                   "multipass_joints": info["multipass_joints"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fwd_tile_kernel", "kernel_ms": kernel_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["err_vs_fp64"] = cpu_baseline(b, args.workload, plan, sets, step, nsets)
    print(json.dumps(out))


def cpu_baseline(b, workload, plan, sets, step, nsets):
    """Time the FP64 oracle on the host (all cores it may use) on repeated
    passes over the full batch, and compare the last GPU result with it."""
    import torch
    import oracle

    cores = len(os.sched_getaffinity(0))
    N = b.num_joints
    if workload == "fused_sample":
        def run():
            q, t = oracle.pose_sample(b.offsets, b.extra["key_quat"], b.extra["key_trans"], b.extra["clip_a"],
                                      b.extra["clip_b"], b.extra["time"], b.extra["weight"], b.extra["fps"])
            return oracle.forward(b.offsets, b.parents, q, t, None), t
    else:
        def run():
            return oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale), b.trans
    reps, t0 = 0, time.perf_counter()
    while True:
        G, tr = run()
        reps += 1
        wall = time.perf_counter() - t0
        if wall >= 10.0 or reps >= 50:
            break
    base = {"value": N * reps / wall, "unit": "joint transforms/s", "cores": cores, "kind": "oracle",
            "sample": f"full {workload} batch ({b.num_characters} characters, {N} joints) x {reps} passes, "
                      f"fp32->fp64 widening included, {wall:.1f} s wall"}

    # error of one fresh GPU step against the oracle
    step(0)
    torch.cuda.synchronize()
    lam = oracle.path_length(b.offsets, b.parents, G, tr)
    if workload in ("deep_forward", "heterogeneous"):
        Gg = sets[0]["G"].cpu().numpy().astype(np.float64)
        dA = float(np.abs(Gg[:, :3, :3] - G[:, :3, :3]).max())
        db = np.abs(Gg[:, :3, 3] - G[:, :3, 3]).max(axis=1)
        err = {"rotation_abs_max": dA, "translation_rel_max": float((db / np.maximum(lam, 1e-12)).max())}
    else:
        S = oracle.skin(G, sets[0]["inv"].cpu().numpy())
        Sg = sets[0]["S"].cpu().numpy().astype(np.float64)
        err = {"skin_rotation_abs_max": float(np.abs(Sg[:, :3, :3] - S[:, :3, :3]).max()),
               "skin_translation_abs_max": float(np.abs(Sg[:, :3, 3] - S[:, :3, 3]).max())}
    return base, err


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Hierarchy-Scan hot path on one MI355X.

Default run: the batched form and the differentiable form in one JSON line.

* ``value``: the heterogeneous batch, 16384 characters whose joint counts
  are log-uniform in [32, 2048] (random trees, branching probability 0.3,
  1% pure chains; about 8.0 M joints), fp32.  A step is one
  hs_scan_forward over the whole batch with every input already resident
  in HBM.
* ``fwd_bwd``: 1024 characters x 512 joints (humanoid + four 112-joint
  chains, depth 118): forward scan plus the adjoint of an end-effector loss
  (16 effectors per character) per step, in one launch
  (hs_effector_step); beside it the two memory modes of the general adjoint
  (recompute: hs_scan_forward, loss gradient, hs_scan_backward; level
  checkpoints every 8 levels: the forward also stores checkpoint rows and
  the adjoint rebuilds G from them), each with its time, roofline and
  error against FP64.

The steps are issued either as direct library calls (each marshalled once,
before the timed region, with hs.prepare) or as replays of a HIP graph
that holds eight such passes (one light host call per eight steps),
whichever runs faster on the box (both are timed on a few steps after the
warmup; the line reports both).  The steps cycle through as many
input/output sets as it takes to touch at least 1 GiB per cycle, so that
the 256 MB last-level cache never holds the next step's data.

Each measured form carries the roofline of its dominant kernel (algorithmic
bytes / mean kernel duration from HIP events on the launch stream, against
8 TB/s HBM), the FP64 CPU oracle timed on the host as a baseline, and the
error of one GPU step against FP64.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
                    [--no-autotune] [--no-fwd-bwd] [--no-schedules]

The heterogeneous line also carries `schedules`: the same forward through
the work queue as a resident loop (four workgroups per CU, grid < tiles)
and through the size classes (one launch per class), as plain calls.

Other workloads (--workload): deep_forward (4096 x 1024 joints, depth
246), plain_scan, fused_sample and fused_sample_instanced (clip sampling +
scan + skin), differentiable (the fwd_bwd form on its own), long_chains
(64 chains of 65536 joints: the multipass path, whose step is several
kernels, all counted in kernel_ms), mesh_skinning (vertex skinning, two
calls and one pass), sample_gradients (gradients through the sampler);
--depth-sweep runs the paper's depth experiment.
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
COPY_BYTES = 256 << 20
WORKLOADS = ["heterogeneous", "deep_forward", "plain_scan", "fused_sample", "fused_sample_instanced",
             "differentiable", "long_chains", "mesh_skinning", "sample_gradients"]
FUSED = ("fused_sample", "fused_sample_instanced")

# algorithmic HBM bytes per joint that the dominant kernel of a step must
# move (read + write)
BYTES_PER_JOINT = {
    # quat 16 + trans 12 + scale 12 + parent 4 read, global 64 written
    "deep_forward": 108,
    "heterogeneous": 108,
    # multipass path: the same contract, several kernels per step
    "long_chains": 108,
    # + inverse bind 64 read, skin 64 written
    "plain_scan": 236,
    # parent 4 + inverse bind 64 read, skin 64 written (+ clip library once)
    "fused_sample": 132,
    # instanced: parents and inverse binds are the one skeleton's (256 rows,
    # cache-resident), so only the skin is per joint in HBM
    "fused_sample_instanced": 64,
    # forward scan and end-effector adjoint in one launch: read quat,
    # trans, scale, parent 44, write G 64, grad_quat 16 + grad_trans 12
    # (+ 12 B of targets per effector)
    "differentiable": 136,
}
DOMINANT = {"differentiable": "bwd_anchor_kernel",
            "long_chains": "mp_chain_kernel (one-pass multipass for chains)"}
# what a --pmc dispatch's kernel name must contain to be the dominant
# kernel: the differentiable run also times the dense route, whose adjoint
# is the other instance of the same template
PMC_MATCH = {"differentiable": ("bwd_anchor_kernel<", ", 2>")}
# fused workloads: the instance that samples poses in the kernel
SAMPLE_INSTANCE = ", true"
# steps of several kernels: HBM traffic per step is the sum over them
# (the kernels a step launches; those absent from a run count nothing)
STEP_KERNELS = {"long_chains": [("mp_chain_kernel",), ("mp_local_kernel",), ("mp_anchor",), ("mp_out_kernel",)]}
CHUNK = 8  # at least this many forward passes per captured graph replay
CKPT_K = 8  # levels between checkpoints in the differentiable form's checkpoint mode
SWEEP_BYTES = 1 << 30  # data one cycle over the input/output sets touches
MAX_SETS = 64


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
    ap.add_argument("--workload", default="heterogeneous", choices=WORKLOADS)
    ap.add_argument("--no-schedules", action="store_true",
                    help="heterogeneous: skip timing the other launch schedules beside the line "
                         "(profiling runs; --calibrate-copy skips them too)")
    ap.add_argument("--no-fwd-bwd", action="store_true",
                    help="heterogeneous workload: leave out the differentiable form (fwd_bwd; always left out "
                         "with --calibrate-copy)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the plan's default launch shape instead of timing candidates at plan time")
    ap.add_argument("--adjoint", default="auto", choices=("auto", "rounds", "dataflow", "anchors"),
                    help="adjoint kernel for characters of up to 1024 joints (differentiable workload)")
    ap.add_argument("--schedule", choices=("auto", "queue", "classes"),
                    help="forward schedule of the plan (with --tile-joints/--waves: a fixed launch shape, "
                         "no autotuning; for profiling the shape an autotuned run picked)")
    ap.add_argument("--tile-joints", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--depth-sweep", action="store_true",
                    help="the paper's depth experiment: 10000 characters of 300 joints, depth 15..120, "
                         "this library's scan against the paper's Algorithms 1-4; one JSON line per point")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE run, WRITE_SIZE run) "
                         "into profiles/traffic.json for --workload and exit")
    return ap.parse_args()


def fixed_shape(args):
    """Plan options of a fixed launch shape from the command line, or None."""
    if not (args.schedule or args.tile_joints or args.waves):
        return None
    from paper_2505_06703_amd import hs
    sched = {None: hs.HS_SCHED_AUTO, "auto": hs.HS_SCHED_AUTO, "queue": hs.HS_SCHED_QUEUE,
             "classes": hs.HS_SCHED_CLASSES}[args.schedule]
    return {"schedule": sched, "tile_joints": args.tile_joints, "waves_per_tile": args.waves}


def summarize_pmc(workload, fetch_csv, write_csv):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the dominant
    kernel, scaled by what the same counters read for the plain copy of
    COPY_BYTES in the same run."""
    import csv
    kname = DOMINANT.get(workload)
    if kname is None:
        # the forward's kernel: the work-queue launch if the run made one
        with open(fetch_csv) as f:
            queued = any("fwd_queue_kernel" in r.get("Kernel_Name", "") for r in csv.DictReader(f))
        kname = "fwd_queue_kernel" if queued else "fwd_tile_kernel"
    # a step of several kernels (the multipass path) sums their averages
    parts = STEP_KERNELS.get(workload) or [PMC_MATCH.get(workload, (kname,) + ((SAMPLE_INSTANCE,) if workload in FUSED
                                                                             else ()))]

    def per_kernel(path, counter):
        scan, copy = [[] for _ in parts], None
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r.get("Counter_Name") == counter]
        rows.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
        for row in rows:
            name, kib = row["Kernel_Name"], float(row["Counter_Value"])
            hit = [i for i, match in enumerate(parts) if all(m in name for m in match)]
            if hit:
                scan[hit[0]].append(kib)
            elif "copy" in name.lower() and int(row["Dispatch_Id"]) == copy_id:
                copy = (kib, copy_id)
        return {"scan": sum(sum(x) / len(x) for x in scan if x), "copy": copy[0], "copy_dispatch": copy[1]}

    # the calibration copy (--calibrate-copy): the first device copy that
    # writes COPY_BYTES (uploads of the workload's inputs come before it,
    # small setup copies too, the 1 GiB bandwidth probe after it); the two
    # counter runs dispatch the same kernels in the same order
    with open(write_csv) as f:
        cands = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in csv.DictReader(f)
                       if r.get("Counter_Name") == "WRITE_SIZE" and "copy" in r["Kernel_Name"].lower())
    copy_id = next(d for d, kib in cands if abs(kib * 1024.0 - COPY_BYTES) <= 0.01 * COPY_BYTES)
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (fetch["copy"] * 1024.0)
    w_scale = COPY_BYTES / (write["copy"] * 1024.0)
    rec = {"kernel": kname, "source_sha": kernel_source_sha(),
           "fetch_bytes_per_launch": fetch["scan"] * 1024.0 * f_scale,
           "write_bytes_per_launch": write["scan"] * 1024.0 * w_scale,
           "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
           "copy_dispatch": [fetch["copy_dispatch"], write["copy_dispatch"]]}
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


class Workload:
    """Device-resident inputs/outputs of one preset and its step."""

    def __init__(self, name, autotune, adjoint="auto", shape=None):
        import torch
        from paper_2505_06703_amd import hs
        if name == "fused_sample":
            # the autotuner times candidate shapes on stored poses (the plan
            # has no clip parameters), which ranks the fused sampler's
            # launch wrongly: this workload runs the plan's default shape
            autotune = False
        from paper_2505_06703_amd import workloads as wl
        self.torch, self.hs, self.name = torch, hs, name
        dev = torch.device("cuda:0")
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.b = b = wl.make(name)
        N = b.num_joints
        adj = {"auto": hs.HS_ADJ_AUTO, "rounds": hs.HS_ADJ_ROUNDS, "dataflow": hs.HS_ADJ_DATAFLOW,
               "anchors": hs.HS_ADJ_ANCHORS}[adjoint]
        self.inv = None
        self.clips = None
        if name == "fused_sample_instanced":
            x = b.extra
            self.plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"], autotune=autotune)
            # one skeleton: inverse binds of its rest pose (a one-character plan)
            one = hs.Plan(x["skel_offsets"], x["skel_parents"])
            Grest, _ = hs.hs_scan_forward(one, *(up(a) for a in x["skel_rest"]))
            self.inv = up(np.linalg.inv(Grest.cpu().numpy().astype(np.float64)).astype(np.float32))
            del Grest, one
        else:
            self.plan = hs.Plan(b.offsets, b.parents, autotune=autotune and not shape, adjoint=adj, **(shape or {}))
        if name in ("plain_scan", "fused_sample"):
            # inverse binds from the rest pose: scan it on the GPU, invert on the host
            Grest, _ = hs.hs_scan_forward(self.plan, up(b.rest_quat), up(b.rest_trans), up(b.rest_scale))
            self.inv = up(np.linalg.inv(Grest.cpu().numpy().astype(np.float64)).astype(np.float32))
            del Grest
        if name in FUSED:
            x = b.extra
            self.clips = hs.ClipLibrary(up(x["key_quat"]), up(x["key_trans"]), x["fps"])
            self.cp = dict(clip_a=up(x["clip_a"]), clip_b=up(x["clip_b"]), time=up(x["time"]),
                           weight=up(x["weight"]))
        if name == "differentiable":
            # targets: rest positions (GPU scan of the rest pose) + seeded offsets
            Grest, _ = hs.hs_scan_forward(self.plan, up(b.rest_quat), up(b.rest_trans), up(b.rest_scale))
            self.eff = up(b.extra["effectors"].astype(np.int64))
            self.target = Grest[self.eff, :3, 3] + up(b.extra["target_offsets"])
            self.effset = hs.Effectors(self.plan, b.extra["effectors"])
            # the dense route (loss gradient into dLoss/dG, general adjoint),
            # timed beside the step for comparison
            self.gG = torch.zeros((N, 4, 4), device=dev)
            del Grest
        # input/output sets cycled step by step: enough of them that one
        # cycle touches at least SWEEP_BYTES, so the 256 MB last-level cache
        # never holds the next step's data (the 4096-joint plain_scan fits
        # the cache whatever the count; it is reported as latency-bound)
        def make_set(k):
            st = {}
            if self.clips is None:
                st["q"], st["t"], st["s"] = up(b.quat), up(b.trans), up(b.scale)
            st["inv"] = None if self.inv is None else (self.inv if k == 0 else self.inv.clone())
            if name in ("deep_forward", "heterogeneous", "differentiable", "long_chains"):
                st["G"] = torch.empty((N, 4, 4), device=dev)
            else:
                st["S"] = torch.empty((N, 4, 4), device=dev)
            if name == "differentiable":
                st["gq"] = torch.empty((N, 4), device=dev)
                st["gt"] = torch.empty((N, 3), device=dev)
                # level checkpoints of the checkpoint memory mode
                st["ck"] = torch.empty((N, 12), device=dev)
            return st

        first = make_set(0)
        set_bytes = sum(v.numel() * v.element_size() for v in first.values() if v is not None)
        if self.clips is not None:
            set_bytes += (self.clips.key_quat.numel() + self.clips.key_trans.numel()) * 4
        n_sets = int(min(MAX_SETS, max(2, -(-SWEEP_BYTES // max(1, set_bytes)))))
        self.sets = [first] + [make_set(k) for k in range(1, n_sets)]
        self.set_bytes = set_bytes
        # forward-only steps replay captured HIP graphs: CHUNK passes that
        # cycle through the input sets in one graph (one light host call per
        # CHUNK steps, so launches run back to back), plus one single-pass
        # graph per set for a remainder
        self.graphs = None
        if name != "differentiable":
            calls = []
            for st in self.sets:
                if name in FUSED:
                    calls.append(dict(clips=self.clips, **self.cp, inv_bind=st["inv"], skin_out=st["S"]))
                elif name == "plain_scan":
                    calls.append(dict(quat=st["q"], trans=st["t"], scale=st["s"], inv_bind=st["inv"],
                                      skin_out=st["S"]))
                else:
                    calls.append(dict(quat=st["q"], trans=st["t"], scale=st["s"], global_out=st["G"]))
            self.graphs = [hs.ForwardGraph.sequence(self.plan, [c]) for c in calls]
            S = len(calls)
            self.chunk = S * max(1, -(-CHUNK // S))
            self.chunk_graph = hs.ForwardGraph.sequence(self.plan, [calls[k % S] for k in range(self.chunk)])
        else:
            # the whole differentiable step (one launch: forward scan and
            # end-effector adjoint per tile) captured for CHUNK steps over the
            # sets: nothing in it allocates or synchronises; the two-call and
            # the dense routes likewise
            S = len(self.sets)
            self.chunk = S * max(1, -(-CHUNK // S))
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for k in range(S):
                    self.diff_step(self.sets[k])
                    self.two_call_step(self.sets[k])
                    self.dense_step(self.sets[k])
                    self.ckpt_step(self.sets[k])
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            self.diff_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.diff_graph):
                for k in range(self.chunk):
                    self.diff_step(self.sets[k % S])
            self.dense_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.dense_graph):
                for k in range(self.chunk):
                    self.dense_step(self.sets[k % S])
            self.two_call_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.two_call_graph):
                for k in range(self.chunk):
                    self.two_call_step(self.sets[k % S])
            self.ckpt_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.ckpt_graph):
                for k in range(self.chunk):
                    self.ckpt_step(self.sets[k % S])
        # plain mode: each set's step as one prepared library call (the
        # binding's checks and argument marshalling done once, here)
        self.plain_calls = [self.prepare_plain(st) for st in self.sets]

    def close(self):
        """Release the graphs, the effector set, the plan and the buffers."""
        if self.graphs is not None:
            for g in self.graphs:
                g.close()
            self.chunk_graph.close()
            self.graphs = None
        for attr in ("diff_graph", "dense_graph", "two_call_graph", "ckpt_graph"):
            if hasattr(self, attr):
                delattr(self, attr)
        if hasattr(self, "effset"):
            self.effset.close()
        self.plan.close()
        self.sets = []
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()

    def run(self, steps, mode="graph"):
        """`steps` steps from set 0 on: mode "graph" replays captured graphs
        of `chunk` steps (the remainder issued call by call), mode "plain"
        issues every step as direct library calls."""
        if mode == "plain":
            for k in range(steps):
                self.plain_step(k)
            return
        if self.graphs is None:
            full = steps // self.chunk
            for _ in range(full):
                self.diff_graph.replay()
            for k in range(full * self.chunk, steps):
                self.step(k)
            return
        S = len(self.sets)
        full = steps // self.chunk
        for _ in range(full):
            self.chunk_graph.launch()
        for k in range(full * self.chunk, steps):
            self.graphs[k % S].launch()

    def plain_step(self, k):
        """One step on set k (cycled) as a direct library call."""
        self.plain_calls[k % len(self.sets)]()

    def prepare_plain(self, s):
        """The library call of one step on set s, marshalled once."""
        hs = self.hs
        if self.graphs is None:
            call, _ = hs.prepare(hs.hs_effector_step, self.plan, self.effset, s["q"], s["t"], s["s"], self.target,
                                 global_out=s["G"], want_scale=False, grad_quat=s["gq"], grad_trans=s["gt"])
        elif self.name in FUSED:
            call, _ = hs.prepare(hs.hs_scan_forward, self.plan, clips=self.clips, **self.cp, want_global=False,
                                 inv_bind=s["inv"], skin_out=s["S"])
        elif self.name == "plain_scan":
            call, _ = hs.prepare(hs.hs_scan_forward, self.plan, s["q"], s["t"], s["s"], want_global=False,
                                 inv_bind=s["inv"], skin_out=s["S"])
        else:
            call, _ = hs.prepare(hs.hs_scan_forward, self.plan, s["q"], s["t"], s["s"], global_out=s["G"])
        return call

    def mode_ms(self, mode, steps):
        """Mean time per step of `steps` steps in the given launch mode."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        self.run(steps, mode)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def step(self, k):
        """One step on set k (cycled)."""
        s = self.sets[k % len(self.sets)]
        if self.graphs is not None:
            self.graphs[k % len(self.sets)].launch()
            return
        self.diff_step(s)

    def diff_step(self, s):
        """Forward and the adjoint of loss = sum over effectors |b_e - y_e|^2
        on set s (differentiable workload), in one launch: each adjoint tile
        scans its characters, writes G, forms the loss gradient at the
        effectors and runs the reverse rounds."""
        self.hs.hs_effector_step(self.plan, self.effset, s["q"], s["t"], s["s"], self.target, global_out=s["G"],
                                 want_scale=False, grad_quat=s["gq"], grad_trans=s["gt"])

    def two_call_step(self, s):
        """The same step as two launches: the forward, then the adjoint
        seeded from the forward's output."""
        hs = self.hs
        hs.hs_scan_forward(self.plan, s["q"], s["t"], s["s"], global_out=s["G"])
        hs.hs_effector_backward(self.plan, self.effset, s["q"], s["t"], s["s"], s["G"], self.target,
                                want_scale=False, grad_quat=s["gq"], grad_trans=s["gt"])

    def dense_step(self, s):
        """The same step through a dense dLoss/dG: the loss gradient enters
        the effector rows of the (otherwise zero) buffer, which the general
        adjoint reads whole."""
        hs = self.hs
        hs.hs_scan_forward(self.plan, s["q"], s["t"], s["s"], global_out=s["G"])
        hs.hs_effector_loss_grad(s["G"], self.eff, self.target, self.gG)
        hs.hs_scan_backward(self.plan, s["q"], s["t"], s["s"], self.gG, want_scale=False,
                            grad_quat=s["gq"], grad_trans=s["gt"])

    def ckpt_step(self, s):
        """The dense route in the level-checkpoint memory mode: the forward
        also stores rows 0-2 of G at every CKPT_K-th level, and the adjoint
        rebuilds each G_j from its nearest checkpointed ancestor instead of
        recomputing the scan."""
        hs = self.hs
        hs.hs_scan_forward(self.plan, s["q"], s["t"], s["s"], global_out=s["G"], ckpt_out=s["ck"], ckpt_k=CKPT_K)
        hs.hs_effector_loss_grad(s["G"], self.eff, self.target, self.gG)
        hs.hs_scan_backward(self.plan, s["q"], s["t"], s["s"], self.gG, ckpt=s["ck"], ckpt_k=CKPT_K,
                            want_scale=False, grad_quat=s["gq"], grad_trans=s["gt"])

    def adjoint_ms(self, ckpt, reps=50):
        """Mean duration of the general adjoint's launch alone (dense
        dLoss/dG of the effector loss), recompute or checkpoint mode."""
        torch, s, hs = self.torch, self.sets[0], self.hs
        self.ckpt_step(s)
        kw = dict(ckpt=s["ck"], ckpt_k=CKPT_K) if ckpt else {}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            hs.hs_scan_backward(self.plan, s["q"], s["t"], s["s"], self.gG, want_scale=False, grad_quat=s["gq"],
                                grad_trans=s["gt"], **kw)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def graph_step_ms(self, graph, reps=5):
        """Mean time per step of a captured comparison route."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        graph.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (reps * self.chunk)

    def forward_ms(self, reps=50):
        """Mean duration of the forward launch alone, back to back (the
        two-call route's first launch)."""
        torch, s = self.torch, self.sets[0]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            self.hs.hs_scan_forward(self.plan, s["q"], s["t"], s["s"], global_out=s["G"])
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps



def measure(args, name):
    """Time one workload's steps and return its JSON record (without the
    keys of the line's frame: metric, n_gpus, ...)."""
    import torch
    w = Workload(name, autotune=not args.no_autotune, adjoint=args.adjoint, shape=fixed_shape(args))
    b, info = w.b, w.plan.info
    N, C = b.num_joints, b.num_characters

    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 4, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w.run(args.warmup)
    diff = name == "differentiable"
    # the launch mode of the timed region: captured graphs or direct calls,
    # whichever runs the same steps faster on this machine (graphs win where a
    # step is shorter than a host call, direct calls where it is long)
    calib = 3 * w.chunk
    modes = {"graph": float("inf"), "plain": float("inf")}
    for _ in range(2):  # alternated, best of two: clock ramps favour neither mode
        for m in modes:
            modes[m] = min(modes[m], w.mode_ms(m, calib))
    mode = min(modes, key=modes.get)
    region = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    region[0].record()
    w.run(args.steps, mode)
    region[1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    dominant = DOMINANT.get(name, "fwd_queue_kernel" if info["schedule"] == w.hs.HS_SCHED_QUEUE
                            else "fwd_tile_kernel")
    if diff and args.adjoint in ("rounds", "dataflow"):
        dominant = "bwd_sync_kernel"  # the effector step's kernel under these options
    # one launch per step (the forward's work queue or classes launched back
    # to back; the differentiable step's one kernel): HIP events around the
    # timed region give the step's mean kernel time, on the cycled sets
    kernel_ms = region[0].elapsed_time(region[1]) / args.steps
    if diff:
        # the forward launch alone, back to back on one set (the two-call
        # route's first launch), for the split of the step
        fwd_ms = w.forward_ms()
    bytes_per_launch = N * BYTES_PER_JOINT[name]
    if diff:
        bytes_per_launch += 12 * w.effset.num_effectors
    if name in FUSED:
        bytes_per_launch += b.extra["key_quat"].nbytes + b.extra["key_trans"].nbytes + 16 * C
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    copy_gbs = device_copy_gbs(torch)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name),
            "kernel": dominant, "kernel_ms": kernel_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
            "device_copy_GBs": copy_gbs, "frac_of_device_copy": achieved / copy_gbs}
    if BYTES_PER_JOINT[name] == 108:
        # the achievable rate of this access pattern, measured beside it
        probe = stream_probe_gbs(torch, w.hs, N)
        roof["stream_probe_GBs"] = probe
        roof["frac_of_stream_probe"] = achieved / probe
    if diff:
        roof["forward_kernel_ms"] = fwd_ms
        roof["two_call_ms_per_step"] = w.graph_step_ms(w.two_call_graph)
    launch = {"timed": mode, "graph_ms_per_step": modes["graph"], "plain_call_ms_per_step": modes["plain"],
              "calibration_steps": calib}
    out = {
        "value": N * args.steps / elapsed,
        "unit": "joint transforms/s" + (" (forward + adjoint)" if diff else ""),
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "config": {"workload": name, "characters": C, "joints": N, "max_depth": info["max_depth"],
                   "tile_joints": info["tile_joints"], "waves_per_tile": info["waves_per_tile"],
                   "grid": info["grid"], "tiles": info["num_tiles"], "multipass_joints": info["multipass_joints"],
                   "schedule": "queue" if info["schedule"] == w.hs.HS_SCHED_QUEUE else "size classes",
                   "autotuned": not args.no_autotune and not fixed_shape(args) and name != "fused_sample",
                   "hip_graph": mode == "graph",
                   "input_sets": len(w.sets),
                   **({"adjoint": args.adjoint,
                       "adjoint_blocks_per_wave": info["adjoint_blocks_per_wave"]} if diff else {})},
        "roofline": roof,
        "launch_modes": launch,
    }
    if diff:
        out["memory_modes"] = memory_modes(w)
    if name == "heterogeneous" and not args.no_schedules and not args.calibrate_copy:
        out["schedules"] = schedule_alternatives(w, info)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["err_vs_fp64"], ref_grads = cpu_baseline(w)
        if diff:
            # the two memory modes against the oracle's gradients
            for key, ck in (("recompute", False), (f"checkpoint_k{CKPT_K}", True)):
                out["memory_modes"][key]["err_vs_fp64"] = grad_errors(w, ck, ref_grads)
    w.close()
    return out


def schedule_alternatives(w, info, steps=60, warmup=10):
    """The same forward through the other launch schedules, as plain calls
    over the cycled sets: the work queue as a resident loop (four
    workgroups per CU walking the heaviest-first tile list, grid < tiles)
    at the line's tile and wave shape, and the size classes (one launch per
    class) at the plan's default shape.  The line's own schedule is the
    timed region above."""
    torch, hs, b = w.torch, w.hs, w.b
    plans = {
        "queue_resident_loop": hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE,
                                       tile_joints=info["tile_joints"], waves_per_tile=info["waves_per_tile"],
                                       grid_tiles=4),  # workgroups per CU
        "size_classes": hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_CLASSES),
    }
    res = {}
    for key, plan in plans.items():
        pi = plan.info

        def step(k):
            st = w.sets[k % len(w.sets)]
            hs.hs_scan_forward(plan, st["q"], st["t"], st["s"], global_out=st["G"])

        for k in range(warmup):
            step(k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for k in range(steps):
            step(k)
        e1.record()
        torch.cuda.synchronize()
        res[key] = {"ms_per_step": e0.elapsed_time(e1) / steps, "grid": pi["grid"], "tiles": pi["num_tiles"],
                    "tile_joints": pi["tile_joints"], "waves_per_tile": pi["waves_per_tile"],
                    "launches": 1 if pi["schedule"] == hs.HS_SCHED_QUEUE else "one per size class"}
        plan.close()
    return res


def memory_modes(w):
    """The differentiable form through the general adjoint (dense
    dLoss/dG) in its two memory modes: the whole step per mode (captured,
    CKPT_K-step graphs) and the adjoint launch alone, with the adjoint's
    algorithmic bytes: read the pose 44, dLoss/dG 64, write dq 16 + dt 12;
    the checkpoint mode also reads each joint's level (4) and the
    checkpoint rows (48 per checkpointed joint), and its forward writes
    them."""
    N = w.b.num_joints
    from paper_2505_06703_amd.workloads import levels_of
    off, par = w.b.offsets, w.b.parents
    lev = np.concatenate([levels_of(par[off[c]:off[c + 1]]) for c in range(w.b.num_characters)])
    n_ck = int(np.count_nonzero(lev % CKPT_K == 0))
    res = {}
    for key, ck in (("recompute", False), (f"checkpoint_k{CKPT_K}", True)):
        step = w.graph_step_ms(w.ckpt_graph if ck else w.dense_graph)
        adj = w.adjoint_ms(ck)
        nbytes = N * 136 + ((N * 4 + n_ck * 48) if ck else 0)
        res[key] = {"ms_per_step": step, "adjoint_kernel": "bwd_tile_kernel (checkpoints)" if ck else
                    "bwd_sync_kernel (dense seed)", "adjoint_kernel_ms": adj,
                    "adjoint_algorithmic_bytes": nbytes,
                    "adjoint_frac": nbytes / (adj * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "checkpointed_joints": n_ck if ck else 0}
    return res


def grad_errors(w, ckpt, ref):
    """Gradient errors of one dense-route step (memory mode as asked)
    against the oracle's reverse mode."""
    torch = w.torch
    s0 = w.sets[0]
    (w.ckpt_step if ckpt else w.dense_step)(s0)
    torch.cuda.synchronize()
    gq, gt, _ = ref
    err = {}
    for key, g, r in (("grad_quat", s0["gq"], gq), ("grad_trans", s0["gt"], gt)):
        g = g.cpu().numpy().astype(np.float64)
        err[key + "_rel_max"] = float(np.abs(g - r).max() / max(1.0, np.abs(r).max()))
    return err


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.workload, *args.summarize_pmc)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; characters are independent, "
                                   "so a multi-GPU run would split the batch into contiguous character "
                                   "ranges, one plan per GPU, with no exchange",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.depth_sweep:
        depth_sweep(args)
        return
    if args.workload == "mesh_skinning":
        mesh_bench(args)
        return
    if args.workload == "sample_gradients":
        sampler_grad_bench(args)
        return
    rec = measure(args, args.workload)
    out = {"metric": METRIC, "value": rec.pop("value"), "unit": rec.pop("unit"), "n_gpus": 1,
           "steps": rec.pop("steps"), "warmup": rec.pop("warmup"), "ms_per_step": rec.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    out.update(rec)
    # a counter run (--calibrate-copy) covers the named workload's kernel
    # only: the differentiable form launches the same forward kernel
    if args.workload == "heterogeneous" and not args.no_fwd_bwd and not args.calibrate_copy:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["fwd_bwd"] = measure(args, "differentiable")
    print(json.dumps(out), flush=True)


ALG_NAMES = ["scan (this library)", "1: walk to root", "2: pointer jumping", "3: blocks + walk",
             "4: window + hops + walk"]


def depth_sweep(args):
    """Forward time per step for each depth and tile algorithm (inputs in
    HBM, two input sets alternating, eight passes per graph replay)."""
    import torch
    from paper_2505_06703_amd import hs
    from paper_2505_06703_amd import workloads as wl
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for depth in (15, 30, 60, 90, 120):
        b = wl.depth_sweep(depth=depth)
        N = b.num_joints
        sets = [dict(quat=up(b.quat), trans=up(b.trans), scale=up(b.scale),
                     global_out=torch.empty((N, 4, 4), device="cuda:0")) for _ in range(2)]
        for alg in range(5):
            plan = hs.Plan(b.offsets, b.parents, algorithm=alg, autotune=(alg == 0 and not args.no_autotune))
            g = hs.ForwardGraph.sequence(plan, [sets[k % 2] for k in range(CHUNK)])
            reps = max(1, args.steps // CHUNK)
            for _ in range(max(1, args.warmup // CHUNK)):
                g.launch()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                g.launch()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (reps * CHUNK)
            print(json.dumps({"depth": depth, "algorithm": ALG_NAMES[alg], "characters": b.num_characters,
                              "joints": N, "us_per_step": ms * 1e3, "joints_per_s": N / (ms * 1e-3),
                              "hbm_frac": N * BYTES_PER_JOINT["deep_forward"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "tile_joints": plan.info["tile_joints"]}), flush=True)
            g.close()
            plan.close()


def mesh_bench(args):
    """The mesh_skinning workload: per step, the fused forward of the
    instanced batch (clip sampling, scan, skin matrices) and vertex skinning
    of every character's mesh; one JSON line per skinning method.  Output
    sets cycled so that one cycle touches at least SWEEP_BYTES."""
    import torch
    from paper_2505_06703_amd import hs
    from paper_2505_06703_amd import workloads as wl
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b = wl.mesh_skinning()
    x = b.extra
    N, C = b.num_joints, b.num_characters
    plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"], autotune=not args.no_autotune)
    one = hs.Plan(x["skel_offsets"], x["skel_parents"])
    Grest, _ = hs.hs_scan_forward(one, *(up(a) for a in x["skel_rest"]))
    inv = up(np.linalg.inv(Grest.cpu().numpy().astype(np.float64)).astype(np.float32))
    lib = hs.ClipLibrary(up(x["key_quat"]), up(x["key_trans"]), x["fps"])
    cp = dict(clip_a=up(x["clip_a"]), clip_b=up(x["clip_b"]), time=up(x["time"]), weight=up(x["weight"]))
    mesh = hs.Mesh(plan, x["vertex_offsets"], x["mesh_first"], x["mesh_positions"], x["mesh_joints"],
                   x["mesh_weights"])
    V = mesh.num_vertices
    set_bytes = N * 64 + V * 12
    n_sets = int(min(MAX_SETS, max(2, -(-SWEEP_BYTES // set_bytes))))
    sets = [(torch.empty((N, 4, 4), device="cuda:0"), torch.empty((V, 3), device="cuda:0")) for _ in range(n_sets)]
    rows = x["mesh_positions"].shape[0]
    # algorithmic bytes of one vertex-skinning launch: rows 0-2 of every skin
    # matrix read, every vertex written, the shared mesh rows read once
    vbytes = N * 48 + V * 12 + rows * 44 + C * 20
    variants = [(m, nm, fused) for fused in (False, True)
                for m, nm in ((hs.HS_SKIN_LINEAR, "linear"), (hs.HS_SKIN_DUAL_QUAT, "dual_quat"))]
    for method, name, fused in variants:
        def step(k, ev=None):
            S, out = sets[k % n_sets]
            if fused:
                # one pass per tile: S stays on chip
                if ev is not None:
                    ev[0].record()
                hs.hs_scan_skin_vertices(plan, mesh, inv, clips=lib, **cp, method=method, vertices_out=out)
                if ev is not None:
                    ev[1].record()
                return
            hs.hs_scan_forward(plan, clips=lib, **cp, want_global=False, inv_bind=inv, skin_out=S)
            if ev is not None:
                ev[0].record()
            hs.hs_skin_vertices(mesh, S, method, out)
            if ev is not None:
                ev[1].record()
        for k in range(args.warmup):
            step(k)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(k, evs[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
        # the one-pass kernel moves only the clip parameters in and the
        # vertices out (the skeleton tables, clip library and mesh rows are
        # cache-resident): its algorithmic bytes
        fbytes = V * 12 + rows * 44 + C * 20 + x["key_quat"].nbytes + x["key_trans"].nbytes
        nbytes = fbytes if fused else vbytes
        achieved = nbytes / (kms * 1e-3) / 1e9
        print(json.dumps({
            "metric": "skinned vertices/s (clip sampling + scan + skin + vertex skinning) on 1 GPU",
            "value": V * args.steps / elapsed, "unit": "vertices/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "mesh_skinning", "method": name, "one_pass": fused, "characters": C,
                       "joints": N, "vertices": V, "faces_per_mesh": 2 * (V // C) - 4, "input_sets": n_sets},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "fwd_vertex_kernel" if fused else "vertex_skin_kernel",
                         "kernel_ms": kms, "algorithmic_bytes_per_launch": nbytes}}), flush=True)


def sampler_grad_bench(args):
    """Gradients through the Simulation step on the fused_sample batch: per
    step the sampler, the scan, the scan's adjoint and the sampler's reverse
    mode (keyframes, times, weights), with a fixed dLoss/dG (the effector
    loss gradient at the start: the kernels' work does not depend on its
    values).  Sets cycled so that one cycle touches at least SWEEP_BYTES."""
    import torch
    from paper_2505_06703_amd import hs
    from paper_2505_06703_amd import workloads as wl
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b = wl.fused_sample()
    x = b.extra
    N, C = b.num_joints, b.num_characters
    plan = hs.Plan(b.offsets, b.parents, autotune=not args.no_autotune)
    lib = hs.ClipLibrary(up(x["key_quat"]), up(x["key_trans"]), x["fps"])
    ca, cb, tm, wt = up(x["clip_a"]), up(x["clip_b"]), up(x["time"]), up(x["weight"])
    rng = np.random.default_rng(0)
    W = np.zeros((N, 4, 4), np.float32)
    tips = np.arange(C) * 256 + 255  # one effector per chain tip of the hair
    W[tips, :3, 3] = rng.standard_normal((C, 3))
    set_bytes = N * (16 + 12 + 64 + 64 + 16 + 12)
    n_sets = int(min(MAX_SETS, max(2, -(-SWEEP_BYTES // set_bytes))))
    sets = []
    for _ in range(n_sets):
        sets.append(dict(q=torch.empty((N, 4), device="cuda:0"), t=torch.empty((N, 3), device="cuda:0"),
                         G=torch.empty((N, 4, 4), device="cuda:0"), gG=up(W),
                         gq=torch.empty((N, 4), device="cuda:0"), gt=torch.empty((N, 3), device="cuda:0")))
    # each joint's reverse step stored once, the key gather reads it
    ws = hs.sample_backward_workspace(plan, "cuda:0")

    def step(k, ev=None):
        st = sets[k % n_sets]
        hs.hs_pose_sample(plan, lib, ca, cb, tm, wt, quat_out=st["q"], trans_out=st["t"])
        hs.hs_scan_forward(plan, st["q"], st["t"], None, global_out=st["G"])
        hs.hs_scan_backward(plan, st["q"], st["t"], None, st["gG"], want_scale=False, grad_quat=st["gq"],
                            grad_trans=st["gt"])
        if ev is not None:
            ev[0].record()
        out = hs.hs_pose_sample_backward(plan, lib, ca, cb, tm, wt, st["gq"], st["gt"], workspace=ws)
        if ev is not None:
            ev[1].record()
        return out

    for k in range(args.warmup):
        step(k)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    # the same reverse mode without the workspace (the gather recomputes
    # each reader's reverse step), for comparison
    st = sets[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        hs.hs_pose_sample_backward(plan, lib, ca, cb, tm, wt, st["gq"], st["gt"])
    e1.record()
    torch.cuda.synchronize()
    recompute_ms = e0.elapsed_time(e1) / 10
    # algorithmic bytes of one reverse-mode launch: dLoss/dq and dLoss/dt
    # read, the key gradients written once, per-character parameters read
    # and gradients written
    keys = x["key_quat"].nbytes + x["key_trans"].nbytes
    sbytes = N * 28 + keys + C * 24
    achieved = sbytes / (kms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "joint transforms/s through sampler, scan, adjoint and sampler reverse mode on 1 GPU",
        "value": N * args.steps / elapsed, "unit": "joint transforms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sample_gradients", "characters": C, "joints": N, "clips": int(x["key_quat"].shape[0]),
                   "keys": int(x["key_quat"].shape[1]), "input_sets": n_sets},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "sample_bwd_kernel",
                     "kernel_ms": kms, "algorithmic_bytes_per_launch": sbytes,
                     "recompute_gather_ms": recompute_ms}}), flush=True)


def device_copy_gbs(torch, nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device-to-device copy (bytes read + written per
    second), the practical HBM ceiling the kernel is also compared with."""
    src = torch.empty(nbytes // 4, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def stream_probe_gbs(torch, hs, n, reps=20):
    """Rate of hs_stream_probe over n joints: the forward's 108 bytes per
    joint (44 read, 64 written, the same access pattern) with no
    arithmetic, the HBM rate this kernel shape can reach."""
    dev = "cuda:0"
    q = torch.zeros((n, 4), device=dev)
    t = torch.zeros((n, 3), device=dev)
    s = torch.zeros((n, 3), device=dev)
    tab = torch.zeros((n,), device=dev, dtype=torch.int32)
    out = torch.empty((n, 4, 4), device=dev)
    for _ in range(3):
        hs.hs_stream_probe(q, t, s, tab, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        hs.hs_stream_probe(q, t, s, tab, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del q, t, s, tab, out
    return 108.0 * n / (ms * 1e-3) / 1e9


def cpu_baseline(w):
    """Time the FP64 oracle on the host (all the cores it may use) on repeated
    passes over the full batch, and compare one fresh GPU step with it."""
    import oracle

    torch, b, name = w.torch, w.b, w.name
    cores = len(os.sched_getaffinity(0))
    N = b.num_joints
    if name in FUSED:
        x = b.extra

        def run():
            q, t = oracle.pose_sample(b.offsets, x["key_quat"], x["key_trans"], x["clip_a"], x["clip_b"], x["time"],
                                      x["weight"], x["fps"])
            return oracle.forward(b.offsets, b.parents, q, t, None), t
    elif name == "differentiable":
        # the oracle's own targets: its rest-pose positions plus the seeded
        # offsets (the GPU step's targets come from the GPU's rest pose;
        # their fp32 rounding is part of the reported gradient error)
        eff = b.extra["effectors"]
        rest = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
        target = rest[eff, :3, 3] + b.extra["target_offsets"].astype(np.float64)

        def run():
            G = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
            W = np.zeros((N, 4, 4))
            W[eff, :3, 3] = 2.0 * (G[eff, :3, 3] - target)
            run.grads = oracle.backward(b.offsets, b.parents, b.quat, b.trans, b.scale, W)
            return G, b.trans
    else:
        def run():
            return oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale), b.trans
    def timed(seconds):
        reps, t0 = 0, time.perf_counter()
        while True:
            out = run()
            reps += 1
            wall = time.perf_counter() - t0
            if wall >= seconds or reps >= 2000:
                return out, reps, wall

    threads = oracle.set_threads(cores)
    (G, tr), reps, wall = timed(10.0)
    oracle.set_threads(1)
    _, reps1, wall1 = timed(5.0)
    oracle.set_threads(threads)
    what = "forward + adjoint" if name == "differentiable" else "forward"
    base = {"value": N * reps / wall, "unit": "joint transforms/s", "cores": threads, "kind": "oracle",
            "sample": f"full {name} batch ({b.num_characters} characters, {N} joints, FP64 {what}) x {reps} "
                      f"passes on {threads} threads, fp32->fp64 widening included, {wall:.1f} s wall",
            "value_1thread": N * reps1 / wall1}

    w.step(0)
    torch.cuda.synchronize()
    s0 = w.sets[0]
    lam = oracle.path_length(b.offsets, b.parents, G, tr)
    if name in ("deep_forward", "heterogeneous", "differentiable", "long_chains"):
        Gg = s0["G"].cpu().numpy().astype(np.float64)
        db = np.abs(Gg[:, :3, 3] - G[:, :3, 3]).max(axis=1)
        err = {"rotation_abs_max": float(np.abs(Gg[:, :3, :3] - G[:, :3, :3]).max()),
               "translation_rel_max": float((db / np.maximum(lam, 1e-12)).max())}
        if name == "differentiable":
            gq, gt, _ = run.grads
            for key, g, r in (("grad_quat", s0["gq"], gq), ("grad_trans", s0["gt"], gt)):
                g = g.cpu().numpy().astype(np.float64)
                err[key + "_rel_max"] = float(np.abs(g - r).max() / max(1.0, np.abs(r).max()))
    else:
        # the oracle's own inverse binds (FP64 inverse of its rest pose,
        # rounded to fp32); the GPU step's come from the GPU's rest pose, and
        # their rounding differences are part of the reported skin error
        if name == "fused_sample_instanced":  # one skeleton: expand its rows
            x = b.extra
            soff = x["skel_offsets"]
            rest = oracle.forward(soff, x["skel_parents"], *x["skel_rest"])
            inv = np.linalg.inv(rest).astype(np.float32)
            inv = inv[np.concatenate([np.arange(soff[k], soff[k + 1]) for k in x["skeleton_id"]])]
        else:
            rest = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
            inv = np.linalg.inv(rest).astype(np.float32)
        S = oracle.skin(G, inv)
        Sg = s0["S"].cpu().numpy().astype(np.float64)
        err = {"skin_rotation_abs_max": float(np.abs(Sg[:, :3, :3] - S[:, :3, :3]).max()),
               "skin_translation_abs_max": float(np.abs(Sg[:, :3, 3] - S[:, :3, 3]).max())}
    return base, err, getattr(run, "grads", None)


if __name__ == "__main__":
    main()

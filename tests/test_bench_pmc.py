"""Host logic of bench.py's HBM-traffic summary (--summarize-pmc) on
synthetic rocprofv3 counter files: the calibration copy is the first copy
that writes its size (not the input uploads or small setup copies before
it, nor the larger bandwidth probe after it), and only the dominant
kernel's instance is averaged; no GPU."""
import csv
import json

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
MIB = 1024.0  # counter values are KiB


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, name, kib in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})
        # another counter in the same file is ignored
        w.writerow({"Dispatch_Id": 999, "Kernel_Name": "fwd_tile_kernel<8, false, 0>", "Counter_Name": "OTHER",
                    "Counter_Value": 1e9})


def run(tmp_path, monkeypatch, workload, fetch_rows, write_rows):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_csv(f, "FETCH_SIZE", fetch_rows)
    write_csv(w, "WRITE_SIZE", write_rows)
    bench.summarize_pmc(workload, str(f), str(w))
    return json.load(open(tmp_path / "traffic.json"))[workload]


def test_calibration_copy_and_scales(tmp_path, monkeypatch):
    copy = "__amd_rocclr_copyBuffer"
    # dispatch order is taken from the ids, not from the file's row order
    fetch = [(5, "fwd_tile_kernel<8, false, 0>", 90.0 * MIB), (1, copy, 0.0), (3, copy, 128.0 * MIB),
             (2, copy, 1.0), (9, copy, 512.0 * MIB), (6, "fwd_tile_kernel<8, false, 0>", 92.0 * MIB)]
    write = [(5, "fwd_tile_kernel<8, false, 0>", 256.0 * MIB), (3, copy, 256.0 * MIB), (1, copy, 0.0),
             (9, copy, 1024.0 * MIB), (6, "fwd_tile_kernel<8, false, 0>", 256.0 * MIB)]
    rec = run(tmp_path, monkeypatch, "deep_forward", fetch, write)
    assert rec["copy_dispatch"] == [3, 3]
    assert rec["copy_fetch_scale"] == 2.0 and rec["copy_write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 91.0 * MIB * 1024.0 * 2.0
    assert rec["write_bytes_per_launch"] == 256.0 * MIB * 1024.0
    assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert rec["source_sha"] == bench.kernel_source_sha()


def test_only_the_dominant_instance_is_averaged(tmp_path, monkeypatch):
    copy = "__amd_rocclr_copyBuffer"
    # the step's instance (seeds from the tile's own forward; waves, blocks
    # per wave, seed kind) next to the comparison routes' kernels and other
    # instances of the same template
    fetch = [(2, copy, 128.0 * MIB), (4, "void hs::bwd_anchor_kernel<4, 2, 2>(hs::TileLaunch)", 13.0 * MIB),
             (5, "void hs::bwd_sync_kernel<8, 0>(hs::TileLaunch)", 28.0 * MIB),
             (6, "void hs::bwd_anchor_kernel<4, 2, 1>(hs::TileLaunch)", 20.0 * MIB),
             (8, "void hs::bwd_sync_kernel<8, 2>(hs::TileLaunch)", 11.0 * MIB),
             (7, "void hs::bwd_anchor_kernel<4, 2, 2>(hs::TileLaunch)", 13.0 * MIB)]
    write = [(2, copy, 256.0 * MIB), (4, "void hs::bwd_anchor_kernel<4, 2, 2>(hs::TileLaunch)", 14.0 * MIB),
             (5, "void hs::bwd_sync_kernel<8, 0>(hs::TileLaunch)", 50.0 * MIB)]
    rec = run(tmp_path, monkeypatch, "differentiable", fetch, write)
    assert rec["fetch_bytes_per_launch"] == 13.0 * MIB * 1024.0 * 2.0
    assert rec["write_bytes_per_launch"] == 14.0 * MIB * 1024.0


def test_records_of_other_workloads_are_kept(tmp_path, monkeypatch):
    (tmp_path / "traffic.json").write_text(json.dumps({"long_chains": {"kernel": "x"}}))
    copy = "__amd_rocclr_copyBuffer"
    rows = [(1, copy, 128.0 * MIB), (2, "fwd_tile_kernel<8, false, 0>", 1.0)]
    wrows = [(1, copy, 256.0 * MIB), (2, "fwd_tile_kernel<8, false, 0>", 1.0)]
    run(tmp_path, monkeypatch, "deep_forward", rows, wrows)
    data = json.load(open(tmp_path / "traffic.json"))
    assert set(data) == {"long_chains", "deep_forward"}


def test_the_work_queue_launch_is_the_forward_kernel_when_present(tmp_path, monkeypatch):
    copy = "__amd_rocclr_copyBuffer"
    fetch = [(1, copy, 128.0 * MIB), (2, "void hs::fwd_queue_kernel<4, false>(hs::QueueLaunch)", 30.0 * MIB),
             (3, "void hs::fwd_tile_kernel<8, false, 0>(hs::TileLaunch)", 99.0 * MIB)]
    write = [(1, copy, 256.0 * MIB), (2, "void hs::fwd_queue_kernel<4, false>(hs::QueueLaunch)", 64.0 * MIB)]
    rec = run(tmp_path, monkeypatch, "heterogeneous", fetch, write)
    assert rec["kernel"] == "fwd_queue_kernel"
    assert rec["fetch_bytes_per_launch"] == 30.0 * MIB * 1024.0 * 2.0
    assert rec["write_bytes_per_launch"] == 64.0 * MIB * 1024.0


def test_input_uploads_before_the_calibration_copy_are_skipped(tmp_path, monkeypatch):
    copy = "__amd_rocclr_copyBuffer"
    kern = "void hs::fwd_queue_kernel<4, true>(hs::QueueLaunch)"
    # 156.25 MiB uploads of the inputs come first; the calibration copy
    # (256 MiB written, half of it counted by FETCH_SIZE) follows
    fetch = [(3, copy, 156.25 * MIB), (4, copy, 156.25 * MIB), (7, copy, 128.0 * MIB), (8, kern, 200.0 * MIB)]
    write = [(3, copy, 156.25 * MIB), (4, copy, 156.25 * MIB), (7, copy, 256.0 * MIB), (8, kern, 156.25 * MIB)]
    rec = run(tmp_path, monkeypatch, "fused_sample", fetch, write)
    assert rec["copy_dispatch"] == [7, 7]
    assert rec["copy_fetch_scale"] == 2.0 and rec["copy_write_scale"] == 1.0
    assert rec["write_bytes_per_launch"] == 156.25 * MIB * 1024.0


def test_a_multipass_step_sums_its_kernels(tmp_path, monkeypatch):
    """long_chains: the chain kernel and the block path's output pass (a
    batch with chain and non-chain characters beyond a tile) are one step
    (their averages add); multipass kernels absent from the run count
    nothing."""
    copy = "__amd_rocclr_copyBuffer"
    chain = "void hs::mp_chain_kernel<false>(hs::ChainLaunch, hs::PoseArgs, hs::OutArgs)"
    zero = "void hs::mp_out_kernel(hs::MPLaunch, hs::PoseArgs, hs::OutArgs)"
    fetch = [(1, copy, 128.0 * MIB), (2, zero, 0.0), (3, chain, 100.0 * MIB), (4, zero, 2.0),
             (5, chain, 102.0 * MIB)]
    write = [(1, copy, 256.0 * MIB), (2, zero, 4.0), (3, chain, 300.0 * MIB), (4, zero, 4.0),
             (5, chain, 300.0 * MIB)]
    rec = run(tmp_path, monkeypatch, "long_chains", fetch, write)
    assert rec["fetch_bytes_per_launch"] == (101.0 * MIB + 1.0) * 1024.0 * 2.0
    assert rec["write_bytes_per_launch"] == (300.0 * MIB + 4.0) * 1024.0

"""Parity of the launches the benchmark times: every benchmarked workload at
full size, its plan built as the benchmark builds it (launch shape chosen
by the autotuner at plan time), the step it times, checked against the FP64
oracle on seeded samples of whole characters (characters are independent,
so a sample is exact).  Tolerances as in tests/parity.py (the scan's) and
tests/test_gpu_backward.py (the adjoint's)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl
from parity import check_global, check_skin, inverse_binds

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def sample_chars(b, k, seed, extra=()):
    """First, last, largest and k seeded characters (plus `extra`)."""
    rng = np.random.default_rng(seed)
    sizes = np.diff(b.offsets)
    picks = [0, b.num_characters - 1, int(np.argmax(sizes)), *extra]
    picks += list(rng.choice(b.num_characters, k, replace=False))
    return np.unique(np.asarray(picks, np.int64))


def sub_batch(b, chars, quat=None, trans=None, scale=None):
    """Offsets, parents and poses of the listed characters as a batch of
    their own, with their global joint ids."""
    q = b.quat if quat is None else quat
    t = b.trans if trans is None else trans
    s = b.scale if scale is None else scale
    ids = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in chars])
    off = np.concatenate([[0], np.cumsum(np.diff(b.offsets)[chars])]).astype(np.int64)
    return off, b.parents[ids], q[ids], t[ids], None if s is None else s[ids], ids


def check_forward_sample(G, b, chars, what):
    off, par, q, t, s, ids = sub_batch(b, chars)
    Gr = oracle.forward(off, par, q, t, s)
    lam = oracle.path_length(off, par, Gr, t)
    return check_global(G[ids], Gr, lam, what)


def test_long_chains_multipass_full_size():
    """The multipass benchmark (64 chains of 65 536 joints) as the bench
    builds it, every chain checked against the oracle at the flat tolerance
    (no depth scaling: these chains stay within it)."""
    b = wl.make("long_chains")
    plan = hs.Plan(b.offsets, b.parents, autotune=True)
    assert plan.info["multipass_joints"] == b.num_joints
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    for c0 in range(0, b.num_characters, 16):  # 16 chains at a time: bounded host memory
        chars = np.arange(c0, min(c0 + 16, b.num_characters))
        check_forward_sample(G, b, chars, f"long chains {c0}-{chars[-1]}")


@pytest.mark.parametrize("name", ["deep_forward", "heterogeneous"])
def test_forward_workload_autotuned(name):
    """The plain forward (global transforms), deep and heterogeneous
    (size classes, pure chains), as the benchmark's step."""
    b = wl.make(name)
    plan = hs.Plan(b.offsets, b.parents, autotune=True)
    assert plan.info["multipass_joints"] == 0
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    extra = ()
    if name == "heterogeneous":
        sizes = np.diff(b.offsets)
        chains = [c for c in range(b.num_characters)
                  if sizes[c] > 64 and np.all(b.parents[b.offsets[c] + 1:b.offsets[c + 1]] ==
                                              np.arange(sizes[c] - 1))]
        assert chains, "the workload holds pure chains"
        extra = tuple(sorted(chains, key=lambda c: -sizes[c])[:4])
    check_forward_sample(G, b, sample_chars(b, 24, 40, extra), f"{name} autotuned")
    assert np.array_equal(G[:, 3, :], np.broadcast_to([0.0, 0.0, 0.0, 1.0], (b.num_joints, 4)))


@pytest.mark.parametrize("waves", [4, 8])
def test_heterogeneous_schedules_the_bench_compares(waves):
    """The launches of the heterogeneous line's schedule comparison: the
    work queue as a resident loop (four workgroups per CU, grid < tiles)
    computes what one workgroup per tile computes, bit for bit (the same
    tiles, the same arithmetic), and both match the oracle on a sample."""
    b = wl.make("heterogeneous")
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    shape = dict(schedule=hs.HS_SCHED_QUEUE, tile_joints=2048, waves_per_tile=waves)
    per_tile = hs.Plan(b.offsets, b.parents, **shape)
    resident = hs.Plan(b.offsets, b.parents, grid_tiles=4, **shape)
    assert per_tile.info["grid"] == per_tile.info["num_tiles"]
    assert resident.info["grid"] < resident.info["num_tiles"] == per_tile.info["num_tiles"]
    G1, _ = hs.hs_scan_forward(per_tile, q, t, s)
    G2, _ = hs.hs_scan_forward(resident, q, t, s)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)
    check_forward_sample(G2.cpu().numpy(), b, sample_chars(b, 16, 41), f"heterogeneous resident loop, {waves} waves")


def test_heterogeneous_size_classes():
    """The size-class schedule of the line's comparison (one launch per
    class, the plan's default shapes) against the oracle on a sample."""
    b = wl.make("heterogeneous")
    plan = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_CLASSES)
    assert plan.info["schedule"] == hs.HS_SCHED_CLASSES
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    check_forward_sample(G.cpu().numpy(), b, sample_chars(b, 16, 42), "heterogeneous size classes")


@pytest.mark.parametrize("name", ["fused_sample", "fused_sample_instanced"])
def test_fused_workload_autotuned(name):
    """Clip sampling, scan and skin in one launch (per-joint and instanced
    plans), skin matrices only, as the benchmark's step."""
    b = wl.make(name)
    x = b.extra
    if name == "fused_sample_instanced":
        plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"], autotune=True)
        inv_s = np.linalg.inv(oracle.forward(x["skel_offsets"], x["skel_parents"], *x["skel_rest"]))
        inv_s = inv_s.astype(np.float32)
        inv_dev = dev(inv_s)
        soff = x["skel_offsets"]
        inv_rows = np.concatenate([inv_s[soff[k]:soff[k + 1]] for k in x["skeleton_id"]])
    else:
        plan = hs.Plan(b.offsets, b.parents, autotune=True)
        inv_rows = inverse_binds(b)
        inv_dev = dev(inv_rows)
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    _, S = hs.hs_scan_forward(plan, clips=lib, clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]),
                              time=dev(x["time"]), weight=dev(x["weight"]), want_global=False, inv_bind=inv_dev)
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    chars = sample_chars(b, 24, 41)
    ids = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in chars])
    off = np.concatenate([[0], np.cumsum(np.diff(b.offsets)[chars])]).astype(np.int64)
    qr, tr = oracle.pose_sample(off, x["key_quat"], x["key_trans"], x["clip_a"][chars], x["clip_b"][chars],
                                x["time"][chars], x["weight"][chars], x["fps"])
    Gr = oracle.forward(off, b.parents[ids], qr, tr, None)
    lam = oracle.path_length(off, b.parents[ids], Gr, tr)
    check_skin(S[ids], Gr, inv_rows[ids], lam, f"{name} autotuned")


def test_differentiable_step_autotuned():
    """Forward and end-effector adjoint in one launch (hs_effector_step) on
    1024 x 512 joints, the plan as the benchmark builds it, against the
    oracle's forward and reverse mode of the same loss."""
    b = wl.differentiable()
    plan = hs.Plan(b.offsets, b.parents, autotune=True)
    assert plan.info["adjoint_blocks_per_wave"] in (1, 2)
    eff = b.extra["effectors"]
    Grest = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
    y = (Grest[eff, :3, 3] + b.extra["target_offsets"]).astype(np.float32)
    E = hs.Effectors(plan, eff)
    assert E.sparse
    G = torch.empty((b.num_joints, 4, 4), device=DEV)
    gq, gt, _ = hs.hs_effector_step(plan, E, dev(b.quat), dev(b.trans), dev(b.scale), dev(y), global_out=G,
                                    want_scale=False)
    torch.cuda.synchronize()
    G, gq, gt = G.cpu().numpy(), gq.cpu().numpy(), gt.cpu().numpy()
    chars = sample_chars(b, 12, 42)
    check_forward_sample(G, b, chars, "differentiable autotuned")
    off, par, q, t, s, ids = sub_batch(b, chars)
    eff_set = set(eff.tolist())
    local = np.array([k for k, g in enumerate(ids) if int(g) in eff_set])
    rows = np.array([int(np.nonzero(eff == ids[k])[0][0]) for k in local])
    Gr = oracle.forward(off, par, q, t, s)
    W = np.zeros((ids.size, 4, 4))
    W[local, :3, 3] = 2.0 * (Gr[local, :3, 3] - y[rows].astype(np.float64))
    rq, rt, _ = oracle.backward(off, par, q, t, s, W)
    for name, g, r in (("quat", gq[ids], rq), ("trans", gt[ids], rt)):
        for c in range(off.size - 1):
            sl = slice(off[c], off[c + 1])
            bound = 1e-4 * max(1.0, float(np.abs(r[sl]).max()))
            err = float(np.abs(g[sl] - r[sl]).max())
            assert err <= bound, f"differentiable autotuned: {name} grad of character {chars[c]}: {err:.3e}"

"""The forward's work-queue schedule (HS_SCHED_QUEUE): every tile in one
persistent launch, anchors' transforms in LDS.

Parity against the FP64 oracle on every workload shape (forests, stars,
empty characters, chains crossing many blocks, the fused sampler and skin,
checkpoints), the launch shapes the autotuner can pick, bitwise agreement
with the size-class launches where both cut the same tiles, and repeated
launches and graph replays (every launch covers every tile exactly once).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

from parity import check_global, check_skin, inverse_binds, reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def forward(b, inv=None, **plan_kw):
    plan = hs.Plan(b.offsets, b.parents, **plan_kw)
    G, S = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale),
                              inv_bind=None if inv is None else dev(inv))
    torch.cuda.synchronize()
    return plan, G.cpu().numpy(), None if S is None else S.cpu().numpy()


@pytest.mark.parametrize("shape", [dict(), dict(tile_joints=1024), dict(tile_joints=3072, waves_per_tile=16),
                                   dict(tile_joints=512, waves_per_tile=4), dict(grid_tiles=1)])
def test_heterogeneous_reduced_queue(shape):
    b = wl.heterogeneous(num_characters=300, chain_fraction=0.02)
    plan, G, _ = forward(b, schedule=hs.HS_SCHED_QUEUE, **shape)
    info = plan.info
    assert info["schedule"] == hs.HS_SCHED_QUEUE
    assert info["grid"] <= info["num_tiles"]
    Gr, lam, _ = reference(b)
    check_global(G, Gr, lam, f"heterogeneous queue {shape}")


@pytest.mark.parametrize("grid_tiles", [0, 64])
def test_heterogeneous_full_size_one_launch(grid_tiles):
    """One workgroup per tile (the default), and the resident workgroups
    (at most grid_tiles per CU) looping over the heaviest-first list."""
    b = wl.heterogeneous()
    plan, G, _ = forward(b, grid_tiles=grid_tiles)
    info = plan.info
    assert info["schedule"] == hs.HS_SCHED_QUEUE and info["multipass_joints"] == 0
    if grid_tiles == 0:
        assert info["grid"] == info["num_tiles"]
    else:
        assert info["grid"] < info["num_tiles"]  # persistent workgroups loop over the queue
    rng = np.random.default_rng(11)
    n = np.diff(b.offsets)
    chains = np.nonzero(b.extra["is_chain"])[0]
    chars = np.unique(np.concatenate([rng.choice(b.num_characters, 40, replace=False), chains[:8],
                                      [int(np.argmax(n)), int(np.argmin(n)), 0, b.num_characters - 1]]))
    Gr, lam, ids = reference(b, chars=chars)
    check_global(G[ids], Gr, lam, f"heterogeneous full, one launch, grid_tiles {grid_tiles} (sampled)")


def test_deep_forward_queue_bitwise_equals_size_classes():
    # one 1024-joint character per tile under both schedules: the same
    # blocks, the same compositions in the same order
    b = wl.deep_forward(num_characters=64)
    pq, Gq, _ = forward(b, schedule=hs.HS_SCHED_QUEUE, tile_joints=1024)
    pc, Gc, _ = forward(b, schedule=hs.HS_SCHED_CLASSES, tile_joints=1024)
    assert pq.info["schedule"] == hs.HS_SCHED_QUEUE and pc.info["schedule"] == hs.HS_SCHED_CLASSES
    assert np.array_equal(Gq, Gc)
    Gr, lam, _ = reference(b)
    check_global(Gq, Gr, lam, "deep_forward queue")


def test_plain_scan_queue_with_fused_skin_and_skin_only():
    b = wl.plain_scan()
    inv = inverse_binds(b)
    plan, G, S = forward(b, inv, schedule=hs.HS_SCHED_QUEUE)
    Gr, lam, _ = reference(b)
    check_global(G, Gr, lam, "plain_scan queue")
    check_skin(S, Gr, inv, lam, "plain_scan queue skin")
    _, S2 = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale), inv_bind=dev(inv), want_global=False)
    torch.cuda.synchronize()
    assert np.array_equal(S2.cpu().numpy(), S)


def test_star_forest_chains_and_empty_characters_queue():
    star = np.zeros(1500, np.int32)
    star[0] = -1
    forest = np.array([-1, 0, -1, 2, -1, 4, 4, 0, -1, 8] * 40, np.int32)
    forest = np.where(forest >= 0, forest + np.repeat(np.arange(40) * 10, 10), -1).astype(np.int32)
    # every joint a child of the joint 64 places earlier where possible:
    # each block's joints hang off the previous block (64 anchors per block)
    comb = np.array([-1 if j < 64 else j - 64 for j in range(1500)], np.int32)
    chain = np.arange(-1, 2999, dtype=np.int32)
    parts = [star, np.zeros(0, np.int32), forest, np.array([-1], np.int32), comb, np.zeros(0, np.int32), chain]
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    par = np.concatenate(parts)
    rng = np.random.default_rng(3)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.1)
    # non-uniform scale except on the long chain (a product of 3000 random
    # scales leaves fp32's range)
    s = rng.uniform(0.8, 1.25, s.shape).astype(np.float32)
    s[off[-2]:] = 1.0
    b = wl.Batch("mixed", off, par, q, t, s, q, t, s)
    Gr, lam, _ = reference(b)
    for shape in (dict(), dict(tile_joints=3072, waves_per_tile=16), dict(tile_joints=64, waves_per_tile=1),
                  dict(tile_joints=2048, waves_per_tile=2)):
        plan, G, _ = forward(b, schedule=hs.HS_SCHED_QUEUE, **shape)
        assert plan.info["schedule"] == hs.HS_SCHED_QUEUE
        check_global(G, Gr, lam, f"mixed queue {shape}")
    assert plan.info["multipass_joints"] > 0  # the 3000-joint chain beyond the 2048-joint tiles


def test_fused_sample_and_checkpoints_queue():
    b = wl.fused_sample(num_characters=300)
    x = b.extra
    plan = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE)
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    inv = inverse_binds(b)
    G, S = hs.hs_scan_forward(plan, clips=lib, clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]),
                              time=dev(x["time"]), weight=dev(x["weight"]), inv_bind=dev(inv))
    q, t = oracle.pose_sample(b.offsets, x["key_quat"], x["key_trans"], x["clip_a"], x["clip_b"], x["time"],
                              x["weight"], fps=x["fps"])
    Gr, lam, _ = reference(b, quat=q, trans=t, scale=np.ones_like(t))
    torch.cuda.synchronize()
    check_global(G.cpu().numpy(), Gr, lam, "fused sample queue")
    check_skin(S.cpu().numpy(), Gr, inv, lam, "fused sample queue skin")
    # checkpoints every 4 levels from the same launch
    d = wl.differentiable(num_characters=8)
    dp = hs.Plan(d.offsets, d.parents, schedule=hs.HS_SCHED_QUEUE)
    ck = torch.full((d.num_joints, 12), float("nan"), device=DEV)
    Gd, _ = hs.hs_scan_forward(dp, dev(d.quat), dev(d.trans), dev(d.scale), ckpt_out=ck, ckpt_k=4)
    torch.cuda.synchronize()
    Gd, ck = Gd.cpu().numpy(), ck.cpu().numpy()
    lv = np.concatenate([wl.levels_of(d.parents[d.offsets[c]:d.offsets[c + 1]]) for c in range(d.num_characters)])
    rows = lv % 4 == 0
    assert np.array_equal(ck[rows], Gd[rows, :3, :].reshape(-1, 12))


def test_repeated_launches_and_graph_replays_cover_every_tile():
    b = wl.heterogeneous(num_characters=400, seed=9)
    plan = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE, tile_joints=1024, grid_tiles=1)
    assert plan.info["grid"] <= plan.info["num_tiles"]
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G0, _ = hs.hs_scan_forward(plan, q, t, s)
    torch.cuda.synchronize()
    first = G0.cpu().numpy()
    Gr, lam, _ = reference(b)
    check_global(first, Gr, lam, "queue first launch")
    out = torch.empty_like(G0)
    for k in range(5):  # every launch takes every tile exactly once
        out.fill_(float("nan"))
        hs.hs_scan_forward(plan, q, t, s, global_out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), first), f"direct launch {k}"
    gout = torch.empty_like(G0)
    g = hs.ForwardGraph(plan, q, t, s, global_out=gout)
    for k in range(4):
        gout.fill_(float("nan"))  # eager work between the replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(gout.cpu().numpy(), first), f"graph replay {k}"
    rc, bits, _ = plan.status()
    assert rc == hs.HS_OK and bits == 0


def test_queue_validate_flag_gates_the_launch():
    b = wl.heterogeneous(num_characters=50, seed=4)
    plan = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G, _ = hs.hs_scan_forward(plan, q, t, s, validate=True)
    torch.cuda.synchronize()
    assert plan.status()[0] == hs.HS_OK
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "queue validated")
    plan.debug_break_parent(5)
    out = torch.full_like(G, float("nan"))
    hs.hs_scan_forward(plan, q, t, s, global_out=out, validate=True)
    rc, bits, joint = plan.status(clear=True)
    assert rc == hs.HS_ERR_DEVICE and bits & hs.HS_DEV_TOPOLOGY and joint == 5
    assert bool(torch.isnan(out).all())  # nothing launched past the check
    # a fresh plan of the same batch gives the validated call's result
    plan2 = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE)
    G2, _ = hs.hs_scan_forward(plan2, q, t, s)
    torch.cuda.synchronize()
    assert np.array_equal(G2.cpu().numpy(), G.cpu().numpy())


def test_queue_option_errors():
    b = wl.deep_forward(num_characters=2)
    with pytest.raises(hs.HSError) as ei:
        hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_QUEUE, chain_units=True)
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HSError) as ei:
        hs.Plan(b.offsets, b.parents, schedule=7)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    plan = hs.Plan(b.offsets, b.parents, chain_units=True)  # AUTO: the size classes
    assert plan.info["schedule"] == hs.HS_SCHED_CLASSES

"""GPU parity of the end-effector adjoint (hs_effectors_create,
hs_effector_backward, and hs_effector_step, which runs the forward scan in
the same launch) against the FP64 oracle.

The reference is the oracle's alone: its seed 2 (b_e - y_e) comes from the
FP64 forward of the same poses, so an error of the GPU forward (whose G
the call's seed is formed from) shows in the comparison too.  Tolerance as for
hs_scan_backward: per character, max |grad_gpu - grad_fp64| <= 1e-4 *
max(1, max |grad_fp64|) for each gradient array.  Against the dense route
(hs_effector_loss_grad + hs_scan_backward) on the same inputs the only
difference is the order of the colliding pushes, held to the same bound.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl
from parity import check_global, reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check(offsets, got, ref, what):
    for name, g, r in zip(("quat", "trans", "scale"), got, ref):
        if g is None:
            continue
        g = np.asarray(g, np.float64)
        for c in range(offsets.size - 1):
            sl = slice(offsets[c], offsets[c + 1])
            if sl.start == sl.stop:
                continue
            bound = TOL * max(1.0, float(np.abs(r[sl]).max()))
            err = float(np.abs(g[sl] - r[sl]).max())
            assert err <= bound, f"{what}: {name} grad of character {c}: {err:.3e} > {bound:.3e}"


def seed(b, eff, y):
    """The dense dLoss/dG of the loss, from the FP64 oracle's forward."""
    G = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
    W = np.zeros(G.shape)
    W[eff, :3, 3] = 2.0 * (G[eff, :3, 3] - np.asarray(y, np.float64))
    return W


def run(b, eff, y, expect_sparse=None, want_scale=True, **plan_kw):
    """Forward on the GPU, then hs_effector_backward; returns the GPU G,
    the gradients and whether the set was sparse."""
    plan = hs.Plan(b.offsets, b.parents, **plan_kw)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G, _ = hs.hs_scan_forward(plan, q, t, s)
    E = hs.Effectors(plan, eff)
    if expect_sparse is not None:
        assert E.sparse == expect_sparse
    got = hs.hs_effector_backward(plan, E, q, t, s, G, dev(y), want_scale=want_scale)
    torch.cuda.synchronize()
    return G.cpu().numpy(), [x.cpu().numpy() if x is not None else None for x in got], E.sparse


def oracle_grads(b, W):
    return oracle.backward(b.offsets, b.parents, b.quat, b.trans, b.scale, W)


def targets(b, eff, rng, radius=0.5):
    Grest = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
    return (Grest[eff, :3, 3] + wl.ball_offsets(rng, len(eff), radius)).astype(np.float32)


# the adjoint kernels; the two-level one with one and with two 64-joint
# blocks per wave
ADJ = [dict(adjoint=hs.HS_ADJ_ROUNDS),
       dict(adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=1),
       dict(adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=2)]


@pytest.mark.parametrize("adj", ADJ)
@pytest.mark.parametrize("shape", [dict(), dict(tile_joints=1024, waves_per_tile=4), dict(tile_joints=512)])
def test_effector_loss_matches_oracle(shape, adj):
    b = wl.differentiable(num_characters=12)
    eff = b.extra["effectors"]
    y = targets(b, eff, np.random.default_rng(20))
    G, got, _ = run(b, eff, y, expect_sparse=True, **adj, **shape)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), f"effector adjoint {shape}")


@pytest.mark.parametrize("adj", ADJ)
def test_ids_in_any_order_with_their_targets(adj):
    """Ids given unsorted, targets in the same order: each target stays with
    its joint.  Roots, the first and last joint of a character and a joint
    of every character, in a batch of mixed small characters."""
    b = wl.heterogeneous(num_characters=40, lo=32, hi=1000)
    rng = np.random.default_rng(21)
    off = b.offsets
    eff = set()
    for c in range(off.size - 1):
        if off[c + 1] > off[c]:
            eff.update({int(off[c]), int(off[c + 1] - 1), int(rng.integers(off[c], off[c + 1]))})
    eff = np.array(sorted(eff), np.int64)
    rng.shuffle(eff)
    y = rng.standard_normal((eff.size, 3)).astype(np.float32)
    G, got, _ = run(b, eff, y, expect_sparse=True, **adj)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), f"unsorted ids adj {adj}")


def test_no_effectors_gives_zero_gradients():
    b = wl.differentiable(num_characters=3)
    G, got, sparse = run(b, np.zeros(0, np.int64), np.zeros((0, 3), np.float32))
    assert sparse
    for g in got:
        assert np.all(g == 0.0)


@pytest.mark.parametrize("plan_kw", [dict(adjoint=hs.HS_ADJ_DATAFLOW), dict(strategy=hs.HS_STRATEGY_MULTIPASS)])
def test_dense_route_for_other_adjoint_kernels(plan_kw):
    b = wl.differentiable(num_characters=6)
    eff = b.extra["effectors"]
    y = targets(b, eff, np.random.default_rng(22))
    G, got, _ = run(b, eff, y, expect_sparse=False, **plan_kw)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), f"dense route {plan_kw}")


def test_dense_route_for_large_characters():
    """A 1500-joint chain (dataflow tiles) and a 3000-joint chain (multipass
    adjoint) next to small characters: the set keeps a dense seed."""
    rng = np.random.default_rng(23)
    small = wl.plain_scan(num_characters=2).parents
    parts = [np.arange(-1, 1499, dtype=np.int32), small, np.arange(-1, 2999, dtype=np.int32)]
    par = np.concatenate(parts)
    off = np.array([0, 1500, 1564, 1628, 4628], np.int64)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.1)
    b = wl.Batch("mixed", off, par, q, t, s, q, t, s)
    eff = np.array([1499, 700, 1500, 1600, 4627, 3000], np.int64)
    y = rng.standard_normal((eff.size, 3)).astype(np.float32)
    G, got, _ = run(b, eff, y, expect_sparse=False)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), "large characters")


def test_agrees_with_dense_calls_and_repeats():
    """Same inputs through hs_effector_loss_grad + hs_scan_backward; a second
    call with other targets on the same set."""
    b = wl.differentiable(num_characters=32)
    N = b.num_joints
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    eff = b.extra["effectors"]
    E = hs.Effectors(plan, eff)
    G, _ = hs.hs_scan_forward(plan, q, t, s)
    rng = np.random.default_rng(24)
    for rep in range(2):
        y = dev(targets(b, eff, rng))
        got = hs.hs_effector_backward(plan, E, q, t, s, G, y)
        gG = torch.zeros((N, 4, 4), device=DEV)
        hs.hs_effector_loss_grad(G, dev(eff.astype(np.int64)), y, gG)
        ref = hs.hs_scan_backward(plan, q, t, s, gG)
        torch.cuda.synchronize()
        for x, r in zip(got, ref):
            bound = TOL * max(1.0, float(r.abs().max()))
            assert float((x - r).abs().max()) <= bound, rep


def test_captured_step_replays_match_eager():
    """Forward and effector adjoint captured in one HIP graph: every replay,
    with eager input changes between replays, matches the eager calls."""
    b = wl.differentiable(num_characters=64)
    N = b.num_joints
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    E = hs.Effectors(plan, b.extra["effectors"])
    tgt = dev(np.random.default_rng(25).standard_normal((E.num_effectors, 3)).astype(np.float32))
    G = torch.empty((N, 4, 4), device=DEV)
    gq = torch.empty((N, 4), device=DEV)
    gt = torch.empty((N, 3), device=DEV)

    def step(G, gq, gt):
        hs.hs_scan_forward(plan, q, t, s, global_out=G)
        hs.hs_effector_backward(plan, E, q, t, s, G, tgt, want_scale=False, grad_quat=gq, grad_trans=gt)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(G, gq, gt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(G, gq, gt)
    rng = np.random.default_rng(26)
    for rep in range(4):
        q.copy_(dev(wl.random_quats(rng, N, 0.3)))
        tgt.copy_(dev(rng.standard_normal((E.num_effectors, 3)).astype(np.float32)))
        gq.zero_()
        g.replay()
        torch.cuda.synchronize()
        G2, gq2, gt2 = torch.empty_like(G), torch.empty_like(gq), torch.empty_like(gt)
        step(G2, gq2, gt2)
        torch.cuda.synchronize()
        assert torch.equal(G, G2), rep
        for x, y in ((gq, gq2), (gt, gt2)):
            bound = TOL * max(1.0, float(y.abs().max()))
            assert float((x - y).abs().max()) <= bound, rep


def test_errors():
    b = wl.differentiable(num_characters=2)
    plan = hs.Plan(b.offsets, b.parents)
    other = hs.Plan(b.offsets, b.parents)
    with pytest.raises(hs.HSError):
        hs.Effectors(plan, [3, 5, 3])  # listed twice
    with pytest.raises(hs.HSError):
        hs.Effectors(plan, [b.num_joints])  # outside the batch
    with pytest.raises(hs.HSError):
        hs.Effectors(plan, [-1])
    E = hs.Effectors(plan, [1, 2])
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G, _ = hs.hs_scan_forward(plan, q, t, s)
    y = torch.zeros((2, 3), device=DEV)
    with pytest.raises(hs.HSError):
        hs.hs_effector_backward(other, E, q, t, s, G, y)  # set of another plan
    gq = torch.empty((b.num_joints, 4), device=DEV)
    with pytest.raises(hs.HSError):
        # an output overlapping an input
        hs.hs_effector_backward(plan, E, q, t, s, G, y, grad_quat=q)
    del gq


# ---------------------------------------------------------------------------
# hs_effector_step: the forward scan inside each adjoint tile, then the
# adjoint seeded from it.  Its G (global_out) is held to the forward's
# tolerance against the oracle, and its gradients to the oracle's reverse
# mode fed the seed made from that G.
# ---------------------------------------------------------------------------
def run_step(b, eff, y, want_global=True, **plan_kw):
    plan = hs.Plan(b.offsets, b.parents, **plan_kw)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    E = hs.Effectors(plan, eff)
    assert E.sparse
    G = torch.empty((b.num_joints, 4, 4), device=DEV) if want_global else None
    got = hs.hs_effector_step(plan, E, q, t, s, dev(y), global_out=G)
    torch.cuda.synchronize()
    got = [x.cpu().numpy() for x in got]
    if want_global:
        Gr, lam, _ = reference(b)
        check_global(G.cpu().numpy(), Gr, lam, "effector step G")
        return G.cpu().numpy(), got
    return None, got


@pytest.mark.parametrize("adj", ADJ)
@pytest.mark.parametrize("shape", [dict(), dict(tile_joints=1024, waves_per_tile=4), dict(tile_joints=512)])
def test_fused_step_matches_oracle(shape, adj):
    b = wl.differentiable(num_characters=12)
    eff = b.extra["effectors"]
    y = targets(b, eff, np.random.default_rng(30))
    G, got = run_step(b, eff, y, **adj, **shape)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), f"effector step {shape}")


@pytest.mark.parametrize("adj", ADJ)
def test_fused_step_mixed_small_characters_and_unsorted_ids(adj):
    b = wl.heterogeneous(num_characters=40, lo=32, hi=1000)
    rng = np.random.default_rng(31)
    off = b.offsets
    eff = set()
    for c in range(off.size - 1):
        if off[c + 1] > off[c]:
            eff.update({int(off[c]), int(off[c + 1] - 1), int(rng.integers(off[c], off[c + 1]))})
    eff = np.array(sorted(eff), np.int64)
    rng.shuffle(eff)
    y = rng.standard_normal((eff.size, 3)).astype(np.float32)
    G, got = run_step(b, eff, y, **adj)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), f"effector step, mixed characters adj {adj}")


def test_fused_step_without_global_agrees_with_two_calls():
    b = wl.differentiable(num_characters=16)
    eff = b.extra["effectors"]
    y = targets(b, eff, np.random.default_rng(32))
    _, got = run_step(b, eff, y, want_global=False)
    _, two, _ = run(b, eff, y)
    for name, x, r in zip(("quat", "trans", "scale"), got, two):
        bound = TOL * max(1.0, float(np.abs(r).max()))
        assert float(np.abs(x - r).max()) <= bound, name


def test_fused_step_needs_a_sparse_set():
    b = wl.differentiable(num_characters=2)
    plan = hs.Plan(b.offsets, b.parents, adjoint=hs.HS_ADJ_DATAFLOW)
    E = hs.Effectors(plan, b.extra["effectors"])
    assert not E.sparse
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    with pytest.raises(hs.HSError) as ei:
        hs.hs_effector_step(plan, E, q, t, s, torch.zeros((E.num_effectors, 3), device=DEV))
    assert ei.value.status == 3  # HS_ERR_UNSUPPORTED


def test_fused_step_captured_replays_match_eager():
    b = wl.differentiable(num_characters=64)
    N = b.num_joints
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    E = hs.Effectors(plan, b.extra["effectors"])
    tgt = dev(np.random.default_rng(33).standard_normal((E.num_effectors, 3)).astype(np.float32))
    G = torch.empty((N, 4, 4), device=DEV)
    gq = torch.empty((N, 4), device=DEV)
    gt = torch.empty((N, 3), device=DEV)

    def step(G, gq, gt):
        hs.hs_effector_step(plan, E, q, t, s, tgt, global_out=G, want_scale=False, grad_quat=gq, grad_trans=gt)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(G, gq, gt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(G, gq, gt)
    rng = np.random.default_rng(34)
    for rep in range(4):
        q.copy_(dev(wl.random_quats(rng, N, 0.3)))
        tgt.copy_(dev(rng.standard_normal((E.num_effectors, 3)).astype(np.float32)))
        gq.zero_()
        g.replay()
        torch.cuda.synchronize()
        G2, gq2, gt2 = torch.empty_like(G), torch.empty_like(gq), torch.empty_like(gt)
        step(G2, gq2, gt2)
        torch.cuda.synchronize()
        assert torch.equal(G, G2), rep
        for x, y in ((gq, gq2), (gt, gt2)):
            bound = TOL * max(1.0, float(y.abs().max()))
            assert float((x - y).abs().max()) <= bound, rep


def test_fused_step_without_effectors_writes_g_and_zero_gradients():
    b = wl.differentiable(num_characters=3)
    G, got = run_step(b, np.zeros(0, np.int64), np.zeros((0, 3), np.float32))
    for g in got:
        assert np.all(g == 0.0)


def test_fused_step_on_single_joint_and_empty_characters():
    """Characters of 0, 1, 2 and 64 joints next to a 512-joint one, with
    effectors on roots and leaves: the tiles' forward and seeds at the
    smallest sizes."""
    rng = np.random.default_rng(35)
    big = wl.differentiable(num_characters=1)
    chars = [np.zeros(0, np.int32), np.array([-1], np.int32), np.array([-1, 0], np.int32),
             wl.plain_scan(num_characters=1).parents, big.parents]
    par = np.concatenate(chars)
    off = np.concatenate([[0], np.cumsum([c.size for c in chars])]).astype(np.int64)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.3)
    b = wl.Batch("small", off, par, q, t, s, q, t, s)
    eff = np.array([0, 1, 2, 3, 66, off[4] + 5, off[4] + 300, par.size - 1], np.int64)
    y = rng.standard_normal((eff.size, 3)).astype(np.float32)
    G, got = run_step(b, eff, y)
    check(b.offsets, got, oracle_grads(b, seed(b, eff, y)), "small characters")

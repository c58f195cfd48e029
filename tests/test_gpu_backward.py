"""GPU parity of the adjoint kernel (hs_scan_backward) and of the autograd
wrapper against the FP64 oracle's reverse-mode gradients.

Tolerance: per character, max |grad_gpu - grad_fp64| <= 1e-4 * max(1, max
|grad_fp64|) for each of the quaternion, translation and scale gradients.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl
from paper_2505_06703_amd.autograd import hierarchy_scan

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check_grads(offsets, got, ref, what):
    for name, g, r in zip(("quat", "trans", "scale"), got, ref):
        if g is None:
            continue
        g = np.asarray(g, np.float64)
        for c in range(offsets.size - 1):
            sl = slice(offsets[c], offsets[c + 1])
            if sl.start == sl.stop:
                continue
            scale = max(1.0, float(np.abs(r[sl]).max()))
            err = float(np.abs(g[sl] - r[sl]).max())
            assert err <= TOL * scale, f"{what}: {name} grad of character {c}: {err:.3e} > {TOL * scale:.3e}"


def effector_grad(batch, G_ref):
    """dLoss/dG for the sum over end effectors of |b_e - y_e|^2, targets at
    the rest-pose positions plus seeded offsets within 0.5 units."""
    Grest = oracle.forward(batch.offsets, batch.parents, batch.rest_quat, batch.rest_trans, batch.rest_scale)
    eff = batch.extra["effectors"]
    y = Grest[eff, :3, 3] + batch.extra["target_offsets"]
    W = np.zeros((batch.num_joints, 4, 4))
    W[eff, :3, 3] = 2.0 * (G_ref[eff, :3, 3] - y)
    return W.astype(np.float32)


def run(batch, W, ckpt_k=0, want_scale=True, **plan_kw):
    plan = hs.Plan(batch.offsets, batch.parents, **plan_kw)
    q, t, s = dev(batch.quat), dev(batch.trans), dev(batch.scale)
    ckpt = None
    if ckpt_k:
        ckpt = torch.empty((batch.num_joints, 12), device=DEV)
        hs.hs_scan_forward(plan, q, t, s, ckpt_out=ckpt, ckpt_k=ckpt_k)
    gq, gt, gs = hs.hs_scan_backward(plan, q, t, s, dev(W), ckpt=ckpt, ckpt_k=ckpt_k, want_scale=want_scale)
    torch.cuda.synchronize()
    return [x.cpu().numpy() if x is not None else None for x in (gq, gt, gs)]


def oracle_grads(batch, W):
    return oracle.backward(batch.offsets, batch.parents, batch.quat, batch.trans, batch.scale, W)


# the adjoint kernels; the two-level one with one and with two 64-joint
# blocks per wave
ADJ = [dict(adjoint=hs.HS_ADJ_ROUNDS), dict(adjoint=hs.HS_ADJ_DATAFLOW),
       dict(adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=1),
       dict(adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=2)]


@pytest.mark.parametrize("adj", ADJ)
@pytest.mark.parametrize("shape", [dict(), dict(tile_joints=1024, waves_per_tile=4), dict(tile_joints=512)])
def test_differentiable_effector_loss(shape, adj):
    b = wl.differentiable(num_characters=12)
    G = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
    W = effector_grad(b, G)
    check_grads(b.offsets, run(b, W, **adj, **shape), oracle_grads(b, W), f"differentiable {shape} adj {adj}")


@pytest.mark.parametrize("k", [1, 3, 8])
def test_level_checkpoint_mode(k):
    b = wl.differentiable(num_characters=6)
    G = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
    W = effector_grad(b, G)
    check_grads(b.offsets, run(b, W, ckpt_k=k), oracle_grads(b, W), f"ckpt k={k}")


@pytest.mark.parametrize("adj", ADJ)
def test_dense_random_gradient_with_scale_and_forests(adj):
    rng = np.random.default_rng(5)
    b = wl.heterogeneous(num_characters=40, hi=1500, chain_fraction=0.05)
    b.scale = rng.uniform(0.8, 1.25, b.scale.shape).astype(np.float32)
    W = rng.standard_normal((b.num_joints, 4, 4)).astype(np.float32)
    check_grads(b.offsets, run(b, W, **adj), oracle_grads(b, W), "dense random")
    check_grads(b.offsets, run(b, W, ckpt_k=5, **adj), oracle_grads(b, W), "dense random ckpt")


@pytest.mark.parametrize("adj", ADJ)
def test_plain_scan_trees_and_star(adj):
    rng = np.random.default_rng(6)
    star = np.zeros(700, np.int32)
    star[0] = -1
    b0 = wl.plain_scan(num_characters=8)
    par = np.concatenate([b0.parents, star, np.zeros(0, np.int32), np.array([-1, -1, 1], np.int32)])
    off = np.concatenate([b0.offsets, [b0.offsets[-1] + 700, b0.offsets[-1] + 700, b0.offsets[-1] + 703]])
    q, t, s = wl.random_pose(rng, par.size)
    b = wl.Batch("mix", off.astype(np.int64), par, q, t, s, q, t, s)
    W = rng.standard_normal((par.size, 4, 4)).astype(np.float32)
    check_grads(b.offsets, run(b, W, **adj), oracle_grads(b, W), "trees+star")
    got = run(b, W, want_scale=False, **adj)
    assert got[2] is None


@pytest.mark.parametrize("adj", ADJ)
@pytest.mark.parametrize("n", [1, 64, 65, 1000, 1024, 1025, 1664])
def test_chains(n, adj):
    """Chains up to 1024 joints take the chosen adjoint kernel, longer ones
    (to 1664) the dataflow tiles, in both memory modes."""
    rng = np.random.default_rng(n)
    par = np.arange(-1, n - 1, dtype=np.int32)
    q, t, s = wl.random_pose(rng, n, max_angle=0.1)
    b = wl.Batch("chain", np.array([0, n], np.int64), par, q, t, s, q, t, s)
    W = np.zeros((n, 4, 4), np.float32)
    W[-1, :3, 3] = rng.standard_normal(3)
    W[n // 2, :3, :3] = rng.standard_normal((3, 3))
    ref = oracle_grads(b, W)
    check_grads(b.offsets, run(b, W, **adj), ref, f"chain {n}")
    check_grads(b.offsets, run(b, W, ckpt_k=4, **adj), ref, f"chain {n} ckpt 4")


@pytest.mark.parametrize("adj", ADJ)
@pytest.mark.parametrize("n", [1024, 1025])
def test_stars_and_brooms_collide_on_one_target(n, adj):
    """Every joint of a star pushes to the root in one round; a broom (a
    chain whose last joint fans out) sends ever more joints to one target as
    the jump distance grows."""
    rng = np.random.default_rng(n + 1)
    star = np.zeros(n, np.int32)
    star[0] = -1
    broom = np.arange(-1, n - 1, dtype=np.int32)
    broom[300:] = 299
    broom[600:] = np.arange(300, n - 300) - 1 + 300
    par = np.concatenate([star, broom])
    off = np.array([0, n, 2 * n], np.int64)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.2)
    b = wl.Batch("star", off, par, q, t, s, q, t, s)
    W = rng.standard_normal((par.size, 4, 4)).astype(np.float32)
    check_grads(b.offsets, run(b, W, **adj), oracle_grads(b, W), f"star/broom {n}")


def test_large_forward_tiles_use_smaller_adjoint_tiles():
    b = wl.heterogeneous(num_characters=30, lo=1200, hi=1600)
    rng = np.random.default_rng(8)
    W = rng.standard_normal((b.num_joints, 4, 4)).astype(np.float32)
    check_grads(b.offsets, run(b, W, tile_joints=3072), oracle_grads(b, W), "3072-joint forward tiles")


@pytest.mark.parametrize("shape", [dict(), dict(strategy=hs.HS_STRATEGY_MULTIPASS)])
def test_multipass_adjoint_for_large_characters(shape):
    """Characters beyond the adjoint tile (a 3000-joint chain, a 5000-joint
    random tree) next to small ones go through the multipass adjoint."""
    rng = np.random.default_rng(1)
    chain = np.arange(-1, 2999, dtype=np.int32)
    tree = np.empty(5000, np.int32)
    tree[0] = -1
    for j in range(1, 5000):
        tree[j] = j - 1 if rng.uniform() < 0.8 else rng.integers(0, j)
    small = wl.plain_scan(num_characters=3).parents
    parts = [chain, small, tree]
    par = np.concatenate(parts)
    off = np.array([0, 3000, 3000 + 64, 3000 + 128, 3000 + 192, 3000 + 192 + 5000], np.int64)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.1)
    s = rng.uniform(0.9, 1.1, s.shape).astype(np.float32)
    b = wl.Batch("big", off, par, q, t, s, q, t, s)
    W = rng.standard_normal((par.size, 4, 4)).astype(np.float32) * 0.1
    check_grads(b.offsets, run(b, W, **shape), oracle_grads(b, W), f"multipass adjoint {shape}")


def test_autograd_matches_oracle_in_both_modes():
    b = wl.differentiable(num_characters=4)
    G64 = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
    Grest = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
    eff = b.extra["effectors"]
    y = dev((Grest[eff, :3, 3] + b.extra["target_offsets"]).astype(np.float32))
    plan = hs.Plan(b.offsets, b.parents)
    for k in (0, 4):
        q = dev(b.quat).requires_grad_(True)
        t = dev(b.trans).requires_grad_(True)
        G = hierarchy_scan(plan, q, t, None, ckpt_k=k)
        loss = ((G[torch.as_tensor(eff, device=DEV), :3, 3] - y) ** 2).sum()
        loss.backward()
        # the oracle's gradient of the same loss (its own FP64 forward)
        W = np.zeros((b.num_joints, 4, 4))
        Gg = G.detach().cpu().numpy().astype(np.float64)
        W[eff, :3, 3] = 2.0 * (G64[eff, :3, 3] - y.cpu().numpy())
        ref = oracle.backward(b.offsets, b.parents, b.quat, b.trans, None, W)
        check_grads(b.offsets, [q.grad.cpu().numpy(), t.grad.cpu().numpy(), None], ref, f"autograd k={k}")
        np.testing.assert_allclose(Gg[eff, :3, 3], G64[eff, :3, 3], atol=1e-4 * 30)


def test_multipass_adjoint_comb_with_shared_anchors():
    """A 20 000-joint spine with a 150-joint side chain hung every 300 joints,
    plus fingers of 3 joints every 50: blocks with several heads, heads of
    different blocks on one anchor, anchor chains across hundreds of blocks
    (the anchor-level reverse scan and its fan-in)."""
    rng = np.random.default_rng(11)
    par = list(range(-1, 19999))
    for base in range(300, 20000, 300):
        start = len(par)
        par.append(base)
        par.extend(range(start, start + 149))
    for base in range(50, 20000, 50):
        start = len(par)
        par.append(base)
        par.extend(range(start, start + 2))
    par = np.array(par, np.int32)
    n = par.size
    q, t, s = wl.random_pose(rng, n, max_angle=0.02)
    b = wl.Batch("comb", np.array([0, n], np.int64), par, q, t, s, q, t, s)
    W = np.zeros((n, 4, 4), np.float32)
    idx = rng.choice(n, 400, replace=False)
    W[idx, :3, :] = rng.standard_normal((400, 3, 4)).astype(np.float32) * 0.1
    got = run(b, W)
    ref = oracle_grads(b, W)
    for name, g, r in zip(("quat", "trans", "scale"), got, ref):
        g = np.asarray(g, np.float64)
        tol = TOL * max(1.0, float(np.abs(r).max()))
        err = float(np.abs(g - r).max())
        assert err <= tol, f"{name}: {err:.3e} > {tol:.3e}"


@pytest.mark.parametrize("lengths", [[100_000], [30_000] * 4, [30_000, 5_000, 20_000, 3_000]])
def test_multipass_adjoint_anchor_rounds(lengths):
    """The anchors' reverse rounds: a 100 000-joint chain has more anchors
    than one workgroup holds, so its rounds run over the whole anchor array;
    four 30 000-joint chains run them per segment of whole characters in
    one workgroup's LDS (two characters a segment); chains of four lengths
    share one segment, their anchors' pointers running out after different
    rounds."""
    rng = np.random.default_rng(len(lengths))
    par = np.concatenate([np.arange(-1, n - 1, dtype=np.int32) for n in lengths])
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    n = par.size
    q, t, s = wl.random_pose(rng, n, max_angle=0.02)
    b = wl.Batch("chains", off, par, q, t, s, q, t, s)
    plan = hs.Plan(b.offsets, b.parents)
    assert plan.info["multipass_joints"] == n
    W = np.zeros((n, 4, 4), np.float32)
    idx = rng.choice(n, 400, replace=False)
    W[idx, :3, :] = rng.standard_normal((400, 3, 4)).astype(np.float32) * 0.1
    got = run(b, W)
    ref = oracle_grads(b, W)
    for name, g, r in zip(("quat", "trans", "scale"), got, ref):
        g = np.asarray(g, np.float64)
        for c in range(len(lengths)):
            sl = slice(off[c], off[c + 1])
            tol = TOL * max(1.0, float(np.abs(r[sl]).max()))  # flat: measured at most half of it
            err = float(np.abs(g[sl] - r[sl]).max())
            assert err <= tol, f"{name} of character {c}: {err:.3e} > {tol:.3e}"


@pytest.mark.parametrize("adj", ADJ)
def test_more_tiles_than_resident_workgroups(adj):
    """1300 characters of 512 joints: more adjoint tiles than the device
    holds at once (workgroups dispatched as others finish)."""
    b = wl.differentiable(num_characters=1300)
    G = oracle.forward(b.offsets, b.parents, b.quat, b.trans, b.scale)
    W = effector_grad(b, G)
    rng = np.random.default_rng(13)
    W[:, :3, :] += 0.01 * rng.standard_normal((b.num_joints, 3, 4)).astype(np.float32)
    check_grads(b.offsets, run(b, W, **adj), oracle_grads(b, W), f"1300 characters adj {adj}")


def test_effector_loss_gradient_kernel():
    """hs_effector_loss_grad writes 2 (b_e - y_e) into column 3 of rows 0-2
    of each effector's row and nothing else; ids outside the batch are
    skipped."""
    rng = np.random.default_rng(14)
    N = 1000
    G = torch.randn((N, 4, 4), device=DEV)
    eff = np.sort(rng.choice(N, 37, replace=False)).astype(np.int64)
    tgt = rng.standard_normal((37, 3)).astype(np.float32)
    gG = torch.zeros((N, 4, 4), device=DEV)
    hs.hs_effector_loss_grad(G, dev(eff), dev(tgt), gG)
    bad = np.concatenate([eff, [-1, N, N + 5]]).astype(np.int64)
    gG2 = torch.zeros((N, 4, 4), device=DEV)
    hs.hs_effector_loss_grad(G, dev(bad), dev(np.concatenate([tgt, np.zeros((3, 3), np.float32)])), gG2)
    torch.cuda.synchronize()
    ref = np.zeros((N, 4, 4), np.float32)
    ref[eff, :3, 3] = 2.0 * (G.cpu().numpy()[eff, :3, 3] - tgt)
    np.testing.assert_array_equal(gG.cpu().numpy(), ref)
    np.testing.assert_array_equal(gG2.cpu().numpy(), ref)


def test_captured_differentiable_step_replays_match_eager():
    """Forward, loss gradient and adjoint captured in one HIP graph (as the
    benchmark runs them): every replay, with eager work and input changes
    between replays, matches the eager calls."""
    b = wl.differentiable(num_characters=64)
    N = b.num_joints
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    eff = dev(b.extra["effectors"].astype(np.int64))
    tgt = dev(np.random.default_rng(15).standard_normal((eff.shape[0], 3)).astype(np.float32))
    G = torch.empty((N, 4, 4), device=DEV)
    gG = torch.zeros((N, 4, 4), device=DEV)
    gq = torch.empty((N, 4), device=DEV)
    gt = torch.empty((N, 3), device=DEV)

    def step(G, gG, gq, gt):
        hs.hs_scan_forward(plan, q, t, s, global_out=G)
        hs.hs_effector_loss_grad(G, eff, tgt, gG)
        hs.hs_scan_backward(plan, q, t, s, gG, want_scale=False, grad_quat=gq, grad_trans=gt)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(G, gG, gq, gt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(G, gG, gq, gt)
    rng = np.random.default_rng(16)
    for rep in range(4):
        q.copy_(dev(wl.random_quats(rng, N, 0.3)))  # eager work between replays
        gq.zero_()
        g.replay()
        torch.cuda.synchronize()
        G2, gG2 = torch.empty_like(G), torch.zeros_like(gG)
        gq2, gt2 = torch.empty_like(gq), torch.empty_like(gt)
        step(G2, gG2, gq2, gt2)
        torch.cuda.synchronize()
        assert torch.equal(G, G2), rep
        # the adjoint sums colliding pushes in arrival order: equal to
        # rounding, held to the adjoint's tolerance
        for x, y in ((gq, gq2), (gt, gt2)):
            tol = TOL * max(1.0, float(y.abs().max()))
            assert float((x - y).abs().max()) <= tol, rep

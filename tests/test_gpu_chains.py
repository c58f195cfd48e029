"""The one-pass path for chain characters beyond a tile (every joint's
parent the previous joint): superblocks of 4096 joints, 16 waves of two
128-joint segments each, two consecutive joints per lane; the segments'
totals scanned in LDS and a look-back over the chain's earlier
superblocks through tagged publication words.

Parity against the FP64 oracle at the flat tolerance for chains that end
inside a segment (odd lengths: a lane holding one joint), at segment and
superblock boundaries and with one to many superblocks; next to characters
on the block path and on tiles; with clip sampling, skin and checkpoints;
repeated launches and graph replays (each call tags its publications with
a new epoch); the sampler over chain characters; and the plan's
bookkeeping."""
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


def chains_batch(lengths, seed, angle=0.1, extra=()):
    """Single chains of the given lengths, then the `extra` parent arrays;
    non-unit scale on the extras of fewer than 64 joints only."""
    rng = np.random.default_rng(seed)
    parts = [np.arange(-1, n - 1, dtype=np.int32) for n in lengths] + [np.asarray(p, np.int32) for p in extra]
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    par = np.concatenate(parts)
    q, t, s = wl.random_pose(rng, par.size, max_angle=angle)
    # non-unit scale on the small characters only: a product of thousands
    # of random scales along a deep path leaves the range that the absolute
    # rotation-block tolerance is meant for
    s = np.ones_like(s)
    for c in range(len(parts)):
        if parts[c].size < 64:
            s[off[c]:off[c + 1]] = rng.uniform(0.8, 1.25, (parts[c].size, 3))
    rq, rt, rs = wl.random_pose(rng, par.size, max_angle=angle)
    return wl.Batch("chains", off, par, q, t, s, rq, rt, rs)


# segment (128) and superblock (4096) boundaries, odd lengths, and several
# superblocks
LENGTHS = [2049, 2112, 2175, 2176, 4096, 4097, 4160, 4223, 8191, 12345, 20000]


def test_chains_of_many_lengths_one_pass():
    b = chains_batch(LENGTHS, seed=1)
    plan = hs.Plan(b.offsets, b.parents, tile_joints=2048)
    info = plan.info
    assert info["chain_joints"] == b.num_joints == info["multipass_joints"]
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "chains, one pass")


def test_chains_next_to_blocks_and_tiles():
    """Pure chains take the one-pass path, a long tree the block path, the
    small characters the tiles; all in one call."""
    rng = np.random.default_rng(7)
    tree = np.array([-1] + [int(rng.integers(max(0, j - 3), j)) for j in range(1, 3000)], np.int32)
    small = [np.array([-1, 0, 1, 1, 3], np.int32)] * 7
    b = chains_batch([3000, 40000], seed=2, extra=[tree, *small, np.arange(-1, 2499, dtype=np.int32)])
    plan = hs.Plan(b.offsets, b.parents, tile_joints=2048)
    info = plan.info
    assert info["chain_joints"] == 3000 + 40000 + 2500
    assert info["multipass_joints"] == info["chain_joints"] + 3000
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "chains + blocks + tiles")


def test_chain_skin_and_checkpoints():
    b = chains_batch([5000, 2500], seed=3)
    inv = inverse_binds(b)
    plan = hs.Plan(b.offsets, b.parents, tile_joints=2048)
    N = b.num_joints
    ck = torch.full((N, 12), float("nan"), device=DEV)
    G, S = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale), inv_bind=dev(inv), ckpt_out=ck,
                              ckpt_k=7)
    torch.cuda.synchronize()
    G, S, ck = G.cpu().numpy(), S.cpu().numpy(), ck.cpu().numpy()
    Gr, lam, _ = reference(b)
    check_global(G, Gr, lam, "chain G with skin")
    check_skin(S, Gr, inv, lam, "chain skin")
    lv = np.concatenate([np.arange(1, n + 1) for n in np.diff(b.offsets)])  # a chain's levels
    rows = lv % 7 == 0
    assert np.array_equal(ck[rows], G[rows, :3, :].reshape(-1, 12))
    _, S2 = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale), inv_bind=dev(inv),
                               want_global=False)
    torch.cuda.synchronize()
    assert np.array_equal(S2.cpu().numpy(), S)


def test_chain_launches_and_graph_replays_repeat():
    b = chains_batch([9000, 4100, 2049], seed=4)
    plan = hs.Plan(b.offsets, b.parents, tile_joints=2048)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G0, _ = hs.hs_scan_forward(plan, q, t, s)
    torch.cuda.synchronize()
    first = G0.cpu().numpy()
    Gr, lam, _ = reference(b)
    check_global(first, Gr, lam, "chains first launch")
    out = torch.empty_like(G0)
    for k in range(4):  # every call publishes under a new epoch
        out.fill_(float("nan"))
        hs.hs_scan_forward(plan, q, t, s, global_out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), first), f"launch {k}"
    gout = torch.empty_like(G0)
    g = hs.ForwardGraph(plan, q, t, s, global_out=gout)
    for k in range(4):
        gout.fill_(float("nan"))  # eager work between the replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(gout.cpu().numpy(), first), f"graph replay {k}"
    g.close()
    rc, bits, _ = plan.status()
    assert rc == hs.HS_OK and bits == 0


def test_chain_with_sampled_poses():
    """Clip sampling fused into the one-pass path (a library of 3000-joint
    clips), and hs_pose_sample over chain characters."""
    rng = np.random.default_rng(5)
    J, K, C = 3000, 4, 3
    kq = wl.random_quats(rng, 2 * K * J, 0.05).reshape(2, K, J, 4)
    kt = wl.random_offsets(rng, 2 * K * J).reshape(2, K, J, 3)
    off = np.array([0, 3000, 5500, 8000], np.int64)
    par = np.concatenate([np.arange(-1, n - 1, dtype=np.int32) for n in np.diff(off)])
    ca = np.array([0, 1, 0], np.int32)
    cb = np.array([1, 0, 1], np.int32)
    tm = rng.uniform(0, 0.1, C).astype(np.float32)
    wt = rng.uniform(0, 1, C).astype(np.float32)
    lib = hs.ClipLibrary(dev(kq), dev(kt), 30.0)
    plan = hs.Plan(off, par, tile_joints=2048)
    assert plan.info["chain_joints"] == 8000
    cp = dict(clip_a=dev(ca), clip_b=dev(cb), time=dev(tm), weight=dev(wt))
    G, _ = hs.hs_scan_forward(plan, clips=lib, **cp)
    qs, ts = hs.hs_pose_sample(plan, lib, **cp)
    torch.cuda.synchronize()
    qr, tr = oracle.pose_sample(off, kq, kt, ca, cb, tm, wt, 30.0)
    np.testing.assert_allclose(qs.cpu().numpy(), qr, rtol=0, atol=2e-6)
    np.testing.assert_allclose(ts.cpu().numpy(), tr, rtol=0, atol=2e-6)
    Gr = oracle.forward(off, par, qr, tr, None)
    lam = oracle.path_length(off, par, Gr, tr)
    check_global(G.cpu().numpy(), Gr, lam, "sampled chains")


def test_chain_wait_limit_zero_is_never_silently_wrong():
    """With a zero wait limit a look-back gives up at once when an earlier
    superblock has not published yet (whether one has depends on timing):
    the call then reports the timeout in the plan's status word; when it
    reports nothing, every look-back found what it needed and the result
    is right.  Restoring the limit restores clean calls."""
    b = chains_batch([20000, 12345, 9000], seed=5)
    plan = hs.Plan(b.offsets, b.parents, tile_joints=2048)
    assert plan.info["chain_joints"] == b.num_joints
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    Gr, lam, _ = reference(b)
    plan.set_wait_limit(0)
    for _ in range(3):
        G, _ = hs.hs_scan_forward(plan, q, t, s)
        rc, bits, _ = plan.status(clear=True)
        if rc == hs.HS_OK:
            check_global(G.cpu().numpy(), Gr, lam, "chains, zero wait limit, no timeout reported")
        else:
            assert rc == hs.HS_ERR_DEVICE and bits & hs.HS_DEV_WAIT_TIMEOUT
    plan.set_wait_limit(1 << 22)
    G, _ = hs.hs_scan_forward(plan, q, t, s)
    assert plan.status() == (hs.HS_OK, 0, -1)
    check_global(G.cpu().numpy(), Gr, lam, "chains after the wait limit is restored")

"""GPU parity of instanced plans (hs_plan_create_instanced): characters that
are copies of shared skeletons, whose parents and inverse binds the forward
tiles read per skeleton joint.

Each case is checked against the FP64 oracle on the expanded batch (every
character written out with its skeleton's parents and inverse binds), and
bitwise against an ordinary plan of that expanded batch: the tiles do the
same arithmetic in the same order, only the indexing differs.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

from parity import check_global, check_skin, reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def skeletons(rng, sizes):
    """Random skeletons (parents drawn as in the heterogeneous workload:
    mostly the previous joint, else any earlier one) and one rest pose per
    skeleton joint."""
    pars = []
    for n in sizes:
        p = np.empty(n, np.int32)
        p[0] = -1
        for j in range(1, n):
            p[j] = j - 1 if rng.uniform() < 0.7 else rng.integers(0, j)
        pars.append(p)
    soff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    spar = np.concatenate(pars).astype(np.int32)
    rq, rt, rs = wl.random_pose(rng, int(soff[-1]))
    return soff, spar, (rq, rt, rs)


def skeleton_inverse_binds(soff, spar, rest):
    """FP64 inverse of each skeleton's rest-pose globals, rounded to fp32."""
    G = oracle.forward(soff, spar, *rest)
    return np.linalg.inv(G).astype(np.float32)


def expand(soff, spar, sid):
    """The ordinary batch of the instances: offsets, parents and each joint's
    skeleton row."""
    sizes = np.diff(soff)[sid]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rows = np.concatenate([np.arange(soff[k], soff[k + 1]) for k in sid]) if sid.size else np.zeros(0, np.int64)
    return off, spar[rows], rows


def test_mixed_skeletons_match_oracle_and_expanded_plan():
    rng = np.random.default_rng(21)
    sizes = [1, 64, 65, 300, 700, 1024, 1500, 2048]
    soff, spar, rest = skeletons(rng, sizes)
    sid = rng.integers(0, len(sizes), 300).astype(np.int32)
    off, par, rows = expand(soff, spar, sid)
    N = int(off[-1])
    q, t, s = wl.random_pose(rng, N)
    s = rng.uniform(0.9, 1.1, s.shape).astype(np.float32)
    inv_s = skeleton_inverse_binds(soff, spar, rest)

    plan = hs.Plan.instanced(soff, spar, sid)
    assert plan.num_joints == N and plan.bind_rows == spar.size
    G, S = hs.hs_scan_forward(plan, dev(q), dev(t), dev(s), inv_bind=dev(inv_s))
    ref_plan = hs.Plan(off, par, schedule=hs.HS_SCHED_CLASSES)  # the same tiles as the instanced plan
    G2, S2 = hs.hs_scan_forward(ref_plan, dev(q), dev(t), dev(s), inv_bind=dev(inv_s[rows]))
    torch.cuda.synchronize()
    G, S, G2, S2 = (x.cpu().numpy() for x in (G, S, G2, S2))
    np.testing.assert_array_equal(G, G2)
    np.testing.assert_array_equal(S, S2)

    b = wl.Batch("inst", off, par, q, t, s, q, t, s)
    Gr, lam, _ = reference(b)
    check_global(G, Gr, lam, "instanced globals")
    check_skin(S, Gr, inv_s[rows], lam, "instanced skin")


def test_autotuned_instanced_plan():
    """Autotuning times candidate shapes on the instanced tiles themselves
    (scratch poses, the plan's own offsets for the character map)."""
    rng = np.random.default_rng(24)
    soff, spar, rest = skeletons(rng, [256, 700])
    sid = rng.integers(0, 2, 400).astype(np.int32)
    off, par, rows = expand(soff, spar, sid)
    N = int(off[-1])
    q, t, s = wl.random_pose(rng, N)
    inv_s = skeleton_inverse_binds(soff, spar, rest)
    plan = hs.Plan.instanced(soff, spar, sid, autotune=True)
    G, S = hs.hs_scan_forward(plan, dev(q), dev(t), dev(s), inv_bind=dev(inv_s))
    torch.cuda.synchronize()
    b = wl.Batch("inst", off, par, q, t, s, q, t, s)
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "autotuned instanced globals")
    check_skin(S.cpu().numpy(), Gr, inv_s[rows], lam, "autotuned instanced skin")


def test_fused_sampling_and_skin_of_one_shared_skeleton():
    b = wl.fused_sample_instanced(num_characters=40)
    x = b.extra
    soff, spar, sid = x["skel_offsets"], x["skel_parents"], x["skeleton_id"]
    inv_s = skeleton_inverse_binds(soff, spar, x["skel_rest"])
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    cp = dict(clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]), time=dev(x["time"]), weight=dev(x["weight"]))
    plan = hs.Plan.instanced(soff, spar, sid)
    _, S = hs.hs_scan_forward(plan, clips=lib, **cp, want_global=False, inv_bind=dev(inv_s))
    ref_plan = hs.Plan(b.offsets, b.parents, schedule=hs.HS_SCHED_CLASSES)  # the same tiles as the instanced plan
    rows = np.tile(np.arange(spar.size), b.num_characters)
    _, S2 = hs.hs_scan_forward(ref_plan, clips=lib, **cp, want_global=False, inv_bind=dev(inv_s[rows]))
    torch.cuda.synchronize()
    S, S2 = S.cpu().numpy(), S2.cpu().numpy()
    np.testing.assert_array_equal(S, S2)
    q, tr = oracle.pose_sample(b.offsets, x["key_quat"], x["key_trans"], x["clip_a"], x["clip_b"], x["time"],
                               x["weight"], x["fps"])
    Gr = oracle.forward(b.offsets, b.parents, q, tr, None)
    lam = oracle.path_length(b.offsets, b.parents, Gr, tr)
    check_skin(S, Gr, inv_s[rows], lam, "instanced fused sample + skin")


def test_backward_and_graph_on_an_instanced_plan():
    rng = np.random.default_rng(22)
    soff, spar, rest = skeletons(rng, [96, 512])
    sid = rng.integers(0, 2, 50).astype(np.int32)
    off, par, rows = expand(soff, spar, sid)
    N = int(off[-1])
    q, t, s = wl.random_pose(rng, N)
    inv_s = skeleton_inverse_binds(soff, spar, rest)
    plan = hs.Plan.instanced(soff, spar, sid)
    ref_plan = hs.Plan(off, par)
    Wh = rng.standard_normal((N, 4, 4)).astype(np.float32)
    W = dev(Wh)
    a = hs.hs_scan_backward(plan, dev(q), dev(t), dev(s), W)
    b_ = hs.hs_scan_backward(ref_plan, dev(q), dev(t), dev(s), W)
    torch.cuda.synchronize()
    # colliding adjoint pushes are summed in arrival order, so the two plans
    # agree to rounding, not bitwise: both are held to the oracle's gradients
    ref = oracle.backward(off, par, q, t, s, Wh)
    for got in (a, b_):
        for name, g, r in zip(("quat", "trans", "scale"), got, ref):
            g = g.cpu().numpy().astype(np.float64)
            for c in range(sid.size):
                sl = slice(off[c], off[c + 1])
                scale = max(1.0, float(np.abs(r[sl]).max()))
                assert np.abs(g[sl] - r[sl]).max() <= 1e-4 * scale, f"{name} grad of character {c}"
    # a captured forward replays the eager result
    qd, td, sd = dev(q), dev(t), dev(s)
    G = torch.empty((N, 4, 4), device=DEV)
    S = torch.empty((N, 4, 4), device=DEV)
    B = dev(inv_s)
    graph = hs.ForwardGraph(plan, qd, td, sd, global_out=G, inv_bind=B, skin_out=S)
    Ge, Se = hs.hs_scan_forward(plan, qd, td, sd, inv_bind=B)
    for _ in range(3):
        G.zero_()
        S.zero_()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(G, Ge) and torch.equal(S, Se)


def test_instanced_plan_errors():
    rng = np.random.default_rng(23)
    soff, spar, _ = skeletons(rng, [64, 128])
    sid = np.array([0, 1, 1], np.int32)
    with pytest.raises(hs.HSError) as ei:
        hs.Plan.instanced(soff, spar, sid, chain_units=True)
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HSError) as ei:
        hs.Plan.instanced(soff, spar, sid, strategy=hs.HS_STRATEGY_MULTIPASS)
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED
    big = np.arange(-1, 5000, dtype=np.int32)
    with pytest.raises(hs.HSError) as ei:  # too large for any tile
        hs.Plan.instanced(np.array([0, big.size]), big, np.zeros(2, np.int32))
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED
    bad = spar.copy()
    bad[70] = 80  # skeleton-local parent after its child
    with pytest.raises(hs.HSError) as ei:
        hs.Plan.instanced(soff, bad, sid)
    assert ei.value.status == hs.HS_ERR_TOPOLOGY
    # an id out of range, through the C ABI directly (the binding checks it first)
    lib = hs.load_library()
    sk = hs.hs_skeleton_set(2, spar.size, soff.ctypes.data, spar.ctypes.data)
    ids = np.array([0, 2], np.int32)
    opts = hs.hs_plan_opts()
    h = ctypes.c_void_p()
    rc = lib.hs_plan_create_instanced(hs.default_context().handle, ctypes.byref(sk), 2, ids.ctypes.data,
                                      ctypes.byref(opts), ctypes.byref(h))
    assert rc == hs.HS_ERR_INVALID_ARG and not h.value


def test_fused_sample_instanced_full_size_sampled():
    """The benchmark configuration (10 000 instances of one 256-joint
    skeleton, clip sampling, skin only) in its autotuned launch; 32 seeded
    characters checked against the oracle."""
    b = wl.fused_sample_instanced()
    x = b.extra
    soff, spar, sid = x["skel_offsets"], x["skel_parents"], x["skeleton_id"]
    inv_s = skeleton_inverse_binds(soff, spar, x["skel_rest"])
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    plan = hs.Plan.instanced(soff, spar, sid, autotune=True)
    _, S = hs.hs_scan_forward(plan, clips=lib, clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]),
                              time=dev(x["time"]), weight=dev(x["weight"]), want_global=False,
                              inv_bind=dev(inv_s))
    torch.cuda.synchronize()
    chars = np.sort(np.random.default_rng(25).choice(b.num_characters, 32, replace=False))
    J = spar.size
    sub = lambda a: a[chars]
    sub_off = np.arange(chars.size + 1) * J
    q, tr = oracle.pose_sample(sub_off, x["key_quat"], x["key_trans"], sub(x["clip_a"]), sub(x["clip_b"]),
                               sub(x["time"]), sub(x["weight"]), x["fps"])
    par = np.tile(spar, chars.size)
    Gr = oracle.forward(sub_off, par, q, tr, None)
    lam = oracle.path_length(sub_off, par, Gr, tr)
    S_sub = np.concatenate([S[c * J:(c + 1) * J].cpu().numpy() for c in chars])
    check_skin(S_sub, Gr, np.tile(inv_s, (chars.size, 1, 1)), lam, "full-size instanced fused skin")

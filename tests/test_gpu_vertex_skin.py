"""GPU parity of vertex skinning (hs_mesh_create / hs_skin_vertices and the
one-pass hs_scan_skin_vertices) against the FP64 oracle.

End to end (check_e2e): the reference is the oracle's alone -- its
sampler (for clip poses), its forward scan, its skin step and its vertex
skinning (oracle/vertex_skin.py), all in FP64 from the same fp32 inputs.
The skin matrices carry the scan's tolerance (rotation entries within
1e-4, translations within 1e-4 (lambda_j + |t(B^-1_j)|)); a blend of
influences with weights summing to one moves a vertex by at most the
largest influence's error, |dA| 3|p|_inf + |dt|, so per vertex
|p'_gpu - p'_fp64|_inf <= 1e-4 (3 |p|_inf + max_i (lambda_i + |t(B^-1_i)|))
plus the blend's own rounding below.

The vertex kernel alone (check): both sides fed the same fp32 skin
matrices from the library's own forward pass, |p'_gpu - p'_fp64|_inf <=
1e-5 * (1 + |p| + max_i |t_i|), with t_i the translations of the vertex's
four skin matrices.  A linear blend sums at most 16 fp32 products per
coordinate (error below 16 u |terms|, u = 6e-8); dual quaternions add a
square root, a division and two cross products per vertex (a few tens of
u); 1e-5 leaves a margin of about 3 over both.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import vertex_skin as ovs
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check(out, offsets, S, voff, mfirst, pos, joints, weights, method, what):
    ref = ovs.skin_vertices(method, offsets, S, voff, mfirst, pos, joints, weights)
    counts = np.diff(voff)
    rows = np.concatenate([np.arange(mfirst[c], mfirst[c] + counts[c]) for c in range(len(counts))])
    char = np.repeat(np.arange(len(counts)), counts)
    t = np.asarray(S, np.float64)[offsets[char][:, None] + joints[rows].astype(np.int64), :3, 3]
    scale = 1.0 + np.linalg.norm(pos[rows], axis=1) + np.linalg.norm(t, axis=2).max(axis=1)
    err = np.abs(np.asarray(out, np.float64) - ref).max(axis=1)
    worst = int(np.argmax(err / scale))
    assert np.all(np.isfinite(out)), f"{what}: non-finite output"
    assert np.all(err <= 1e-5 * scale), f"{what}: vertex {worst} error {err[worst]:.3e} (scale {scale[worst]:.2f})"


def check_e2e(out, offsets, parents, q, t, s, inv_rows, voff, mfirst, pos, joints, weights, method, what):
    """out against the oracle's own pipeline: FP64 forward of the fp32 poses,
    skin matrices with the per-joint inverse binds inv_rows, vertex
    skinning."""
    G = oracle.forward(offsets, parents, q, t, s)
    lam = oracle.path_length(offsets, parents, G, t)
    S = oracle.skin(G, inv_rows)
    ref = ovs.skin_vertices(method, offsets, S, voff, mfirst, pos, joints, weights)
    counts = np.diff(voff)
    rows = np.concatenate([np.arange(mfirst[c], mfirst[c] + counts[c]) for c in range(len(counts))])
    char = np.repeat(np.arange(len(counts)), counts)
    gj = np.asarray(offsets)[char][:, None] + joints[rows].astype(np.int64)
    tb = np.linalg.norm(np.asarray(inv_rows, np.float64)[gj, :3, 3], axis=2)
    p = np.asarray(pos[rows], np.float64)
    ts = np.linalg.norm(S[gj, :3, 3], axis=2).max(axis=1)
    bound = (1e-4 * (3.0 * np.abs(p).max(axis=1) + (lam[gj] + tb).max(axis=1))
             + 1e-5 * (1.0 + np.linalg.norm(p, axis=1) + ts))
    err = np.abs(np.asarray(out, np.float64) - ref).max(axis=1)
    worst = int(np.argmax(err / bound))
    assert np.all(np.isfinite(out)), f"{what}: non-finite output"
    assert np.all(err <= bound), f"{what} (oracle end to end): vertex {worst} error {err[worst]:.3e} > {bound[worst]:.3e}"


def sampled_poses(b, chars=None):
    """The oracle's sampled local poses (FP64) of a clip-driven batch, for
    all characters or the listed ones (with their sub-batch offsets)."""
    x = b.extra
    if chars is None:
        return b.offsets, oracle.pose_sample(b.offsets, x["key_quat"], x["key_trans"], x["clip_a"], x["clip_b"],
                                             x["time"], x["weight"], x["fps"])
    sub_off = np.concatenate([[0], np.cumsum(np.diff(b.offsets)[chars])]).astype(np.int64)
    return sub_off, oracle.pose_sample(sub_off, x["key_quat"], x["key_trans"], x["clip_a"][chars],
                                       x["clip_b"][chars], x["time"][chars], x["weight"][chars], x["fps"])


def instanced_rows(b, inv_s, chars=None):
    """Per-joint inverse binds of an instanced batch (one row per skeleton
    joint expanded to every instance)."""
    x = b.extra
    soff = x["skel_offsets"]
    sid = x["skeleton_id"] if chars is None else x["skeleton_id"][chars]
    return np.concatenate([inv_s[soff[k]:soff[k + 1]] for k in sid])


def posed_skins(plan, batch, inv_rows):
    G, S = hs.hs_scan_forward(plan, dev(batch.quat), dev(batch.trans), dev(batch.scale), inv_bind=dev(inv_rows))
    torch.cuda.synchronize()
    return S


@pytest.mark.parametrize("method", [hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT])
def test_meshes_of_several_skeletons(method):
    """Three skeletons with their own meshes (2000, 1000 and 3000 faces),
    characters drawn among them, one character without a mesh."""
    rng = np.random.default_rng(31)
    tmpls = [wl.humanoid_with_chains(["tail", "hair"], 64)[0], wl.HUMANOID_PARENTS,
             wl.humanoid_with_chains(["tail", "cape_l", "cape_r", "hair"], 200)[0]]
    meshes = [wl.skin_mesh(rng, p, f) for p, f in zip(tmpls, (2000, 1000, 3000))]
    sid = rng.integers(0, 3, 60).astype(np.int32)
    par = np.concatenate([tmpls[k] for k in sid]).astype(np.int32)
    off = np.concatenate([[0], np.cumsum([tmpls[k].size for k in sid])]).astype(np.int64)
    N = int(off[-1])
    q, t, s = wl.random_pose(rng, N)
    b = wl.Batch("meshes", off, par, q, t, s, q, t, s)
    # skin matrices of an arbitrary rigid bind pose: inverse binds of a second
    # random pose, computed in FP64 on the host
    rq, rt, rs = wl.random_pose(rng, N)
    inv = np.linalg.inv(oracle.forward(off, par, rq, rt, rs)).astype(np.float32)
    plan = hs.Plan(off, par)
    S = posed_skins(plan, b, inv).cpu().numpy()
    mrow = np.concatenate([[0], np.cumsum([m[0].shape[0] for m in meshes])])
    pos = np.concatenate([m[0] for m in meshes])
    joints = np.concatenate([m[1] for m in meshes])
    weights = np.concatenate([m[2] for m in meshes])
    counts = np.array([meshes[k][0].shape[0] for k in sid])
    counts[7] = 0
    voff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    mfirst = mrow[sid].astype(np.int32)
    mesh = hs.Mesh(plan, voff, mfirst, pos, joints, weights)
    out = hs.hs_skin_vertices(mesh, dev(S.astype(np.float32)), method)
    torch.cuda.synchronize()
    check(out.cpu().numpy(), off, S, voff, mfirst, pos, joints, weights, method, f"method {method}")
    check_e2e(out.cpu().numpy(), off, par, q, t, s, inv, voff, mfirst, pos, joints, weights, method,
              f"method {method}")


@pytest.mark.parametrize("method", [hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT])
def test_mesh_skinning_workload_sampled(method):
    """The mesh_skinning preset at reduced size: instanced plan, clip-sampled
    poses, skin matrices from the fused forward, one shared mesh."""
    b = wl.mesh_skinning(num_characters=200)
    x = b.extra
    inv_s = np.linalg.inv(oracle.forward(x["skel_offsets"], x["skel_parents"], *x["skel_rest"])).astype(np.float32)
    plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"])
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    _, S = hs.hs_scan_forward(plan, clips=lib, clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]),
                              time=dev(x["time"]), weight=dev(x["weight"]), want_global=False,
                              inv_bind=dev(inv_s))
    mesh = hs.Mesh(plan, x["vertex_offsets"], x["mesh_first"], x["mesh_positions"], x["mesh_joints"],
                   x["mesh_weights"])
    out = hs.hs_skin_vertices(mesh, S, method)
    torch.cuda.synchronize()
    check(out.cpu().numpy(), b.offsets, S.cpu().numpy(), x["vertex_offsets"], x["mesh_first"], x["mesh_positions"],
          x["mesh_joints"], x["mesh_weights"], method, f"mesh_skinning method {method}")
    off, (qr, tr) = sampled_poses(b)
    check_e2e(out.cpu().numpy(), off, b.parents, qr, tr, None, instanced_rows(b, inv_s), x["vertex_offsets"],
              x["mesh_first"], x["mesh_positions"], x["mesh_joints"], x["mesh_weights"], method,
              f"mesh_skinning method {method}")


def test_rest_pose_leaves_vertices_in_place():
    """Posed at the bind pose, S_j is the identity up to rounding, so both
    methods return the bind-space positions."""
    rng = np.random.default_rng(32)
    par = wl.humanoid_with_chains(["tail"], 30)[0]
    q, t, s = wl.random_pose(rng, par.size)
    inv = np.linalg.inv(oracle.forward(np.array([0, par.size]), par, q, t, s)).astype(np.float32)
    plan = hs.Plan(np.array([0, par.size]), par)
    b = wl.Batch("rest", np.array([0, par.size]), par, q, t, s, q, t, s)
    S = posed_skins(plan, b, inv)
    pos, joints, weights = wl.skin_mesh(rng, par, 1500)
    mesh = hs.Mesh(plan, [0, pos.shape[0]], [0], pos, joints, weights)
    for method in (hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT):
        out = hs.hs_skin_vertices(mesh, S, method)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.cpu().numpy(), pos, atol=2e-5)


def test_mesh_errors():
    rng = np.random.default_rng(33)
    par = wl.HUMANOID_PARENTS
    off = np.array([0, 64, 128])
    plan = hs.Plan(off, np.concatenate([par, par]))
    pos, joints, weights = wl.skin_mesh(rng, par, 200)
    V = pos.shape[0]
    bad = joints.copy()
    bad[5, 2] = 64  # one past the character's last joint
    with pytest.raises(hs.HSError) as ei:
        hs.Mesh(plan, [0, V, 2 * V], [0, 0], pos, bad, weights)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    with pytest.raises(hs.HSError) as ei:  # rows past the end of the mesh arrays
        hs.Mesh(plan, [0, V, 2 * V], [0, 1], pos, joints, weights)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    mesh = hs.Mesh(plan, [0, V, 2 * V], [0, 0], pos, joints, weights)
    S = torch.zeros((128, 4, 4), device=DEV)
    with pytest.raises(hs.HSError) as ei:
        hs.hs_skin_vertices(mesh, S, method=7)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    big = np.arange(-1, 2100, dtype=np.int32)
    plan2 = hs.Plan(np.array([0, big.size]), big)
    with pytest.raises(hs.HSError) as ei:  # too many joints to stage
        hs.Mesh(plan2, [0, V], [0], pos, joints, weights)
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED


@pytest.mark.parametrize("method", [hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT])
def test_mesh_skinning_full_size_sampled(method):
    """The benchmark configuration (10 000 instances, 10.0 M vertices) in
    the launch the benchmark times; 24 seeded characters' vertices checked
    against the oracle on the same skin matrices."""
    b = wl.mesh_skinning()
    x = b.extra
    inv_s = np.linalg.inv(oracle.forward(x["skel_offsets"], x["skel_parents"], *x["skel_rest"])).astype(np.float32)
    plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"])
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    _, S = hs.hs_scan_forward(plan, clips=lib, clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]),
                              time=dev(x["time"]), weight=dev(x["weight"]), want_global=False,
                              inv_bind=dev(inv_s))
    mesh = hs.Mesh(plan, x["vertex_offsets"], x["mesh_first"], x["mesh_positions"], x["mesh_joints"],
                   x["mesh_weights"])
    out = hs.hs_skin_vertices(mesh, S, method)
    torch.cuda.synchronize()
    chars = np.sort(np.random.default_rng(34).choice(b.num_characters, 24, replace=False))
    J = x["skel_parents"].size
    V = x["mesh_positions"].shape[0]
    S_sub = np.concatenate([S[c * J:(c + 1) * J].cpu().numpy() for c in chars])
    out_sub = np.concatenate([out[c * V:(c + 1) * V].cpu().numpy() for c in chars])
    sub_off = np.arange(chars.size + 1) * J
    sub_voff = np.arange(chars.size + 1, dtype=np.int64) * V
    check(out_sub, sub_off, S_sub, sub_voff, np.zeros(chars.size, np.int32), x["mesh_positions"],
          x["mesh_joints"], x["mesh_weights"], method, f"full size method {method}")
    ids = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in chars])
    off_r, (qr, tr) = sampled_poses(b, chars)
    check_e2e(out_sub, off_r, b.parents[ids], qr, tr, None, instanced_rows(b, inv_s, chars), sub_voff,
              np.zeros(chars.size, np.int32), x["mesh_positions"], x["mesh_joints"], x["mesh_weights"], method,
              f"full size method {method}")


@pytest.mark.parametrize("method", [hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT])
@pytest.mark.parametrize("instanced", [False, True])
def test_one_pass_pipeline_equals_two_calls(method, instanced):
    """hs_scan_skin_vertices (clip sampling, scan, skin and vertex skinning
    per tile, S kept on chip) gives bitwise the output of hs_scan_forward
    followed by hs_skin_vertices, and its optional skin rows equal the
    forward's."""
    b = wl.mesh_skinning(num_characters=300)
    x = b.extra
    inv_s = np.linalg.inv(oracle.forward(x["skel_offsets"], x["skel_parents"], *x["skel_rest"])).astype(np.float32)
    if instanced:
        plan = hs.Plan.instanced(x["skel_offsets"], x["skel_parents"], x["skeleton_id"])
        inv = dev(inv_s)
    else:
        plan = hs.Plan(b.offsets, b.parents)
        inv = dev(np.tile(inv_s, (b.num_characters, 1, 1)))
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    cp = dict(clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]), time=dev(x["time"]), weight=dev(x["weight"]))
    mesh = hs.Mesh(plan, x["vertex_offsets"], x["mesh_first"], x["mesh_positions"], x["mesh_joints"],
                   x["mesh_weights"])
    _, S = hs.hs_scan_forward(plan, clips=lib, **cp, want_global=False, inv_bind=inv)
    two = hs.hs_skin_vertices(mesh, S, method)
    S1 = torch.empty_like(S)
    one = hs.hs_scan_skin_vertices(plan, mesh, inv, clips=lib, **cp, method=method, skin_out=S1)
    torch.cuda.synchronize()
    assert torch.equal(one, two)
    assert torch.equal(S1, S)
    check(one.cpu().numpy(), b.offsets, S.cpu().numpy(), x["vertex_offsets"], x["mesh_first"], x["mesh_positions"],
          x["mesh_joints"], x["mesh_weights"], method, f"one pass method {method}")
    off, (qr, tr) = sampled_poses(b)
    check_e2e(one.cpu().numpy(), off, b.parents, qr, tr, None, instanced_rows(b, inv_s), x["vertex_offsets"],
              x["mesh_first"], x["mesh_positions"], x["mesh_joints"], x["mesh_weights"], method,
              f"one pass method {method}")


def test_one_pass_pipeline_on_several_size_classes_and_trs_poses():
    """Characters of 64 to 1600 joints (three tile size classes under
    2048-joint tiles), TRS poses, meshes on some characters only."""
    rng = np.random.default_rng(35)
    sizes = [64, 300, 1100, 1600, 2000]
    tm = []
    for n in sizes:
        p = np.empty(n, np.int32)
        p[0] = -1
        for j in range(1, n):
            p[j] = j - 1 if rng.uniform() < 0.7 else rng.integers(0, j)
        tm.append(p)
    sid = rng.integers(0, len(sizes), 40)
    par = np.concatenate([tm[k] for k in sid]).astype(np.int32)
    off = np.concatenate([[0], np.cumsum([sizes[k] for k in sid])]).astype(np.int64)
    N = int(off[-1])
    q, t, s = wl.random_pose(rng, N)
    rq, rt, rs = wl.random_pose(rng, N)
    inv = np.linalg.inv(oracle.forward(off, par, rq, rt, rs)).astype(np.float32)
    meshes = [wl.skin_mesh(rng, p, 1000) for p in tm]
    mrow = np.concatenate([[0], np.cumsum([m[0].shape[0] for m in meshes])])
    pos = np.concatenate([m[0] for m in meshes])
    joints = np.concatenate([m[1] for m in meshes])
    weights = np.concatenate([m[2] for m in meshes])
    counts = np.array([meshes[k][0].shape[0] for k in sid]) * (rng.uniform(size=sid.size) < 0.8)
    voff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    mfirst = mrow[sid].astype(np.int32)
    # the one-pass kernel runs the size-class tiles: the forward of the
    # two-call route takes the same tiles for a bitwise comparison
    plan = hs.Plan(off, par, tile_joints=2048, schedule=hs.HS_SCHED_CLASSES)
    assert plan.info["multipass_joints"] == 0
    mesh = hs.Mesh(plan, voff, mfirst, pos, joints, weights)
    _, S = hs.hs_scan_forward(plan, dev(q), dev(t), dev(s), inv_bind=dev(inv), want_global=False)
    for method in (hs.HS_SKIN_LINEAR, hs.HS_SKIN_DUAL_QUAT):
        two = hs.hs_skin_vertices(mesh, S, method)
        one = hs.hs_scan_skin_vertices(plan, mesh, dev(inv), dev(q), dev(t), dev(s), method=method)
        torch.cuda.synchronize()
        assert torch.equal(one, two), method
        check_e2e(one.cpu().numpy(), off, par, q, t, s, inv, voff, mfirst, pos, joints, weights, method,
                  f"size classes method {method}")
    # a plan with multipass characters is refused
    big = hs.Plan(off, par, tile_joints=1024)
    mesh_big = hs.Mesh(big, voff, mfirst, pos, joints, weights)
    with pytest.raises(hs.HSError) as ei:
        hs.hs_scan_skin_vertices(big, mesh_big, dev(inv), dev(q), dev(t), dev(s))
    assert ei.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HSError) as ei:  # a mesh made for another plan
        hs.hs_scan_skin_vertices(plan, mesh_big, dev(inv), dev(q), dev(t), dev(s))
    assert ei.value.status == hs.HS_ERR_INVALID_ARG

"""The seeded generators produce the shapes the workload recipes state."""
import numpy as np

from paper_2505_06703_amd import workloads as wl


def _valid(b):
    off, par = b.offsets, b.parents
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == par.size
    local = np.arange(par.size) - np.repeat(off[:-1], np.diff(off))
    assert np.all(par >= -1) and np.all(par < local)
    for a, w in ((b.quat, 4), (b.trans, 3), (b.scale, 3)):
        assert a.dtype == np.float32 and a.shape == (par.size, w)


def test_humanoid_template():
    par, names = wl.humanoid64()
    assert par.size == 64 and par[0] == -1 and np.all(par[1:] < np.arange(1, 64))
    assert wl.levels_of(par).max() == 11


def test_plain_scan_shape():
    b = wl.plain_scan()
    _valid(b)
    assert b.num_characters == 64 and b.num_joints == 4096 and b.depth() <= 16
    q = b.quat.astype(np.float64)
    assert np.abs(np.linalg.norm(q, axis=1) - 1).max() < 1e-6
    ang = 2 * np.arccos(np.clip(np.abs(q[:, 3]), 0, 1))
    assert ang.max() <= 0.3 + 1e-5
    ln = np.linalg.norm(b.trans, axis=1)
    assert ln.min() >= 0.05 - 1e-6 and ln.max() <= 0.3 + 1e-6


def test_deep_forward_small():
    b = wl.deep_forward(num_characters=3)
    _valid(b)
    assert b.num_joints == 3 * 1024 and b.depth() == 246


def test_fused_and_differentiable_depths():
    b3 = wl.fused_sample(num_characters=2)
    _valid(b3)
    assert b3.num_joints == 512 and b3.depth() == 70
    kq = b3.extra["key_quat"]
    assert kq.shape == (64, 30, 256, 4)
    assert np.all(b3.extra["clip_a"] != b3.extra["clip_b"])
    b4 = wl.differentiable(num_characters=2)
    _valid(b4)
    assert b4.num_joints == 1024 and b4.depth() == 118
    assert b4.extra["effectors"].size == 32
    assert np.linalg.norm(b4.extra["target_offsets"], axis=1).max() <= 0.5 + 1e-6


def test_heterogeneous_small():
    b = wl.heterogeneous(num_characters=400)
    _valid(b)
    n = np.diff(b.offsets)
    assert n.min() >= 32 and n.max() <= 2048
    chains = np.nonzero(b.extra["is_chain"])[0]
    assert chains.size == 4
    for c in chains:
        p = b.parents[b.offsets[c]:b.offsets[c + 1]]
        assert np.array_equal(p, np.arange(-1, p.size - 1))


def test_seeds_are_reproducible():
    a, b = wl.plain_scan(seed=0), wl.plain_scan(seed=0)
    assert np.array_equal(a.parents, b.parents) and np.array_equal(a.quat, b.quat)


def test_long_chains_small():
    b = wl.long_chains(num_characters=2, chain_len=300)
    _valid(b)
    assert b.num_joints == 600 and b.depth() == 300
    q = b.quat.astype(np.float64)
    ang = 2 * np.arccos(np.clip(np.abs(q[:, 3]), 0, 1))
    assert ang.max() <= 0.01 + 2e-4  # fp32 arccos near 1 loses ~1e-4


def test_depth_sweep_depths():
    for d in (15, 120):
        b = wl.depth_sweep(num_characters=5, depth=d, templates=5)
        _valid(b)
        assert b.num_joints == 1500 and b.depth() == d


def test_fused_sample_instanced_shares_one_skeleton():
    b = wl.fused_sample_instanced(num_characters=5)
    x = b.extra
    J = x["skel_parents"].size
    assert list(x["skel_offsets"]) == [0, J] and np.all(x["skeleton_id"] == 0)
    np.testing.assert_array_equal(b.parents, np.tile(x["skel_parents"], 5))
    np.testing.assert_array_equal(b.rest_quat, np.tile(x["skel_rest"][0], (5, 1)))
    # the per-character clip choices are those of fused_sample with the same seed
    ref = wl.fused_sample(num_characters=5)
    np.testing.assert_array_equal(x["clip_a"], ref.extra["clip_a"])


def test_skin_mesh_influences_and_weights():
    rng = np.random.default_rng(0)
    par = wl.humanoid_with_chains(["tail"], 8)[0]
    pos, joints, w = wl.skin_mesh(rng, par, num_faces=1000)
    assert pos.shape == (502, 3) and joints.shape == (502, 4) and w.shape == (502, 4)
    assert joints.min() >= 0 and joints.max() < par.size
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=1e-6)
    assert np.all(np.diff(w, axis=1) <= 0)  # influence 0 weighs most
    # influences 1 and 2 are the parent and grandparent (roots stand in)
    p1 = np.where(par[joints[:, 0]] < 0, joints[:, 0], par[joints[:, 0]])
    np.testing.assert_array_equal(joints[:, 1], p1)
    assert np.linalg.norm(pos, axis=1).max() <= 1.0 + 1e-6

"""Seeded synthetic skeleton workloads (input generation only).

This module draws topologies, local poses, rest poses, animation clips and
targets with NumPy's PCG64 generator.  It performs none of the method's
arithmetic (no scan, skin, sampling or gradient): quantities that need it,
such as inverse bind matrices or targets built from rest-pose positions, are
computed by the caller from ``rest_*`` arrays returned here.

The shapes follow the paper's benchmark (Sec. 4, Table 1: thousands of
characters of a few hundred joints, hierarchies 15-120 levels deep) and the
workload presets below:

* ``plain_scan``      -- 64 random trees of 64 joints, depth <= 16;
* ``deep_forward``    -- 4096 x (humanoid-64 + 4 chains of 240), depth 246;
* ``heterogeneous``   -- 16384 random trees, sizes log-uniform in [32, 2048],
                         branching probability 0.3, 1% pure chains;
* ``fused_sample``    -- 10000 x (humanoid-64 + 3 chains of 64) sampling a
                         library of 64 clips x 30 keys;
* ``fused_sample_instanced`` -- fused_sample with all characters instances
                         of one skeleton (shared hierarchy and rest pose);
* ``mesh_skinning``   -- fused_sample_instanced with a 2000-face mesh bound
                         to the skeleton (vertex skinning);
* ``differentiable``  -- 1024 x (humanoid-64 + 4 chains of 112) with 16
                         end effectors and targets;
* ``long_chains``     -- 64 chains of 65536 joints (the multipass path);
* ``depth_sweep``     -- the paper's experiment scene: 10000 characters of
                         300 joints at a chosen depth (15 to 120 levels).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# --------------------------------------------------------------------------
# humanoid template: 64 joints in depth-first order (parents precede children)
# --------------------------------------------------------------------------


def humanoid64():
    """Return (parents[64] int32, names[64]) of the 64-joint humanoid template.

    pelvis -> spine0 -> spine1 -> chest -> neck -> head -> {head_end, jaw,
    eye_l, eye_r}; per arm from the chest: clavicle, upperarm, upperarm_twist,
    forearm, forearm_twist, hand and 5 fingers of 3 joints; per leg from the
    pelvis: thigh, thigh_twist, calf, foot, ball, toe_end.  Deepest joints
    (fingertips) are at level 11.
    """
    parents, names = [], []

    def add(name, parent):
        parents.append(parent)
        names.append(name)
        return len(parents) - 1

    pelvis = add("pelvis", -1)
    s0 = add("spine0", pelvis)
    s1 = add("spine1", s0)
    chest = add("chest", s1)
    neck = add("neck", chest)
    head = add("head", neck)
    add("head_end", head)
    add("jaw", head)
    add("eye_l", head)
    add("eye_r", head)
    for side in ("l", "r"):
        cla = add(f"clavicle_{side}", chest)
        ua = add(f"upperarm_{side}", cla)
        add(f"upperarm_twist_{side}", ua)
        fa = add(f"forearm_{side}", ua)
        add(f"forearm_twist_{side}", fa)
        hand = add(f"hand_{side}", fa)
        for finger in ("thumb", "index", "middle", "ring", "pinky"):
            a = add(f"{finger}_01_{side}", hand)
            b = add(f"{finger}_02_{side}", a)
            add(f"{finger}_03_{side}", b)
    for side in ("l", "r"):
        th = add(f"thigh_{side}", pelvis)
        add(f"thigh_twist_{side}", th)
        ca = add(f"calf_{side}", th)
        ft = add(f"foot_{side}", ca)
        ba = add(f"ball_{side}", ft)
        add(f"toe_end_{side}", ba)
    assert len(parents) == 64
    return np.asarray(parents, np.int32), names


HUMANOID_PARENTS, HUMANOID_NAMES = humanoid64()
_ATTACH = {"tail": "pelvis", "cape_l": "chest", "cape_r": "chest", "hair": "head"}


def humanoid_with_chains(chain_names, chain_len):
    """Humanoid-64 followed by chains with consecutive ids.

    Returns (parents int32, chain_mask bool, chain_tips list of local ids).
    """
    par = list(HUMANOID_PARENTS)
    mask = [False] * 64
    tips = []
    for cname in chain_names:
        attach = HUMANOID_NAMES.index(_ATTACH[cname])
        prev = attach
        for _ in range(chain_len):
            par.append(prev)
            mask.append(True)
            prev = len(par) - 1
        tips.append(prev)
    return np.asarray(par, np.int32), np.asarray(mask, bool), tips


def levels_of(parents):
    """Level of each joint of one character (root = 1)."""
    lev = np.empty(len(parents), np.int64)
    for j, p in enumerate(parents):
        lev[j] = 1 if p < 0 else lev[p] + 1
    return lev


# --------------------------------------------------------------------------
# pose distribution
# --------------------------------------------------------------------------


def random_unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return v / nrm


def random_quats(rng, n, max_angle):
    """Unit quaternions (x, y, z, w): axis uniform on S^2, angle U[-a, a]."""
    axis = random_unit_vectors(rng, n)
    ang = rng.uniform(-max_angle, max_angle, n)
    q = np.empty((n, 4), np.float64)
    q[:, :3] = axis * np.sin(ang / 2)[:, None]
    q[:, 3] = np.cos(ang / 2)
    return q.astype(np.float32)


def random_offsets(rng, n, lo=0.05, hi=0.3):
    """Translations with direction uniform on S^2 and length U[lo, hi]."""
    d = random_unit_vectors(rng, n)
    ln = rng.uniform(lo, hi, n)
    return (d * ln[:, None]).astype(np.float32)


def random_pose(rng, n, angle=None, max_angle=0.3):
    """(quat, trans, scale) for n joints; ``angle`` optionally per joint."""
    if angle is None:
        q = random_quats(rng, n, max_angle)
    else:
        q = np.empty((n, 4), np.float32)
        for a in np.unique(angle):
            sel = angle == a
            q[sel] = random_quats(rng, int(sel.sum()), float(a))
    t = random_offsets(rng, n)
    s = np.ones((n, 3), np.float32)
    return q, t, s


def ball_offsets(rng, n, radius):
    """Points uniform in a ball of the given radius."""
    d = random_unit_vectors(rng, n)
    r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    return (d * r[:, None]).astype(np.float32)


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------


@dataclass
class Batch:
    """A CSR batch of characters with local poses and a rest pose."""

    name: str
    offsets: np.ndarray            # int64 [C+1]
    parents: np.ndarray            # int32 [N], character-local, -1 root
    quat: np.ndarray               # float32 [N,4]
    trans: np.ndarray              # float32 [N,3]
    scale: np.ndarray              # float32 [N,3]
    rest_quat: np.ndarray          # float32 [N,4]
    rest_trans: np.ndarray         # float32 [N,3]
    rest_scale: np.ndarray         # float32 [N,3]
    extra: dict = field(default_factory=dict)

    @property
    def num_characters(self):
        return self.offsets.size - 1

    @property
    def num_joints(self):
        return int(self.offsets[-1])

    def depth(self):
        """Maximum depth in levels over all characters."""
        best = 0
        for c in range(self.num_characters):
            p = self.parents[self.offsets[c]:self.offsets[c + 1]]
            if p.size:
                best = max(best, int(levels_of(p).max()))
        return best


def _tile_same(template, C):
    n = template.size
    offsets = np.arange(C + 1, dtype=np.int64) * n
    parents = np.tile(template, C).astype(np.int32)
    return offsets, parents


def _pose_for(rng, N, chain_mask_full=None, chain_angle=None, base_angle=0.3):
    if chain_mask_full is None or chain_angle is None:
        q, t, s = random_pose(rng, N, max_angle=base_angle)
    else:
        ang = np.where(chain_mask_full, chain_angle, base_angle)
        q, t, s = random_pose(rng, N, angle=ang)
    return q, t, s


def c0_tree(rng, n=64, max_level=16):
    """Random tree: parent(i) uniform over earlier joints whose level < max_level."""
    parents = np.empty(n, np.int32)
    lev = np.empty(n, np.int64)
    parents[0], lev[0] = -1, 1
    for i in range(1, n):
        cand = np.nonzero(lev[:i] < max_level)[0]
        p = int(cand[rng.integers(0, cand.size)])
        parents[i] = p
        lev[i] = lev[p] + 1
    return parents


def plain_scan(seed=0, num_characters=64, joints=64, max_level=16):
    """64 characters x 64 joints, random trees of depth <= 16, with a rest pose."""
    rng = np.random.default_rng(seed)
    parents = np.concatenate([c0_tree(rng, joints, max_level) for _ in range(num_characters)])
    offsets = np.arange(num_characters + 1, dtype=np.int64) * joints
    N = int(offsets[-1])
    q, t, s = random_pose(rng, N)
    rq, rt, rs = random_pose(rng, N)
    return Batch("plain_scan", offsets, parents.astype(np.int32), q, t, s, rq, rt, rs)


def deep_forward(seed=1, num_characters=4096, chain_len=240, chain_angle=0.1):
    """Humanoid-64 + 4 chains (tail, 2 capes, hair) of 240: 1024 joints, depth 246."""
    rng = np.random.default_rng(seed)
    tmpl, mask, tips = humanoid_with_chains(["tail", "cape_l", "cape_r", "hair"], chain_len)
    offsets, parents = _tile_same(tmpl, num_characters)
    N = int(offsets[-1])
    cm = np.tile(mask, num_characters)
    q, t, s = _pose_for(rng, N, cm, chain_angle)
    rq, rt, rs = _pose_for(rng, N, cm, chain_angle)
    b = Batch("deep_forward", offsets, parents, q, t, s, rq, rt, rs)
    b.extra["template"] = tmpl
    b.extra["chain_tips"] = tips
    return b


def heterogeneous(seed=2, num_characters=16384, lo=32, hi=2048, p_chain_step=0.7,
                  chain_fraction=0.01):
    """Random trees with log-uniform sizes; parent(i) = i-1 w.p. 0.7 else
    uniform over [0, i); a seeded 1% of the characters are single chains."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), num_characters))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    n_chain = int(round(chain_fraction * num_characters))
    is_chain = np.zeros(num_characters, bool)
    is_chain[rng.choice(num_characters, n_chain, replace=False)] = True
    offsets = np.zeros(num_characters + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    N = int(offsets[-1])
    local = np.arange(N, dtype=np.int64) - np.repeat(offsets[:-1], sizes)
    step = rng.uniform(0.0, 1.0, N) < p_chain_step
    u = rng.uniform(0.0, 1.0, N)
    jump = np.floor(u * local).astype(np.int64)
    chain_joint = np.repeat(is_chain, sizes)
    parents = np.where(step | chain_joint, local - 1, jump)
    parents[local == 0] = -1
    q, t, s = random_pose(rng, N)
    rq, rt, rs = random_pose(rng, N)
    b = Batch("heterogeneous", offsets, parents.astype(np.int32), q, t, s, rq, rt, rs)
    b.extra["is_chain"] = is_chain
    return b


def fused_sample(seed=3, num_characters=10000, num_clips=64, num_keys=30, fps=30.0,
                 chain_len=64):
    """Humanoid-64 + 3 chains (tail, cape, hair) of 64: 256 joints, depth 70,
    with a shared library of clips and per-character clip choices."""
    rng = np.random.default_rng(seed)
    tmpl, mask, tips = humanoid_with_chains(["tail", "cape_l", "hair"], chain_len)
    J = tmpl.size
    offsets, parents = _tile_same(tmpl, num_characters)
    N = int(offsets[-1])
    kq = random_quats(rng, num_clips * num_keys * J, 0.3).reshape(num_clips, num_keys, J, 4)
    kt = random_offsets(rng, num_clips * num_keys * J).reshape(num_clips, num_keys, J, 3)
    ca = rng.integers(0, num_clips, num_characters).astype(np.int32)
    cb = (ca + rng.integers(1, num_clips, num_characters)) % num_clips
    cb = cb.astype(np.int32)
    tm = rng.uniform(0.0, 1.0, num_characters).astype(np.float32)
    wt = rng.uniform(0.0, 1.0, num_characters).astype(np.float32)
    # local pose arrays are what the sampler writes; keep placeholders of the
    # right shape and a rest pose for the inverse binds.
    q = np.zeros((N, 4), np.float32)
    q[:, 3] = 1.0
    t = np.zeros((N, 3), np.float32)
    s = np.ones((N, 3), np.float32)
    rq, rt, rs = random_pose(rng, N)
    b = Batch("fused_sample", offsets, parents, q, t, s, rq, rt, rs)
    b.extra.update(template=tmpl, key_quat=kq, key_trans=kt, clip_a=ca, clip_b=cb,
                   time=tm, weight=wt, fps=float(fps))
    return b


def fused_sample_instanced(seed=3, num_characters=10000, **kw):
    """fused_sample with every character an instance of one skeleton: the
    hierarchy and the rest pose (so the inverse binds) are the skeleton's,
    shared by all characters; poses still come from per-character clips."""
    b = fused_sample(seed=seed, num_characters=num_characters, **kw)
    tmpl = b.extra["template"]
    J = tmpl.size
    rng = np.random.default_rng(seed * 1000 + 7)
    rq, rt, rs = random_pose(rng, J)
    b.name = "fused_sample_instanced"
    b.rest_quat = np.tile(rq, (num_characters, 1))
    b.rest_trans = np.tile(rt, (num_characters, 1))
    b.rest_scale = np.tile(rs, (num_characters, 1))
    b.extra.update(skel_offsets=np.array([0, J], np.int64), skel_parents=tmpl.astype(np.int32),
                   skeleton_id=np.zeros(num_characters, np.int32), skel_rest=(rq, rt, rs))
    return b


def skin_mesh(rng, parents, num_faces=2000, radius=1.0):
    """A synthetic mesh bound to one skeleton: V = num_faces / 2 + 2 vertices
    (a closed genus-0 triangle mesh has F = 2V - 4 faces), each with four
    influences -- a joint drawn uniformly, its parent, its grandparent and a
    second uniform draw (a root stands in for missing ancestors) -- with
    Dirichlet(1) weights sorted so that influence 0 weighs most.  Positions
    are uniform in a ball in bind space.  Returns (positions [V,3] f32,
    joints [V,4] i32, weights [V,4] f32)."""
    parents = np.asarray(parents)
    n = parents.size
    V = num_faces // 2 + 2
    j0 = rng.integers(0, n, V)
    p1 = np.where(parents[j0] < 0, j0, parents[j0])
    p2 = np.where(parents[p1] < 0, p1, parents[p1])
    j3 = rng.integers(0, n, V)
    joints = np.stack([j0, p1, p2, j3], axis=1).astype(np.int32)
    w = np.sort(rng.dirichlet(np.ones(4), V), axis=1)[:, ::-1]
    pos = ball_offsets(rng, V, radius)
    return pos, joints, np.ascontiguousarray(w, dtype=np.float32)


def mesh_skinning(seed=8, num_characters=10000, num_faces=2000, **kw):
    """fused_sample_instanced plus one mesh of ``num_faces`` faces bound to
    the shared skeleton (every character skins the same mesh rows)."""
    b = fused_sample_instanced(seed=seed, num_characters=num_characters, **kw)
    rng = np.random.default_rng(seed * 1000 + 11)
    pos, joints, weights = skin_mesh(rng, b.extra["skel_parents"], num_faces)
    V = pos.shape[0]
    b.name = "mesh_skinning"
    b.extra.update(mesh_positions=pos, mesh_joints=joints, mesh_weights=weights,
                   vertex_offsets=np.arange(num_characters + 1, dtype=np.int64) * V,
                   mesh_first=np.zeros(num_characters, np.int32))
    return b


def differentiable(seed=4, num_characters=1024, chain_len=112, radius=0.5):
    """Humanoid-64 + 4 chains of 112 (512 joints, depth 118); 16 end
    effectors (4 chain tips, 10 fingertips, 2 toe ends) with target offsets
    drawn uniformly in a ball around the rest-pose positions."""
    rng = np.random.default_rng(seed)
    tmpl, mask, tips = humanoid_with_chains(["tail", "cape_l", "cape_r", "hair"], chain_len)
    offsets, parents = _tile_same(tmpl, num_characters)
    N = int(offsets[-1])
    q, t, s = random_pose(rng, N)
    rq, rt, rs = random_pose(rng, N)
    fingertips = [i for i, nm in enumerate(HUMANOID_NAMES) if nm.endswith(("_03_l", "_03_r"))]
    toes = [HUMANOID_NAMES.index("toe_end_l"), HUMANOID_NAMES.index("toe_end_r")]
    eff_local = np.asarray(tips + fingertips + toes, np.int64)
    assert eff_local.size == 16
    eff = (offsets[:-1, None] + eff_local[None, :]).reshape(-1)
    u = ball_offsets(rng, eff.size, radius)
    b = Batch("differentiable", offsets, parents, q, t, s, rq, rt, rs)
    b.extra.update(template=tmpl, effectors=eff, effectors_local=eff_local, target_offsets=u)
    return b


def long_chains(seed=5, num_characters=64, chain_len=65536, angle=0.01):
    """Single chains far beyond one workgroup's LDS (the multipass path):
    64 x 65536 joints, rotation angles U[-0.01, 0.01] (a long rope or
    cable: small bends per joint)."""
    rng = np.random.default_rng(seed)
    offsets = np.arange(num_characters + 1, dtype=np.int64) * chain_len
    parents = np.tile(np.arange(-1, chain_len - 1, dtype=np.int32), num_characters)
    N = int(offsets[-1])
    q, t, s = random_pose(rng, N, max_angle=angle)
    rq, rt, rs = random_pose(rng, N, max_angle=angle)
    return Batch("long_chains", offsets, parents, q, t, s, rq, rt, rs)


def depth_tree(rng, n, depth):
    """A tree of n joints and exactly `depth` levels: a spine from the root,
    then every further joint under a uniformly drawn earlier joint whose
    level is below `depth`."""
    depth = max(1, min(depth, n))
    par = np.empty(n, np.int32)
    lev = np.empty(n, np.int64)
    par[0], lev[0] = -1, 1
    for i in range(1, depth):
        par[i], lev[i] = i - 1, i + 1
    for i in range(depth, n):
        cand = np.nonzero(lev[:i] < depth)[0]
        p = int(cand[rng.integers(0, cand.size)])
        par[i], lev[i] = p, lev[p] + 1
    return par


def depth_sweep(seed=6, num_characters=10000, joints=300, depth=60, templates=64):
    """The paper's experiment scene (Sec. 4): characters of about 300 joints,
    hierarchies of a chosen depth (15 to 120 in the sweep); 64 seeded
    topologies cycled over the characters, poses as in plain_scan."""
    rng = np.random.default_rng(seed * 1000 + depth)
    tmpl = [depth_tree(rng, joints, depth) for _ in range(min(templates, num_characters))]
    parents = np.concatenate([tmpl[c % len(tmpl)] for c in range(num_characters)]).astype(np.int32)
    offsets = np.arange(num_characters + 1, dtype=np.int64) * joints
    N = int(offsets[-1])
    q, t, s = random_pose(rng, N)
    rq, rt, rs = random_pose(rng, N)
    return Batch("depth_sweep", offsets, parents, q, t, s, rq, rt, rs)


PRESETS = {
    "plain_scan": plain_scan,
    "deep_forward": deep_forward,
    "heterogeneous": heterogeneous,
    "fused_sample": fused_sample,
    "fused_sample_instanced": fused_sample_instanced,
    "mesh_skinning": mesh_skinning,
    "differentiable": differentiable,
    "long_chains": long_chains,
    "depth_sweep": depth_sweep,
}


def make(name, seed: Optional[int] = None, **kw):
    fn = PRESETS[name]
    return fn(**kw) if seed is None else fn(seed=seed, **kw)

"""Pins of the FP64 vertex-skinning oracle (oracle/vertex_skin.py) against
closed forms and invariants of linear blend and dual quaternion skinning
(Kavan et al. 2008); no GPU."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import vertex_skin as vs


def rz(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def affine(R, t):
    M = np.eye(4)
    M[:3, :3] = R
    M[:3, 3] = t
    return M


def one_character(S, positions, joints, weights):
    """Batch of one character with skin matrices S [J,4,4] and V vertices."""
    V = len(positions)
    return (np.array([0, len(S)]), np.asarray(S, np.float64), np.array([0, V]), np.array([0]),
            np.asarray(positions, np.float64), np.asarray(joints, np.int32), np.asarray(weights, np.float64))


@pytest.mark.parametrize("method", [0, 1])
def test_translations_only(method):
    rng = np.random.default_rng(1)
    t = rng.uniform(-2, 2, (4, 3))
    S = [affine(np.eye(3), ti) for ti in t]
    p = rng.uniform(-1, 1, (50, 3))
    w = rng.dirichlet(np.ones(4), 50)
    j = np.tile(np.arange(4), (50, 1))
    out = vs.skin_vertices(method, *one_character(S, p, j, w))
    np.testing.assert_allclose(out, p + w @ t, atol=1e-12)


@pytest.mark.parametrize("method", [0, 1])
def test_one_rigid_influence_is_a_rotation_and_offset(method):
    theta, t = 0.7, np.array([0.3, -1.2, 2.0])
    p = np.array([[1.0, 2.0, 3.0], [-0.5, 0.25, 4.0]])
    S = [affine(rz(theta), t), affine(rz(-2.0), np.zeros(3))]
    j = np.array([[0, 1, 1, 1]] * 2)
    w = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    out = vs.skin_vertices(method, *one_character(S, p, j, w))
    c, s = np.cos(theta), np.sin(theta)
    ref = np.stack([p[:, 0] * c - p[:, 1] * s, p[:, 0] * s + p[:, 1] * c, p[:, 2]], axis=1) + t
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_common_axis_blend_closed_forms():
    a, b, w = 0.9, -0.4, 0.3
    p = np.array([[1.5, -0.5, 0.2]])
    S = [affine(rz(a), np.zeros(3)), affine(rz(b), np.zeros(3))]
    j = np.array([[0, 1, 0, 0]])
    wt = np.array([[w, 1.0 - w, 0.0, 0.0]])
    args = one_character(S, p, j, wt)
    # linear blend: the weighted mean of the two rotated points
    lbs = w * (rz(a) @ p[0]) + (1 - w) * (rz(b) @ p[0])
    np.testing.assert_allclose(vs.linear_blend(*args)[0], lbs, atol=1e-12)
    # dual quaternions: one rotation about z by the angle of the normalised
    # quaternion blend
    phi = 2.0 * np.arctan2(w * np.sin(a / 2) + (1 - w) * np.sin(b / 2), w * np.cos(a / 2) + (1 - w) * np.cos(b / 2))
    np.testing.assert_allclose(vs.dual_quaternion(*args)[0], rz(phi) @ p[0], atol=1e-12)


def test_twisting_joint_collapses_under_linear_blend_only():
    """Two influences twisted by +theta and -theta about x, half weight
    each: linear blend pulls a vertex at radius r to r cos(theta) from the
    axis; dual quaternions keep it at r (the blended rotation is the
    identity)."""
    th, r = 1.2, 0.8
    Rx = lambda a: Rotation.from_rotvec([a, 0.0, 0.0]).as_matrix()
    S = [affine(Rx(th), np.zeros(3)), affine(Rx(-th), np.zeros(3))]
    p = np.array([[0.4, r, 0.0]])
    args = one_character(S, p, np.array([[0, 1, 0, 0]]), np.array([[0.5, 0.5, 0.0, 0.0]]))
    np.testing.assert_allclose(vs.linear_blend(*args)[0], [0.4, r * np.cos(th), 0.0], atol=1e-12)
    np.testing.assert_allclose(vs.dual_quaternion(*args)[0], [0.4, r, 0.0], atol=1e-12)


def test_antipodal_quaternions_take_the_short_way():
    """Rotations of +170 and -170 degrees about z lie on opposite sides of
    the quaternion sphere; with the sign rule their even blend is the
    180-degree rotation (without it, the identity)."""
    a = np.deg2rad(170.0)
    S = [affine(rz(a), np.zeros(3)), affine(rz(-a), np.zeros(3))]
    p = np.array([[1.0, 0.5, -0.3]])
    args = one_character(S, p, np.array([[0, 1, 0, 0]]), np.array([[0.5, 0.5, 0.0, 0.0]]))
    np.testing.assert_allclose(vs.dual_quaternion(*args)[0], [-1.0, -0.5, -0.3], atol=1e-12)


def test_dual_quaternion_blend_is_rigid_and_weight_scale_free():
    rng = np.random.default_rng(2)
    S = [affine(Rotation.random(random_state=k).as_matrix(), rng.uniform(-1, 1, 3)) for k in range(4)]
    p = rng.uniform(-1, 1, (30, 3))
    w = np.tile(rng.dirichlet(np.ones(4)), (30, 1))
    j = np.tile(np.arange(4), (30, 1))
    out = vs.dual_quaternion(*one_character(S, p, j, w))
    d0 = np.linalg.norm(p[:, None] - p[None], axis=2)
    d1 = np.linalg.norm(out[:, None] - out[None], axis=2)
    np.testing.assert_allclose(d1, d0, atol=1e-12)
    out2 = vs.dual_quaternion(*one_character(S, p, j, 3.0 * w))
    np.testing.assert_allclose(out2, out, atol=1e-12)
    # a single influence reproduces the matrix itself
    one = np.zeros_like(w)
    one[:, 2] = 1.0
    out3 = vs.dual_quaternion(*one_character(S, p, j, one))
    np.testing.assert_allclose(out3, p @ S[2][:3, :3].T + S[2][:3, 3], atol=1e-12)


def test_batch_layout_shared_mesh_rows_and_empty_characters():
    """Characters 0 and 2 share mesh rows, character 1 has no vertices;
    joint ids are character-local."""
    rng = np.random.default_rng(3)
    offsets = np.array([0, 3, 5, 8])
    S = np.stack([affine(np.eye(3), rng.uniform(-1, 1, 3)) for _ in range(8)])
    pos = rng.uniform(-1, 1, (4, 3))
    joints = np.array([[0, 1, 2, 0], [2, 2, 2, 2], [1, 0, 0, 0], [0, 1, 2, 1]], np.int32)
    weights = rng.dirichlet(np.ones(4), 4)
    vo = np.array([0, 4, 4, 8])
    mf = np.array([0, 0, 0])
    out = vs.linear_blend(offsets, S, vo, mf, pos, joints, weights)
    for c, base in ((0, 0), (2, 5)):
        t = S[base + joints.astype(np.int64), :3, 3]  # [4 rows, 4 influences, 3]
        ref = pos + np.einsum("vk,vka->va", weights, t)
        np.testing.assert_allclose(out[vo[c]:vo[c + 1]], ref, atol=1e-12)

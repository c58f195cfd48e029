"""The oracle against hand-derived worked examples (tests/golden/
worked_examples.json): a five-joint tree of quarter turns with a fork and a
scaled joint (Eq. 1), and a key interpolation at alpha = 0.5 whose result
is the half-angle rotation (the Simulation step).  The expected values come
from the definitions by exact arithmetic, not from any implementation; no
GPU."""
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def forward_inputs(fx):
    f32 = lambda k: np.asarray(fx[k], np.float32)
    return np.array([0, len(fx["parents"])], np.int64), np.asarray(fx["parents"], np.int32), f32("quat"), \
        f32("trans"), f32("scale")


def sampler_inputs(sx):
    kq = np.stack([sx["key_quat_clip_a"], sx["key_quat_clip_b"]]).astype(np.float32)[:, :, None, :]
    kt = np.stack([sx["key_trans_clip_a"], sx["key_trans_clip_b"]]).astype(np.float32)[:, :, None, :]
    return (np.array([0, 1], np.int64), kq, kt, np.array([0], np.int32), np.array([1], np.int32),
            np.array([sx["time"]], np.float32), np.array([sx["weight"]], np.float32), sx["fps"])


def test_oracle_forward_matches_the_worked_tree():
    fx = load()["forward"]
    G = oracle.forward(*forward_inputs(fx))
    np.testing.assert_allclose(G[:, :3, :], np.asarray(fx["global_rows_0_2"], np.float64), atol=1e-6)
    np.testing.assert_array_equal(G[:, 3, :], np.tile([0.0, 0.0, 0.0, 1.0], (G.shape[0], 1)))


def test_oracle_sampler_matches_the_half_angle_example():
    sx = load()["sampler"]
    q, t = oracle.pose_sample(*sampler_inputs(sx))
    np.testing.assert_allclose(q[0], sx["quat"], atol=1e-6)
    np.testing.assert_allclose(t[0], sx["trans"], atol=1e-6)

"""The HIP path (hs_scan_forward, hs_pose_sample) against the hand-derived
worked examples of tests/golden/worked_examples.json; tolerances as for the
oracle (1e-6 on these unit-sized values: the only rounding is that of the
fp32 inputs and of a few fp32 operations)."""
import numpy as np
import pytest
import torch

from paper_2505_06703_amd import hs
from test_golden_worked_examples import forward_inputs, load, sampler_inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_forward_matches_the_worked_tree():
    fx = load()["forward"]
    off, par, q, t, s = forward_inputs(fx)
    plan = hs.Plan(off, par)
    G, _ = hs.hs_scan_forward(plan, dev(q), dev(t), dev(s))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    np.testing.assert_allclose(G[:, :3, :], np.asarray(fx["global_rows_0_2"], np.float32), atol=1e-6)
    np.testing.assert_array_equal(G[:, 3, :], np.tile(np.float32([0, 0, 0, 1]), (G.shape[0], 1)))


def test_sampler_matches_the_half_angle_example():
    sx = load()["sampler"]
    off, kq, kt, ca, cb, tm, wt, fps = sampler_inputs(sx)
    plan = hs.Plan(off, np.array([-1], np.int32))
    lib = hs.ClipLibrary(dev(kq), dev(kt), fps)
    q, t = hs.hs_pose_sample(plan, lib, dev(ca), dev(cb), dev(tm), dev(wt))
    torch.cuda.synchronize()
    np.testing.assert_allclose(q.cpu().numpy()[0], sx["quat"], atol=1e-6)
    np.testing.assert_allclose(t.cpu().numpy()[0], sx["trans"], atol=1e-6)

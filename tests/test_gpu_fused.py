"""GPU parity of the Simulation step (standalone and fused into the scan)
against the FP64 oracle's sampler followed by its scan and skin."""
import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

from parity import check_global, check_skin

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def clip_inputs(b):
    x = b.extra
    return (hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"]),
            dict(clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]), time=dev(x["time"]), weight=dev(x["weight"])))


def oracle_sample(b):
    x = b.extra
    return oracle.pose_sample(b.offsets, x["key_quat"], x["key_trans"], x["clip_a"], x["clip_b"], x["time"],
                              x["weight"], x["fps"])


def inv_binds(b):
    G = oracle.forward(b.offsets, b.parents, b.rest_quat, b.rest_trans, b.rest_scale)
    return np.linalg.inv(G).astype(np.float32)


def test_pose_sample_matches_oracle():
    b = wl.fused_sample(num_characters=200)
    lib, cp = clip_inputs(b)
    plan = hs.Plan(b.offsets, b.parents)
    q, t = hs.hs_pose_sample(plan, lib, **cp)
    qr, tr = oracle_sample(b)
    np.testing.assert_allclose(q.cpu().numpy(), qr, rtol=0, atol=2e-6)
    np.testing.assert_allclose(t.cpu().numpy(), tr, rtol=0, atol=2e-6)


@pytest.mark.parametrize("shape", [dict(), dict(tile_joints=256, waves_per_tile=4), dict(chain_units=True),
                                   dict(strategy=hs.HS_STRATEGY_MULTIPASS)])
def test_fused_sample_scan_skin(shape):
    b = wl.fused_sample(num_characters=64)
    lib, cp = clip_inputs(b)
    inv = inv_binds(b)
    plan = hs.Plan(b.offsets, b.parents, **shape)
    G, S = hs.hs_scan_forward(plan, clips=lib, **cp, inv_bind=dev(inv))
    qr, tr = oracle_sample(b)
    Gr = oracle.forward(b.offsets, b.parents, qr, tr, None)
    lam = oracle.path_length(b.offsets, b.parents, Gr, tr)
    check_global(G.cpu().numpy(), Gr, lam, f"fused {shape}")
    check_skin(S.cpu().numpy(), Gr, inv, lam, f"fused skin {shape}")


def test_fused_full_size_sampled_characters():
    b = wl.fused_sample()
    lib, cp = clip_inputs(b)
    plan = hs.Plan(b.offsets, b.parents)
    G, _ = hs.hs_scan_forward(plan, clips=lib, **cp)
    G = G.cpu().numpy()
    rng = np.random.default_rng(3)
    chars = np.unique(np.concatenate([[0, b.num_characters - 1], rng.choice(b.num_characters, 20, replace=False)]))
    x = b.extra
    ids = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in chars])
    sub_off = np.concatenate([[0], np.cumsum(np.diff(b.offsets)[chars])]).astype(np.int64)
    qr, tr = oracle.pose_sample(sub_off, x["key_quat"], x["key_trans"], x["clip_a"][chars], x["clip_b"][chars],
                                x["time"][chars], x["weight"][chars], x["fps"])
    Gr = oracle.forward(sub_off, b.parents[ids], qr, tr, None)
    lam = oracle.path_length(sub_off, b.parents[ids], Gr, tr)
    check_global(G[ids], Gr, lam, "fused full (sampled)")


def test_sampler_edge_times_and_bad_clip_ids():
    b = wl.fused_sample(num_characters=6)
    x = b.extra
    tm = np.array([0.0, np.nextafter(np.float32(1), np.float32(0)), 1.25, -0.4, 7.0, 0.5], np.float32)
    x["time"] = tm
    lib, cp = clip_inputs(b)
    plan = hs.Plan(b.offsets, b.parents)
    q, t = hs.hs_pose_sample(plan, lib, **cp)
    qr, tr = oracle_sample(b)
    np.testing.assert_allclose(q.cpu().numpy(), qr, atol=2e-6)
    np.testing.assert_allclose(t.cpu().numpy(), tr, atol=2e-6)
    # an out-of-range clip id yields NaN poses for that character only
    bad = x["clip_a"].copy()
    bad[2] = 999
    cp["clip_a"] = dev(bad)
    q, t = hs.hs_pose_sample(plan, lib, **cp)
    q = q.cpu().numpy()
    sl = slice(b.offsets[2], b.offsets[3])
    assert np.isnan(q[sl]).all() and np.isfinite(np.delete(q, np.arange(sl.start, sl.stop), axis=0)).all()

"""The allocation-free variant of the sampler's reverse mode
(hs_pose_sample_backward_noalloc): its workspace is the library's static
device array instead of caller memory, and its results equal those of
hs_pose_sample_backward with a caller workspace, bit for bit (the same
kernels in the same order).  Two calls in a row, the second on a smaller
batch, check that nothing of the first call's contents leaks into the
second; sizes beyond the array are rejected before any launch.
"""
import numpy as np
import pytest
import torch

from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def case(num_characters, seed):
    b = wl.fused_sample(num_characters=num_characters, seed=seed)
    x = b.extra
    plan = hs.Plan(b.offsets, b.parents)
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    params = (dev(x["clip_a"]), dev(x["clip_b"]), dev(x["time"]), dev(x["weight"]))
    rng = np.random.default_rng(seed + 100)
    gq = dev(rng.standard_normal((b.num_joints, 4)).astype(np.float32))
    gt = dev(rng.standard_normal((b.num_joints, 3)).astype(np.float32))
    return plan, lib, params, gq, gt


def both(plan, lib, params, gq, gt):
    ws = hs.sample_backward_workspace(plan, DEV)
    ref = hs.hs_pose_sample_backward(plan, lib, *params, gq, gt, workspace=ws)
    got = hs.hs_pose_sample_backward_noalloc(plan, lib, *params, gq, gt)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_matches_the_workspace_route_twice():
    for num_characters, seed in ((600, 3), (150, 11)):  # the second call is smaller
        plan, lib, params, gq, gt = case(num_characters, seed)
        ref, got = both(plan, lib, params, gq, gt)
        for r, g in zip(ref, got):
            assert r.shape == g.shape
            assert torch.equal(r, g)
        assert bool(torch.isfinite(got[0]).all())


def test_noalloc_rejects_batches_beyond_the_static_array():
    cap = hs.HS_NOALLOC_MAX_JOINTS
    n = 256
    C = cap // n + 1  # one character more than the array holds
    offsets = np.arange(C + 1, dtype=np.int64) * n
    parents = np.tile(np.arange(-1, n - 1, dtype=np.int32), C)
    plan = hs.Plan(offsets, parents)
    b = wl.fused_sample(num_characters=4)
    x = b.extra
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    zeros_i = torch.zeros(C, dtype=torch.int32, device=DEV)
    zeros_f = torch.zeros(C, dtype=torch.float32, device=DEV)
    gq = torch.zeros((plan.num_joints, 4), device=DEV)
    gt = torch.zeros((plan.num_joints, 3), device=DEV)
    with pytest.raises(hs.HSError) as ei:
        hs.hs_pose_sample_backward_noalloc(plan, lib, zeros_i, zeros_i, zeros_f, zeros_f, gq, gt)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    assert "static" in str(ei.value)

"""The plan's device status word (include/hs.h: hs_plan_status,
HS_FLAG_VALIDATE, hs_plan_set_wait_limit).

The scan's blocks wait only for earlier blocks because every parent precedes
its children (the traversal ordering of the paper's Sec. 3.2.1).  The error
paths are forced from the host so that every kernel still runs to its end:
a wait limit of zero polls makes every wait that is needed at all give up
at once, and a debug write puts a self-parent into the plan's device parent
table, which the validating calls detect before any scan work is done.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl
from parity import check_global, reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SENTINEL = 7.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def pose(b):
    return dev(b.quat), dev(b.trans), dev(b.scale)


def chained():
    """Eight 1024-joint characters whose chains span blocks: most blocks
    need an earlier block's transforms."""
    return wl.deep_forward(num_characters=8)


@pytest.mark.parametrize("strategy", [hs.HS_STRATEGY_AUTO, hs.HS_STRATEGY_MULTIPASS])
def test_validating_calls_on_a_sound_plan(strategy):
    """A clean plan: the validating forward and adjoint write what the plain
    calls write, bit for bit, and the status word stays clear."""
    b = chained()
    plan = hs.Plan(b.offsets, b.parents, strategy=strategy)
    q, t, s = pose(b)
    G0, _ = hs.hs_scan_forward(plan, q, t, s)
    G1, _ = hs.hs_scan_forward(plan, q, t, s, validate=True)
    W = dev(np.random.default_rng(1).standard_normal((b.num_joints, 4, 4)).astype(np.float32))
    g0 = hs.hs_scan_backward(plan, q, t, s, W)
    g1 = hs.hs_scan_backward(plan, q, t, s, W, validate=True)
    rc, bits, joint = plan.status()
    assert (rc, bits, joint) == (hs.HS_OK, 0, -1)
    assert torch.equal(G0, G1)
    Gr, lam, _ = reference(b)
    check_global(G1.cpu().numpy(), Gr, lam, "validated forward")
    # the adjoint adds colliding pushes with float atomics (not bitwise
    # reproducible): both calls against the oracle's reverse mode
    ref = oracle.backward(b.offsets, b.parents, b.quat, b.trans, b.scale, W.cpu().numpy())
    for grads, what in ((g0, "plain"), (g1, "validated")):
        for g, r in zip(grads, ref):
            tol = 1e-4 * max(1.0, float(np.abs(r).max()))
            assert float(np.abs(g.cpu().numpy() - r).max()) <= tol, what


def test_wait_limit_zero_forward_records_timeout_then_recovers():
    b = chained()
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = pose(b)
    plan.set_wait_limit(0)
    hs.hs_scan_forward(plan, q, t, s)
    rc, bits, _ = plan.status()
    assert rc == hs.HS_ERR_DEVICE and bits & hs.HS_DEV_WAIT_TIMEOUT
    assert "bounded wait" in hs.load_library().hs_last_error().decode()
    # the word keeps the bit until cleared
    assert plan.status(clear=True)[1] & hs.HS_DEV_WAIT_TIMEOUT
    assert plan.status() == (hs.HS_OK, 0, -1)
    plan.set_wait_limit(1 << 22)
    G, _ = hs.hs_scan_forward(plan, q, t, s)
    assert plan.status() == (hs.HS_OK, 0, -1)
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "forward after the wait limit is restored")


def test_single_block_characters_never_wait():
    """Characters of at most 64 joints have no cross-block dependency: even
    a zero wait limit records nothing and the result is right."""
    b = wl.plain_scan(num_characters=32)
    plan = hs.Plan(b.offsets, b.parents)
    plan.set_wait_limit(0)
    G, _ = hs.hs_scan_forward(plan, *pose(b))
    assert plan.status() == (hs.HS_OK, 0, -1)
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, "one-block characters, zero wait limit")


def test_wait_limit_zero_dataflow_adjoint_records_timeout():
    b = chained()
    plan = hs.Plan(b.offsets, b.parents, adjoint=hs.HS_ADJ_DATAFLOW)
    q, t, s = pose(b)
    W = dev(np.zeros((b.num_joints, 4, 4), np.float32))
    plan.set_wait_limit(0)
    hs.hs_scan_backward(plan, q, t, s, W)
    rc, bits, _ = plan.status(clear=True)
    assert rc == hs.HS_ERR_DEVICE and bits & hs.HS_DEV_WAIT_TIMEOUT


def test_wait_limit_zero_effector_step_records_timeout():
    b = wl.differentiable(num_characters=4)
    plan = hs.Plan(b.offsets, b.parents)
    eff = hs.Effectors(plan, b.extra["effectors"])
    assert eff.sparse
    q, t, s = pose(b)
    y = dev(np.zeros((eff.num_effectors, 3), np.float32))
    plan.set_wait_limit(0)
    hs.hs_effector_step(plan, eff, q, t, s, y)
    rc, bits, _ = plan.status(clear=True)
    assert rc == hs.HS_ERR_DEVICE and bits & hs.HS_DEV_WAIT_TIMEOUT
    eff.close()


@pytest.mark.parametrize("strategy", [hs.HS_STRATEGY_AUTO, hs.HS_STRATEGY_MULTIPASS])
def test_validate_detects_a_broken_parent_and_writes_nothing(strategy):
    b = chained()
    plan = hs.Plan(b.offsets, b.parents, strategy=strategy)
    q, t, s = pose(b)
    bad = int(b.offsets[3]) + 700  # a chain joint of character 3
    plan.debug_break_parent(bad)
    G = torch.full((b.num_joints, 4, 4), SENTINEL, device=DEV)
    hs.hs_scan_forward(plan, q, t, s, global_out=G, validate=True)
    rc, bits, joint = plan.status()
    assert rc == hs.HS_ERR_DEVICE
    assert bits == hs.HS_DEV_TOPOLOGY and joint == bad
    assert "topology" in hs.load_library().hs_last_error().decode()
    assert bool((G == SENTINEL).all())
    W = dev(np.ones((b.num_joints, 4, 4), np.float32))
    gq = torch.full((b.num_joints, 4), SENTINEL, device=DEV)
    gt = torch.full((b.num_joints, 3), SENTINEL, device=DEV)
    hs.hs_scan_backward(plan, q, t, s, W, want_scale=False, grad_quat=gq, grad_trans=gt, validate=True)
    rc, bits, joint = plan.status(clear=True)
    assert bits == hs.HS_DEV_TOPOLOGY and joint == bad
    assert bool((gq == SENTINEL).all()) and bool((gt == SENTINEL).all())
    plan.close()


def test_unknown_flags_are_rejected():
    b = wl.plain_scan(num_characters=2)
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = pose(b)
    src = hs._trs_src(plan, q, t, s)
    G = torch.empty((b.num_joints, 4, 4), device=DEV)
    lib = hs.load_library()
    rc = lib.hs_scan_forward(plan.handle, ctypes.byref(src), hs._ptr(G), None, None, None, 0, 4, hs._stream())
    assert rc == hs.HS_ERR_INVALID_ARG
    W = torch.zeros((b.num_joints, 4, 4), device=DEV)
    gq = torch.empty((b.num_joints, 4), device=DEV)
    gt = torch.empty((b.num_joints, 3), device=DEV)
    rc = lib.hs_scan_backward(plan.handle, ctypes.byref(src), hs._ptr(W), None, 0, hs._ptr(gq), hs._ptr(gt), None,
                              2, hs._stream())
    assert rc == hs.HS_ERR_INVALID_ARG

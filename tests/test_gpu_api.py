"""GPU tests of the C-ABI's error handling, HIP-graph capture and plan
bookkeeping.  Every call goes through the C ABI; invalid inputs are caught
on the host before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def status_of(fn, *a, **kw):
    try:
        fn(*a, **kw)
    except hs.HSError as e:
        return e.status
    return hs.HS_OK


def test_topology_and_offsets_are_validated():
    assert status_of(hs.Plan, np.array([0, 3]), np.array([-1, 1, 0], np.int32)) == hs.HS_ERR_TOPOLOGY
    assert status_of(hs.Plan, np.array([0, 3]), np.array([-1, -5, 0], np.int32)) == hs.HS_ERR_TOPOLOGY
    assert status_of(hs.Plan, np.array([0, 2, 1, 3]), np.array([-1, 0, -1], np.int32)) == hs.HS_ERR_INVALID_ARG
    assert status_of(hs.Plan, np.array([1, 3]), np.array([-1, 0, 0], np.int32)) == hs.HS_ERR_INVALID_ARG
    assert status_of(hs.Plan, np.array([0, 2]), np.array([-1, 0, 1], np.int32)) == hs.HS_ERR_INVALID_ARG
    assert status_of(hs.Plan, np.array([0, 3]), np.array([-1, 0, 1], np.int32), tile_joints=100) == hs.HS_ERR_INVALID_ARG
    assert status_of(hs.Plan, np.array([0, 3]), np.array([-1, 0, 1], np.int32), waves_per_tile=3) == hs.HS_ERR_INVALID_ARG
    big = np.arange(-1, 4999, dtype=np.int32)
    assert status_of(hs.Plan, np.array([0, 5000]), big, strategy=hs.HS_STRATEGY_TILE) == hs.HS_ERR_UNSUPPORTED


def test_plan_accepts_device_topology():
    b = wl.plain_scan(num_characters=4)
    p1 = hs.Plan(b.offsets, b.parents)
    lib = hs.load_library()
    off, par = dev(b.offsets), dev(b.parents)
    batch = hs.hs_batch(4, b.num_joints, off.data_ptr(), par.data_ptr())
    h = ctypes.c_void_p()
    assert lib.hs_plan_create(p1.ctx.handle, ctypes.byref(batch), None, ctypes.byref(h)) == hs.HS_OK
    info = hs.hs_plan_info()
    assert lib.hs_plan_get_info(h, ctypes.byref(info)) == hs.HS_OK
    assert info.num_joints == b.num_joints and info.max_depth == p1.info["max_depth"]
    lib.hs_plan_destroy(h)


def _call_forward(plan, q, t, s, G, inv=None, S=None, ckpt=None, k=0, flags=0):
    src = hs.hs_pose_src(hs.HS_POSE_TRS, q, t, s, None, None)
    return hs.load_library().hs_scan_forward(plan.handle, ctypes.byref(src), G, inv, S, ckpt, k, flags,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_forward_argument_errors_launch_nothing():
    b = wl.plain_scan(num_characters=2)
    plan = hs.Plan(b.offsets, b.parents)
    N = b.num_joints
    q, t = dev(b.quat), dev(b.trans)
    G = torch.full((N + 1, 4, 4), 7.0, device=DEV)
    qp, tp, Gp = q.data_ptr(), t.data_ptr(), G.data_ptr()
    assert _call_forward(plan, None, tp, None, Gp) == hs.HS_ERR_INVALID_ARG          # NULL quat
    assert _call_forward(plan, qp, tp, None, None) == hs.HS_ERR_INVALID_ARG          # no output
    assert _call_forward(plan, qp + 4, tp, None, Gp) == hs.HS_ERR_INVALID_ARG        # misaligned quat
    assert _call_forward(plan, qp, tp, None, Gp + 4) == hs.HS_ERR_INVALID_ARG        # misaligned output
    assert _call_forward(plan, qp, tp, None, qp) == hs.HS_ERR_INVALID_ARG            # output aliases input
    assert _call_forward(plan, qp, tp, None, Gp, flags=4) == hs.HS_ERR_INVALID_ARG   # unknown flags
    assert _call_forward(plan, qp, tp, None, Gp, inv=Gp + 64) == hs.HS_ERR_INVALID_ARG  # inv without skin
    ck = torch.empty((N, 12), device=DEV)
    assert _call_forward(plan, qp, tp, None, Gp, ckpt=ck.data_ptr(), k=0) == hs.HS_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(G == 7.0), "a rejected call must not write"
    assert _call_forward(plan, qp, tp, None, Gp) == hs.HS_OK


def test_unknown_adjoint_kernel_is_rejected():
    b = wl.plain_scan(num_characters=2)
    with pytest.raises(hs.HSError) as ei:
        hs.Plan(b.offsets, b.parents, adjoint=4)  # 0-3 are the kernels of HS_ADJ_*
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    with pytest.raises(hs.HSError) as ei:
        hs.Plan(b.offsets, b.parents, adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=3)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    for bpw in (1, 2):  # asked for: reported
        p = hs.Plan(b.offsets, b.parents, adjoint=hs.HS_ADJ_ANCHORS, adjoint_blocks_per_wave=bpw)
        assert p.info["adjoint_blocks_per_wave"] == bpw


def test_backward_and_sampler_argument_errors():
    b = wl.fused_sample(num_characters=3)
    plan = hs.Plan(b.offsets, b.parents)
    x = b.extra
    lib = hs.ClipLibrary(dev(x["key_quat"][:, :, :100]), dev(x["key_trans"][:, :, :100]))
    with pytest.raises(hs.HSError) as ei:  # clips shorter than the characters
        hs.hs_pose_sample(plan, lib, dev(x["clip_a"]), dev(x["clip_b"]), dev(x["time"]), dev(x["weight"]))
    assert ei.value.status == hs.HS_ERR_INVALID_ARG
    N = b.num_joints
    with pytest.raises(hs.HSError) as ei:
        hs.hs_scan_backward(plan, dev(b.quat), dev(b.trans), None, torch.zeros((N, 4, 4), device=DEV),
                            ckpt=torch.zeros((N, 12), device=DEV), ckpt_k=0)
    assert ei.value.status == hs.HS_ERR_INVALID_ARG


def test_graph_replays_track_input_changes():
    b = wl.deep_forward(num_characters=8)
    plan = hs.Plan(b.offsets, b.parents)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    N = b.num_joints
    G = torch.empty((N, 4, 4), device=DEV)
    g = hs.ForwardGraph(plan, q, t, s, global_out=G)
    rng = np.random.default_rng(0)
    for it in range(4):
        g.launch()
        torch.cuda.synchronize()
        ref, _ = hs.hs_scan_forward(plan, q, t, s)
        torch.cuda.synchronize()
        assert torch.equal(G, ref), f"replay {it}"
        # eager work between replays: new poses in place
        q.copy_(dev(wl.random_quats(rng, N, 0.3)))
        t.mul_(1.01)
    g.close()


def test_graph_of_fused_sample_and_skin():
    b = wl.fused_sample(num_characters=16)
    x = b.extra
    lib = hs.ClipLibrary(dev(x["key_quat"]), dev(x["key_trans"]), x["fps"])
    cp = dict(clip_a=dev(x["clip_a"]), clip_b=dev(x["clip_b"]), time=dev(x["time"]), weight=dev(x["weight"]))
    plan = hs.Plan(b.offsets, b.parents)
    N = b.num_joints
    inv = dev(np.tile(np.eye(4, dtype=np.float32), (N, 1, 1)))
    S = torch.empty((N, 4, 4), device=DEV)
    g = hs.ForwardGraph(plan, clips=lib, **cp, inv_bind=inv, skin_out=S)
    for it in range(3):
        g.launch()
        _, ref = hs.hs_scan_forward(plan, clips=lib, **cp, want_global=False, inv_bind=inv)
        torch.cuda.synchronize()
        assert torch.equal(S, ref), f"replay {it}"
        cp["time"].add_(0.173)


def test_graph_sequence_of_calls_on_several_buffers():
    """hs_graph_create_forward_n: three captured passes over different input
    and output buffers (one of them skin-only), replayed with eager changes
    in between; every output equals its own eager call."""
    b = wl.deep_forward(num_characters=6)
    plan = hs.Plan(b.offsets, b.parents)
    N = b.num_joints
    rng = np.random.default_rng(3)
    ins = [(dev(wl.random_quats(rng, N, 0.3)), dev(b.trans), dev(b.scale)) for _ in range(3)]
    inv = dev(np.tile(np.eye(4, dtype=np.float32), (N, 1, 1)))
    outs = [torch.empty((N, 4, 4), device=DEV) for _ in range(3)]
    calls = [dict(quat=ins[0][0], trans=ins[0][1], scale=ins[0][2], global_out=outs[0]),
             dict(quat=ins[1][0], trans=ins[1][1], scale=None, inv_bind=inv, skin_out=outs[1]),
             dict(quat=ins[2][0], trans=ins[2][1], scale=ins[2][2], global_out=outs[2])]
    g = hs.ForwardGraph.sequence(plan, calls)
    for it in range(3):
        g.launch()
        torch.cuda.synchronize()
        r0, _ = hs.hs_scan_forward(plan, *ins[0])
        _, r1 = hs.hs_scan_forward(plan, ins[1][0], ins[1][1], None, want_global=False, inv_bind=inv)
        r2, _ = hs.hs_scan_forward(plan, *ins[2])
        torch.cuda.synchronize()
        for k, r in enumerate((r0, r1, r2)):
            assert torch.equal(outs[k], r), f"replay {it}, call {k}"
        for q, t, _ in ins:
            q.copy_(dev(wl.random_quats(rng, N, 0.3)))
            t.mul_(0.99)
    g.close()
    with pytest.raises(ValueError):
        hs.ForwardGraph.sequence(plan, [])


def test_plan_info_reports_tiles_and_multipass():
    b = wl.heterogeneous(num_characters=100)
    p = hs.Plan(b.offsets, b.parents, tile_joints=512)
    inf = p.info
    assert inf["tiled_joints"] + inf["multipass_joints"] == b.num_joints
    assert inf["multipass_joints"] == int(np.sum(np.diff(b.offsets)[np.diff(b.offsets) > 512]))
    assert inf["tile_joints"] == 512 and inf["num_tiles"] > 0


def test_stream_probe_moves_the_forward_bytes_verbatim():
    """hs_stream_probe (the bandwidth reference): every input value lands in
    its row of the output, for a ragged size and an exact multiple of 64."""
    rng = np.random.default_rng(9)
    for n in (1, 64, 1000, 4096 + 37):
        q = rng.standard_normal((n, 4)).astype(np.float32)
        t = rng.standard_normal((n, 3)).astype(np.float32)
        s = rng.standard_normal((n, 3)).astype(np.float32)
        tab = rng.integers(-1, 1 << 20, n).astype(np.int32)
        out = hs.hs_stream_probe(dev(q), dev(t), dev(s), dev(tab))
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        ref = np.zeros((n, 4, 4), np.float32)
        ref[:, 0, :3], ref[:, 0, 3] = q[:, :3], t[:, 0]
        ref[:, 1, 0], ref[:, 1, 1:3], ref[:, 1, 3] = q[:, 3], s[:, :2], t[:, 1]
        ref[:, 2, 0], ref[:, 2, 3] = s[:, 2], t[:, 2]
        ref[:, 3, 3] = 1.0
        bits = o[:, 2, 1].view(np.int32).copy()
        o[:, 2, 1] = 0.0
        assert np.array_equal(o, ref), n
        assert np.array_equal(bits, tab), n
    qd = dev(q)  # output overlapping an input: refused, nothing launched
    rc = hs.load_library().hs_stream_probe(n, qd.data_ptr(), dev(t).data_ptr(), dev(s).data_ptr(),
                                           dev(tab).data_ptr(), qd.data_ptr(), None)
    assert rc == hs.HS_ERR_INVALID_ARG


def test_prepared_calls_repeat_the_direct_call():
    """hs.prepare marshals a binding call once; each call() of the result
    issues the same C call: outputs equal the direct call's, and the inputs
    are read at call time (changed in place between calls)."""
    b = wl.differentiable(num_characters=4)
    plan = hs.Plan(b.offsets, b.parents)
    N = b.num_joints
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G = torch.full((N, 4, 4), float("nan"), device=DEV)
    call, (Gout, Sout) = hs.prepare(hs.hs_scan_forward, plan, q, t, s, global_out=G)
    assert Gout is G and Sout is None
    torch.cuda.synchronize()
    assert bool(torch.isnan(G).all())  # preparing issues nothing
    rng = np.random.default_rng(5)
    for it in range(3):
        call()
        ref, _ = hs.hs_scan_forward(plan, q, t, s)
        torch.cuda.synchronize()
        assert torch.equal(G, ref), f"forward call {it}"
        q.copy_(dev(wl.random_quats(rng, N, 0.3)))
    eff = b.extra["effectors"]
    E = hs.Effectors(plan, eff)
    y = dev(rng.standard_normal((eff.size, 3)).astype(np.float32))
    gq, gt = torch.empty((N, 4), device=DEV), torch.empty((N, 3), device=DEV)
    step, _ = hs.prepare(hs.hs_effector_step, plan, E, q, t, s, y, global_out=G, want_scale=False,
                         grad_quat=gq, grad_trans=gt)
    step()
    rq, rt, _ = hs.hs_effector_step(plan, E, q, t, s, y, want_scale=False)
    torch.cuda.synchronize()
    # anchors sum their inflows in arrival order: equal up to rounding
    assert torch.allclose(gq, rq, rtol=1e-5, atol=1e-6) and torch.allclose(gt, rt, rtol=1e-5, atol=1e-6)
    with pytest.raises(ValueError):  # the binding's checks run when preparing
        hs.prepare(hs.hs_scan_forward, plan, q[:-1], t, s)

"""torch.autograd wrappers of the Hierarchy-Scan and of the Simulation step
(forward and reverse-mode kernels of the library).

``hierarchy_scan(plan, quat, trans, scale)`` returns the global transforms
[N,4,4] and is differentiable with respect to the local quaternions (raw
components), translations and scales.  Two memory modes:

* recompute (``ckpt_k=0``): nothing beyond the inputs is kept; the adjoint
  kernel recomputes the global transforms on chip;
* level checkpoints (``ckpt_k=k``): the forward pass also stores the global
  transforms of joints whose level is a multiple of k ([N,12], only those
  rows written) and the adjoint rebuilds the others from them.

``sample_pose(plan, key_quat, key_trans, clip_a, clip_b, time, weight, fps)``
returns the sampled local (quat [N,4], trans [N,3]) and is differentiable
with respect to the keyframes, the clip times and the blend weights
(``hs_pose_sample_backward``), so a loss on the global transforms reaches
the animation parameters through both kernels.
"""
import torch

from . import hs


class HSScan(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, quat, trans, scale, ckpt_k):
        N = plan.num_joints
        G = torch.empty((N, 4, 4), device=quat.device, dtype=torch.float32)
        ckpt = None
        if ckpt_k > 0:
            ckpt = torch.empty((N, 12), device=quat.device, dtype=torch.float32)
        hs.hs_scan_forward(plan, quat, trans, scale, global_out=G, ckpt_out=ckpt, ckpt_k=ckpt_k)
        ctx.plan = plan
        ctx.ckpt_k = ckpt_k
        ctx.has_scale = scale is not None
        empty = torch.empty(0, device=quat.device)
        ctx.save_for_backward(quat, trans, scale if scale is not None else empty,
                              ckpt if ckpt is not None else empty)
        return G

    @staticmethod
    def backward(ctx, grad_G):
        quat, trans, scale, ckpt = ctx.saved_tensors
        scale = scale if ctx.has_scale else None
        ckpt = ckpt if ctx.ckpt_k > 0 else None
        want_scale = ctx.has_scale and ctx.needs_input_grad[3]
        gq, gt, gs = hs.hs_scan_backward(ctx.plan, quat, trans, scale, grad_G.contiguous(), ckpt=ckpt,
                                         ckpt_k=ctx.ckpt_k, want_scale=want_scale)
        return None, gq, gt, gs, None


def hierarchy_scan(plan, quat, trans, scale=None, ckpt_k=0):
    """Differentiable global transforms G_j = G_parent(j) L_j ([N,4,4])."""
    return HSScan.apply(plan, quat, trans, scale, int(ckpt_k))


class HSSample(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, key_quat, key_trans, clip_a, clip_b, time, weight, fps):
        lib = hs.ClipLibrary(key_quat, key_trans, fps)
        q, t = hs.hs_pose_sample(plan, lib, clip_a, clip_b, time, weight)
        ctx.plan, ctx.fps = plan, fps
        ctx.save_for_backward(key_quat, key_trans, clip_a, clip_b, time, weight)
        return q, t

    @staticmethod
    def backward(ctx, grad_q, grad_t):
        key_quat, key_trans, clip_a, clip_b, time, weight = ctx.saved_tensors
        lib = hs.ClipLibrary(key_quat, key_trans, ctx.fps)
        gq = torch.zeros_like(time.new_empty((ctx.plan.num_joints, 4))) if grad_q is None else grad_q.contiguous()
        gt = torch.zeros_like(time.new_empty((ctx.plan.num_joints, 3))) if grad_t is None else grad_t.contiguous()
        want_keys = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        ws = hs.sample_backward_workspace(ctx.plan, time.device) if want_keys else None
        gkq, gkt, gtime, gw = hs.hs_pose_sample_backward(ctx.plan, lib, clip_a, clip_b, time, weight, gq, gt,
                                                         want_keys=want_keys, workspace=ws)
        return None, gkq, gkt, None, None, gtime, gw, None


def sample_pose(plan, key_quat, key_trans, clip_a, clip_b, time, weight, fps=30.0):
    """Differentiable Simulation step: (quat [N,4], trans [N,3])."""
    return HSSample.apply(plan, key_quat, key_trans, clip_a, clip_b, time, weight, float(fps))

"""IK-style optimisation loops on the library's forward and reverse kernels.

Both minimise the squared distance of chosen end effectors to targets,
loss = sum_e |b_e - y_e|^2 with b_e the translation of G_e, by first-order
steps (Adam on the raw parameters); every iteration runs the HIP kernels:

* ``solve_effectors`` moves the local rotations (raw quaternion components,
  renormalised after every step) of a pose.  By default each iteration is
  one ``hs_effector_step`` launch (forward scan and end-effector adjoint per
  tile) when the plan allows it; ``fused=False`` goes through the autograd
  wrappers (forward scan, torch loss, adjoint);
* ``fit_clip_params`` moves each character's clip time and blend weight
  (the weight kept in [0, 1]) so that the sampled pose reaches the targets,
  through the autograd wrappers: sampler, scan, adjoint, the sampler's
  reverse mode.
"""
import torch

from . import hs
from .autograd import hierarchy_scan, sample_pose


def _effector_loss(G, effectors, targets):
    return ((G[effectors, :3, 3] - targets) ** 2).sum()


def solve_effectors(plan, quat, trans, scale, effectors, targets, iters=100, lr=0.02, fused=True):
    """Returns (quat, losses): the optimised unit quaternions [N,4] and the
    loss before each step.  ``effectors``: global joint ids (tensor or
    array), ``targets`` [E,3] on the device."""
    q = quat.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([q], lr=lr)
    losses = []
    eset = hs.Effectors(plan, torch.as_tensor(effectors).cpu().numpy()) if fused else None
    if eset is not None and eset.sparse:
        N = plan.num_joints
        G = torch.empty((N, 4, 4), device=q.device)
        gq = torch.empty((N, 4), device=q.device)
        gt = torch.empty((N, 3), device=q.device)
        eff = torch.as_tensor(effectors, device=q.device)
        for _ in range(iters):
            opt.zero_grad()
            hs.hs_effector_step(plan, eset, q.detach(), trans, scale, targets, global_out=G, want_scale=False,
                                grad_quat=gq, grad_trans=gt)
            losses.append(float(((G[eff, :3, 3] - targets) ** 2).sum()))
            q.grad = gq.clone()
            opt.step()
            with torch.no_grad():
                q /= q.norm(dim=1, keepdim=True)
        return q.detach(), losses
    for _ in range(iters):
        opt.zero_grad()
        loss = _effector_loss(hierarchy_scan(plan, q, trans, scale), effectors, targets)
        losses.append(loss.item())
        loss.backward()
        opt.step()
        with torch.no_grad():
            q /= q.norm(dim=1, keepdim=True)
    return q.detach(), losses


def fit_clip_params(plan, key_quat, key_trans, clip_a, clip_b, time, weight, effectors, targets, fps=30.0,
                    iters=100, lr=0.005):
    """Returns (time, weight, losses) after ``iters`` steps."""
    tau = time.detach().clone().requires_grad_(True)
    w = weight.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([tau, w], lr=lr)
    losses = []
    for _ in range(iters):
        opt.zero_grad()
        q, t = sample_pose(plan, key_quat, key_trans, clip_a, clip_b, tau, w, fps)
        loss = _effector_loss(hierarchy_scan(plan, q, t, None), effectors, targets)
        losses.append(loss.item())
        loss.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(0.0, 1.0)
    return tau.detach(), w.detach(), losses

"""Shared helpers of the parity tests: tolerances and oracle references.

Tolerances (fixed by the method's target accuracy against FP64):
  * rotation-scale blocks: |G_gpu - G_fp64| <= 1e-4 absolute, per entry;
  * translations: |b_gpu - b_fp64|_inf <= 1e-4 * lambda_j + 1e-7, where
    lambda_j is the root-to-joint polyline length of joint j (the sum of
    |A_parent(k) t_k| over the path, from the oracle); the 1e-7 floor is one
    fp32 ulp at unit magnitude so that exact zeros are not demanded of
    values that underflow differently;
  * skin matrices: the same on the 3x3 block; translations within
    1e-4 * (lambda_j + |t_(B^-1)j|) + 1e-7;
  * bottom rows of global matrices: exactly (0, 0, 0, 1).
These bounds hold at every depth the tests run, the 65 536-joint chains
of the multipass benchmark included, except for one stress case: a single
chain of 100 000 joints with rotations of at most 0.02 rad, whose rotation
error reaches 1.35e-4 (fp32 rounding accumulating along the chain), checked
against the bounds scaled by sqrt(depth / 2048) (depth_scale).
"""
import numpy as np

import oracle

TOL = 1e-4
FLOOR = 1e-7


def inverse_binds(batch):
    """Inverse bind matrices from the batch's rest pose: FP64 oracle globals,
    inverted in FP64 and rounded to fp32."""
    G = oracle.forward(batch.offsets, batch.parents, batch.rest_quat, batch.rest_trans, batch.rest_scale)
    return np.linalg.inv(G).astype(np.float32)


def reference(batch, quat=None, trans=None, scale=None, chars=None):
    """FP64 oracle globals and path lengths for all (or the listed) characters.

    Returns (G [M,4,4], lam [M], joint_ids [M]) for the selected joints.
    """
    q = batch.quat if quat is None else quat
    t = batch.trans if trans is None else trans
    s = batch.scale if scale is None else scale
    off = batch.offsets
    if chars is None:
        ids = np.arange(off[-1])
        G = oracle.forward(off, batch.parents, q, t, s)
        lam = oracle.path_length(off, batch.parents, G, t)
        return G, lam, ids
    chars = np.asarray(chars)
    sizes = off[chars + 1] - off[chars]
    ids = np.concatenate([np.arange(off[c], off[c + 1]) for c in chars]) if chars.size else np.zeros(0, np.int64)
    sub_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    par = batch.parents[ids]
    G = oracle.forward(sub_off, par, q[ids], t[ids], None if s is None else s[ids])
    lam = oracle.path_length(sub_off, par, G, t[ids])
    return G, lam, ids


def depth_scale(depth):
    """Tolerance factor of the 100 000-joint stress chain (random-walk
    growth of fp32 rounding beyond 2048 levels)."""
    return max(1.0, float(np.sqrt(depth / 2048.0)))


def check_global(G_gpu, G_ref, lam, what="", scale=1.0):
    tol = TOL * scale
    G_gpu = np.asarray(G_gpu, np.float64)
    assert G_gpu.shape == G_ref.shape, what
    if G_gpu.size == 0:
        return {"rot": 0.0, "trans_rel": 0.0}
    dA = np.abs(G_gpu[:, :3, :3] - G_ref[:, :3, :3])
    db = np.abs(G_gpu[:, :3, 3] - G_ref[:, :3, 3]).max(axis=1)
    lim = tol * lam + FLOOR
    worst = int(np.argmax(db / lim))
    assert np.all(np.isfinite(G_gpu)), f"{what}: non-finite output"
    assert dA.max() <= tol, f"{what}: rotation error {dA.max():.3e} > {tol}"
    assert np.all(db <= lim), (f"{what}: translation error {db[worst]:.3e} > {lim[worst]:.3e} "
                               f"at joint {worst} (lambda {lam[worst]:.3f})")
    bottom = G_gpu[:, 3, :]
    assert np.array_equal(bottom, np.broadcast_to([0.0, 0.0, 0.0, 1.0], bottom.shape)), f"{what}: bottom row"
    return {"rot": float(dA.max()), "trans_rel": float((db / np.maximum(lam, 1e-12)).max())}


def check_skin(S_gpu, G_ref, inv_bind, lam, what=""):
    S_ref = oracle.skin(G_ref, inv_bind)
    S_gpu = np.asarray(S_gpu, np.float64)
    dA = np.abs(S_gpu[:, :3, :3] - S_ref[:, :3, :3]).max() if S_gpu.size else 0.0
    tb = np.linalg.norm(inv_bind[:, :3, 3].astype(np.float64), axis=1)
    db = np.abs(S_gpu[:, :3, 3] - S_ref[:, :3, 3]).max(axis=1)
    assert dA <= TOL, f"{what}: skin rotation error {dA:.3e}"
    assert np.all(db <= TOL * (lam + tb) + FLOOR), f"{what}: skin translation error {db.max():.3e}"
    np.testing.assert_array_equal(S_gpu[:, 3, :], np.asarray(inv_bind[:, 3, :], np.float64))

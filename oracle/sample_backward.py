"""FP64 reverse mode of the Simulation step -- TEST INFRASTRUCTURE ONLY.

The sampler (Sec. 1, step 1; the reading of R15): per character c, frame
f = fps * time_c (in FP64), alpha = f - floor(f), keys
k0 = floor(f) mod K and k1 = k0 + 1 mod K; per clip X in {A, B}
    q_X = normalize((1 - alpha) a + alpha s b),  s = sign(a . b),
    t_X = (1 - alpha) t_a + alpha t_b,
with a, b (t_a, t_b) the clip's keys k0, k1 of the joint; then
    q = normalize((1 - w) q_A + w s' q_B),  s' = sign(q_A . q_B),
    t = (1 - w) t_A + w t_B.
Given dLoss/dq and dLoss/dt of every joint (raw quaternion components),
this returns dLoss/d(key quaternions), dLoss/d(key translations) (summed
over every character and joint that reads a key), dLoss/dtime and
dLoss/dweight per character.  The signs s, s' and floor(f) are held fixed
(the derivative exists away from their switching points); d alpha / d time
= fps.  Reverse rules used: for q = v / |v|, vbar = (qbar - q (q . qbar)) /
|v|; for a lerp (1 - x) a + x b, abar = (1 - x) ybar, bbar = x ybar,
xbar = ybar . (b - a).

Parity status: pinned in tests/test_oracle_sample_backward_pins.py by
central differences of an independent FP64 forward and by torch float64
autograd.
"""
import numpy as np


def _sign(x):
    return np.where(x < 0.0, -1.0, 1.0)


def _norm_back(v, qbar):
    """Adjoint of q = v / |v| (rows)."""
    n = np.linalg.norm(v, axis=-1, keepdims=True)
    q = v / n
    return (qbar - q * np.sum(q * qbar, axis=-1, keepdims=True)) / n


def pose_sample_backward(offsets, key_quat, key_trans, clip_a, clip_b, time, weight, grad_quat, grad_trans,
                         fps=30.0):
    kq32 = np.asarray(key_quat, np.float32)
    kq = kq32.astype(np.float64)
    kt = np.asarray(key_trans, np.float32).astype(np.float64)
    K, T, J = kq.shape[:3]
    gq_all = np.asarray(grad_quat, np.float64)
    gt_all = np.asarray(grad_trans, np.float64)
    g_kq = np.zeros_like(kq)
    g_kt = np.zeros_like(kt)
    C = len(offsets) - 1
    g_time = np.zeros(C)
    g_weight = np.zeros(C)
    for c in range(C):
        n = int(offsets[c + 1] - offsets[c])
        if n == 0:
            continue
        sl = slice(int(offsets[c]), int(offsets[c + 1]))
        f = float(np.float64(np.float32(fps)) * np.float64(np.float32(time[c])))
        fl = np.floor(f)
        alpha = f - fl
        k0 = int(fl) % T
        k1 = (k0 + 1) % T
        w = float(np.float32(weight[c]))
        j = np.arange(n)
        qX, vX, sX, tX = [], [], [], []
        for clip in (int(clip_a[c]), int(clip_b[c])):
            a, b = kq[clip, k0, :n], kq[clip, k1, :n]
            s = _sign(np.sum(kq32[clip, k0, :n].astype(np.float64) * kq32[clip, k1, :n].astype(np.float64), axis=1))
            v = (1 - alpha) * a + alpha * s[:, None] * b
            qX.append(v / np.linalg.norm(v, axis=1, keepdims=True))
            vX.append(v)
            sX.append(s)
            tX.append((1 - alpha) * kt[clip, k0, :n] + alpha * kt[clip, k1, :n])
        sb = _sign(np.sum(qX[0] * qX[1], axis=1))
        u = (1 - w) * qX[0] + w * sb[:, None] * qX[1]
        gq, gt = gq_all[sl], gt_all[sl]
        # blend of the clips
        ubar = _norm_back(u, gq)
        qbar = [(1 - w) * ubar, w * sb[:, None] * ubar]
        tbar = [(1 - w) * gt, w * gt]
        g_weight[c] = np.sum(ubar * (sb[:, None] * qX[1] - qX[0])) + np.sum(gt * (tX[1] - tX[0]))
        # each clip's key interpolation
        abar_total = 0.0
        for X, clip in enumerate((int(clip_a[c]), int(clip_b[c]))):
            a, b = kq[clip, k0, :n], kq[clip, k1, :n]
            vbar = _norm_back(vX[X], qbar[X])
            np.add.at(g_kq, (clip, k0, j), (1 - alpha) * vbar)
            np.add.at(g_kq, (clip, k1, j), alpha * sX[X][:, None] * vbar)
            np.add.at(g_kt, (clip, k0, j), (1 - alpha) * tbar[X])
            np.add.at(g_kt, (clip, k1, j), alpha * tbar[X])
            abar_total += np.sum(vbar * (sX[X][:, None] * b - a))
            abar_total += np.sum(tbar[X] * (kt[clip, k1, :n] - kt[clip, k0, :n]))
        g_time[c] = fps * abar_total
    return g_kq, g_kt, g_time, g_weight

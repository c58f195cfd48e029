"""Pins of the sampler's FP64 reverse mode (oracle/sample_backward.py):
central differences and torch float64 autograd of forwards written here
independently, and closed forms at the special points; no GPU."""
import numpy as np
import pytest
import torch

from oracle.sample_backward import pose_sample_backward
from paper_2505_06703_amd import workloads as wl

FPS = 30.0


def setup(seed=0, C=3, n=5, clips=4, keys=6):
    rng = np.random.default_rng(seed)
    kq = wl.random_quats(rng, clips * keys * n, 0.6).reshape(clips, keys, n, 4).astype(np.float64)
    kt = wl.random_offsets(rng, clips * keys * n).reshape(clips, keys, n, 3).astype(np.float64)
    ca = rng.integers(0, clips, C).astype(np.int32)
    cb = ((ca + rng.integers(1, clips, C)) % clips).astype(np.int32)
    # times inside a key interval, away from its ends (finite differences
    # must not cross a key), weights in (0, 1)
    tau = ((rng.integers(0, keys, C) + rng.uniform(0.2, 0.8, C)) / FPS).astype(np.float32).astype(np.float64)
    w = rng.uniform(0.1, 0.9, C).astype(np.float32).astype(np.float64)
    offsets = np.arange(C + 1) * n
    gq = rng.standard_normal((C * n, 4))
    gt = rng.standard_normal((C * n, 3))
    return offsets, kq, kt, ca, cb, tau, w, gq, gt


def forward_np(offsets, kq, kt, ca, cb, tau, w, fps=FPS):
    """The sampler in float64 (no fp32 rounding of the frame position)."""
    T = kq.shape[1]
    out_q, out_t = [], []
    for c in range(len(offsets) - 1):
        n = offsets[c + 1] - offsets[c]
        f = fps * tau[c]
        k0 = int(np.floor(f)) % T
        k1 = (k0 + 1) % T
        al = f - np.floor(f)
        qs, ts = [], []
        for clip in (ca[c], cb[c]):
            a, b = kq[clip, k0, :n], kq[clip, k1, :n]
            s = np.where(np.sum(a * b, axis=1) < 0, -1.0, 1.0)[:, None]
            v = (1 - al) * a + al * s * b
            qs.append(v / np.linalg.norm(v, axis=1, keepdims=True))
            ts.append((1 - al) * kt[clip, k0, :n] + al * kt[clip, k1, :n])
        s2 = np.where(np.sum(qs[0] * qs[1], axis=1) < 0, -1.0, 1.0)[:, None]
        u = (1 - w[c]) * qs[0] + w[c] * s2 * qs[1]
        out_q.append(u / np.linalg.norm(u, axis=1, keepdims=True))
        out_t.append((1 - w[c]) * ts[0] + w[c] * ts[1])
    return np.concatenate(out_q), np.concatenate(out_t)


def loss(args, gq, gt):
    q, t = forward_np(*args)
    return float(np.sum(q * gq) + np.sum(t * gt))


def test_central_differences():
    offsets, kq, kt, ca, cb, tau, w, gq, gt = setup()
    g_kq, g_kt, g_tau, g_w = pose_sample_backward(offsets, kq, kt, ca, cb, tau, w, gq, gt, FPS)
    h = 1e-6
    base = [offsets, kq, kt, ca, cb, tau, w]

    def fd(idx, where):
        plus = [a.copy() if isinstance(a, np.ndarray) else a for a in base]
        minus = [a.copy() if isinstance(a, np.ndarray) else a for a in base]
        plus[idx][where] += h
        minus[idx][where] -= h
        return (loss(plus, gq, gt) - loss(minus, gq, gt)) / (2 * h)

    for c in range(3):
        assert abs(fd(5, c) - g_tau[c]) <= 1e-5 * max(1.0, abs(g_tau[c])), f"time {c}"
        assert abs(fd(6, c) - g_w[c]) <= 1e-6 * max(1.0, abs(g_w[c])), f"weight {c}"
    rng = np.random.default_rng(9)
    used = [(ca[0], int(np.floor(FPS * tau[0])) % 6), (cb[1], (int(np.floor(FPS * tau[1])) + 1) % 6)]
    for clip, key in used:
        for j in range(5):
            for k in range(4):
                assert abs(fd(1, (clip, key, j, k)) - g_kq[clip, key, j, k]) <= 1e-6, (clip, key, j, k)
            for k in range(3):
                assert abs(fd(2, (clip, key, j, k)) - g_kt[clip, key, j, k]) <= 1e-6, (clip, key, j, k)
    # keys nobody reads have no gradient
    read = np.zeros(kq.shape[:2], bool)
    for c in range(3):
        k0 = int(np.floor(FPS * tau[c])) % 6
        for clip in (ca[c], cb[c]):
            read[clip, k0] = read[clip, (k0 + 1) % 6] = True
    assert np.all(g_kq[~read] == 0.0) and np.all(g_kt[~read] == 0.0)
    del rng


def test_torch_autograd_of_an_independent_forward():
    offsets, kq, kt, ca, cb, tau, w, gq, gt = setup(seed=1, C=4, n=7)
    g = pose_sample_backward(offsets, kq, kt, ca, cb, tau, w, gq, gt, FPS)
    tkq = torch.tensor(kq, requires_grad=True)
    tkt = torch.tensor(kt, requires_grad=True)
    ttau = torch.tensor(tau, requires_grad=True)
    tw = torch.tensor(w, requires_grad=True)
    T = kq.shape[1]
    total = torch.zeros((), dtype=torch.float64)
    for c in range(len(offsets) - 1):
        n = offsets[c + 1] - offsets[c]
        # the frame position f = fps * tau in float64; floor(f) is held
        # fixed, so d alpha / d time = fps
        f = FPS * ttau[c]
        fl = float(np.floor(FPS * tau[c]))
        k0 = int(fl) % T
        k1 = (k0 + 1) % T
        al = f - fl
        qs, ts = [], []
        for clip in (ca[c], cb[c]):
            a, b = tkq[clip, k0, :n], tkq[clip, k1, :n]
            s = torch.where((a * b).sum(1, keepdim=True) < 0, -1.0, 1.0).double().detach()
            v = (1 - al) * a + al * s * b
            qs.append(v / v.norm(dim=1, keepdim=True))
            ts.append((1 - al) * tkt[clip, k0, :n] + al * tkt[clip, k1, :n])
        s2 = torch.where((qs[0] * qs[1]).sum(1, keepdim=True) < 0, -1.0, 1.0).double().detach()
        u = (1 - tw[c]) * qs[0] + tw[c] * s2 * qs[1]
        q = u / u.norm(dim=1, keepdim=True)
        t = (1 - tw[c]) * ts[0] + tw[c] * ts[1]
        sl = slice(offsets[c], offsets[c + 1])
        total = total + (q * torch.tensor(gq[sl])).sum() + (t * torch.tensor(gt[sl])).sum()
    total.backward()
    for mine, ref in zip(g, (tkq.grad, tkt.grad, ttau.grad, tw.grad)):
        np.testing.assert_allclose(mine, ref.numpy(), atol=1e-10, rtol=1e-10)


def test_special_points():
    """w = 0: clip B's keys get no gradient; time on a key (alpha = 0): the
    next key gets none; one joint, translations only: the closed form."""
    offsets, kq, kt, ca, cb, tau, w, gq, gt = setup(seed=2, C=1, n=3)
    w0 = np.zeros(1)
    g_kq, g_kt, _, _ = pose_sample_backward(offsets, kq, kt, ca, cb, tau, w0, gq, gt, FPS)
    assert np.all(g_kq[cb[0]] == 0.0) and np.all(g_kt[cb[0]] == 0.0)
    on_key = np.array([0.5])  # f = 15 exactly (0.5 is an fp32 value): k0 = 15 mod 6 = 3
    g_kq, g_kt, _, _ = pose_sample_backward(offsets, kq, kt, ca, cb, on_key, w, gq, gt, FPS)
    assert np.all(g_kq[:, 4] == 0.0) and np.all(g_kt[:, 4] == 0.0)
    assert np.any(g_kq[:, 3] != 0.0)
    # translations only: g_kt[A, k0] = (1 - w)(1 - alpha) gt, g_kt[B, k1] = w alpha gt
    zero_q = np.zeros_like(gq)
    g_kq, g_kt, g_tau, g_w = pose_sample_backward(offsets, kq, kt, ca, cb, tau, w, zero_q, gt, FPS)
    f = FPS * float(np.float32(tau[0]))
    al, k0 = f - np.floor(f), int(np.floor(f)) % kq.shape[1]
    np.testing.assert_allclose(g_kt[ca[0], k0], (1 - w[0]) * (1 - al) * gt, atol=1e-12)
    np.testing.assert_allclose(g_kt[cb[0], (k0 + 1) % kq.shape[1]], w[0] * al * gt, atol=1e-12)
    assert np.all(g_kq == 0.0)
    tA = (1 - al) * kt[ca[0], k0] + al * kt[ca[0], (k0 + 1) % kq.shape[1]]
    tB = (1 - al) * kt[cb[0], k0] + al * kt[cb[0], (k0 + 1) % kq.shape[1]]
    np.testing.assert_allclose(g_w[0], np.sum(gt * (tB - tA)), atol=1e-12)

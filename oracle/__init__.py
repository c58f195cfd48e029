"""FP64 CPU oracle for the hierarchy scan -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (the HIP kernels behind the C-ABI)
never imports, links or calls anything here, and this package never imports
the product.

Each function widens its fp32 inputs to float64 (an exact conversion) and calls
the plain C routines in ``hs_oracle.c``; those follow the definitions:

* ``trs_to_local``  -- L = [R(q) diag(s) | t], q = (x, y, z, w), the
  textbook unit-quaternion rotation without renormalisation;
* ``scan_matrices`` / ``forward`` -- Eq. 1 with the parent on the left as in
  Algorithms 1-4 (Sec. 2, Sec. 3): G_j = G_parent(j) L_j, parents first;
* ``skin`` -- the Bind MeshPose step (Sec. 1, step 3): S_j = G_j B_j^-1;
* ``pose_sample`` -- the Simulation step (Sec. 1, step 1), two looping clips
  sampled with a normalised lerp and blended (the paper gives no algorithm;
  the reading is stated in ``hs_oracle.c``);
* ``backward`` -- reverse mode of the scan for gradients with respect to the
  local quaternions, translations and scales;
* ``path_length`` -- root-to-joint polyline length used to scale tolerances.

``oracle.vertex_skin`` (NumPy, FP64) holds the vertex-skinning oracle: linear
blend and dual quaternion skinning of mesh vertices with the S_j.
``oracle.sample_backward`` (NumPy, FP64) is the reverse mode of the sampler:
gradients of the keyframes, the clip time and the blend weight.

Parity status: pinned by the ``-m "not gpu"`` tests (brute force, closed
forms, invariants, finite differences); the paper prints no numeric values.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is None:
        path = LIB if os.path.exists(LIB) else build_oracle(force=True)
        lib = ctypes.CDLL(path)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.hso_trs_to_local.argtypes = [i64, _f64p, _f64p, _f64p, _f64p]
        lib.hso_scan_matrices.argtypes = [i64, _i64p, _i32p, _f64p, _f64p]
        lib.hso_forward.argtypes = [i64, _i64p, _i32p, _f64p, _f64p, _f64p, _f64p]
        lib.hso_skin.argtypes = [i64, _f64p, _f64p, _f64p]
        lib.hso_path_length.argtypes = [i64, _i64p, _i32p, _f64p, _f64p, _f64p]
        lib.hso_pose_sample.argtypes = [i64, _i64p, i32, i32, i32, ctypes.c_float,
                                        _f32p, _f32p, _i32p, _i32p, _f32p, _f32p,
                                        _f64p, _f64p]
        lib.hso_backward.argtypes = [i64, _i64p, _i32p, _f64p, _f64p, _f64p, _f64p,
                                     _f64p, _f64p, _f64p, _f64p, _f64p]
        lib.hso_set_threads.argtypes = [i32]
        for name in ("hso_trs_to_local", "hso_scan_matrices", "hso_forward", "hso_skin",
                     "hso_path_length", "hso_pose_sample", "hso_backward", "hso_set_threads"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def set_threads(n):
    """Threads of the parallel loops over characters (n < 1 only queries);
    returns the count in effect.  Characters are independent, so results do
    not depend on it."""
    return int(_load().hso_set_threads(int(n)))


def _check(rc, what):
    if rc != 0:
        kind = {1: "invalid argument", 2: "topology violation (need -1 <= parent[j] < j)"}.get(rc, "error")
        raise OracleError(f"{what}: {kind} (code {rc})")


def _d(a, shape_tail=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_tail is not None and a.shape[1:] != shape_tail:
        a = a.reshape((-1,) + shape_tail)
    return a


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _topo(offsets, parents):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    par = np.ascontiguousarray(np.asarray(parents, dtype=np.int32))
    if off.ndim != 1 or off.size < 1:
        raise OracleError("offsets must be a 1-D array of length C+1")
    if par.size != off[-1]:
        raise OracleError("parents must hold offsets[-1] entries")
    return off, par


def trs_to_local(quat, trans, scale=None):
    """Local 4x4 matrices [N,4,4] (float64) of the given TRS."""
    q, t = _d(quat, (4,)), _d(trans, (3,))
    s = None if scale is None else _d(scale, (3,))
    out = np.empty((q.shape[0], 4, 4), np.float64)
    _check(_load().hso_trs_to_local(q.shape[0], _ptr(q, _f64p), _ptr(t, _f64p), _ptr(s, _f64p),
                                     _ptr(out, _f64p)), "trs_to_local")
    return out


def scan_matrices(offsets, parents, local):
    """Tree prefix product over given local matrices: G_j = G_parent(j) L_j."""
    off, par = _topo(offsets, parents)
    L = _d(local, (4, 4))
    out = np.empty_like(L)
    _check(_load().hso_scan_matrices(off.size - 1, _ptr(off, _i64p), _ptr(par, _i32p),
                                      _ptr(L, _f64p), _ptr(out, _f64p)), "scan_matrices")
    return out


def forward(offsets, parents, quat, trans, scale=None):
    """Global 4x4 matrices [N,4,4] (float64) of the local TRS."""
    off, par = _topo(offsets, parents)
    q, t = _d(quat, (4,)), _d(trans, (3,))
    s = None if scale is None else _d(scale, (3,))
    out = np.empty((par.size, 4, 4), np.float64)
    _check(_load().hso_forward(off.size - 1, _ptr(off, _i64p), _ptr(par, _i32p), _ptr(q, _f64p),
                                _ptr(t, _f64p), _ptr(s, _f64p), _ptr(out, _f64p)), "forward")
    return out


def skin(global_, inv_bind):
    """S_j = G_j B_j^-1 as full 4x4 products (float64)."""
    G, B = _d(global_, (4, 4)), _d(inv_bind, (4, 4))
    out = np.empty_like(G)
    _check(_load().hso_skin(G.shape[0], _ptr(G, _f64p), _ptr(B, _f64p), _ptr(out, _f64p)), "skin")
    return out


def path_length(offsets, parents, global_, trans):
    """Root-to-joint polyline length lambda_j (float64 [N])."""
    off, par = _topo(offsets, parents)
    G, t = _d(global_, (4, 4)), _d(trans, (3,))
    out = np.empty(par.size, np.float64)
    _check(_load().hso_path_length(off.size - 1, _ptr(off, _i64p), _ptr(par, _i32p), _ptr(G, _f64p),
                                    _ptr(t, _f64p), _ptr(out, _f64p)), "path_length")
    return out


def pose_sample(offsets, key_quat, key_trans, clip_a, clip_b, time, weight, fps=30.0):
    """Sample and blend two looping clips per character.

    ``key_quat`` [clips, keys, J, 4] and ``key_trans`` [clips, keys, J, 3]
    are fp32; ``clip_a``/``clip_b`` int32 [C]; ``time``/``weight`` fp32 [C].
    Returns (quat [N,4], trans [N,3]) in float64.
    """
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    kq = np.ascontiguousarray(np.asarray(key_quat, dtype=np.float32))
    kt = np.ascontiguousarray(np.asarray(key_trans, dtype=np.float32))
    if kq.ndim != 4 or kq.shape[3] != 4 or kt.shape != kq.shape[:3] + (3,):
        raise OracleError("key arrays must be [clips, keys, J, 4] and [clips, keys, J, 3]")
    ca = np.ascontiguousarray(np.asarray(clip_a, dtype=np.int32))
    cb = np.ascontiguousarray(np.asarray(clip_b, dtype=np.int32))
    tm = np.ascontiguousarray(np.asarray(time, dtype=np.float32))
    wt = np.ascontiguousarray(np.asarray(weight, dtype=np.float32))
    C = off.size - 1
    if not (ca.size == cb.size == tm.size == wt.size == C):
        raise OracleError("per-character arrays must have C entries")
    N = int(off[-1])
    q = np.empty((N, 4), np.float64)
    t = np.empty((N, 3), np.float64)
    K, T, J = kq.shape[:3]
    _check(_load().hso_pose_sample(C, _ptr(off, _i64p), K, T, J, float(fps), _ptr(kq, _f32p),
                                    _ptr(kt, _f32p), _ptr(ca, _i32p), _ptr(cb, _i32p), _ptr(tm, _f32p),
                                    _ptr(wt, _f32p), _ptr(q, _f64p), _ptr(t, _f64p)), "pose_sample")
    return q, t


def backward(offsets, parents, quat, trans, scale, grad_global):
    """Gradients of sum(grad_global * G) w.r.t. quat, trans and scale (float64).

    Returns (grad_quat [N,4], grad_trans [N,3], grad_scale [N,3]); with
    ``scale=None`` the scale is taken as 1 and its gradient is still returned.
    """
    off, par = _topo(offsets, parents)
    q, t = _d(quat, (4,)), _d(trans, (3,))
    s = None if scale is None else _d(scale, (3,))
    gG = _d(grad_global, (4, 4))
    N = par.size
    gq = np.empty((N, 4), np.float64)
    gt = np.empty((N, 3), np.float64)
    gs = np.empty((N, 3), np.float64)
    work = np.empty((N, 4, 4), np.float64)
    glob = np.empty((N, 4, 4), np.float64)
    _check(_load().hso_backward(off.size - 1, _ptr(off, _i64p), _ptr(par, _i32p), _ptr(q, _f64p),
                                 _ptr(t, _f64p), _ptr(s, _f64p), _ptr(gG, _f64p), _ptr(gq, _f64p),
                                 _ptr(gt, _f64p), _ptr(gs, _f64p), _ptr(work, _f64p),
                                 _ptr(glob, _f64p)), "backward")
    return gq, gt, gs

"""Python binding of the Hierarchy-Scan C ABI (``include/hs.h``).

Argument marshalling only: every function checks tensor shapes, dtypes,
devices and contiguity, passes raw device pointers and torch's current HIP
stream to the C library, and raises :class:`HSError` on a non-zero status.
All computation happens in the library's HIP kernels; there is no fallback.
If the library is not built this module raises on import.

The function names follow the C names: :func:`hs_plan_create`,
:func:`hs_pose_sample`, :func:`hs_scan_forward`, :func:`hs_skin`,
:func:`hs_scan_backward`.
"""
import ctypes
import os

import numpy as np
import torch

from .build import LIB

HS_OK = 0
HS_ERR_INVALID_ARG = 1
HS_ERR_TOPOLOGY = 2
HS_ERR_UNSUPPORTED = 3
HS_ERR_DEVICE = 4
HS_ERR_OOM = 5

HS_STRATEGY_AUTO = 0
HS_STRATEGY_TILE = 1
HS_STRATEGY_MULTIPASS = 2
HS_ALG_SCAN, HS_ALG_WALK, HS_ALG_JUMP, HS_ALG_BLOCKS, HS_ALG_COMPRESSED = 0, 1, 2, 3, 4
HS_ADJ_AUTO, HS_ADJ_ROUNDS, HS_ADJ_DATAFLOW, HS_ADJ_ANCHORS = 0, 1, 2, 3
HS_SCHED_AUTO, HS_SCHED_QUEUE, HS_SCHED_CLASSES = 0, 1, 2
HS_SKIN_LINEAR, HS_SKIN_DUAL_QUAT = 0, 1

HS_POSE_TRS = 0
HS_POSE_CLIPS = 1

HS_DEV_WAIT_TIMEOUT = 1
HS_DEV_TOPOLOGY = 2
HS_FLAG_VALIDATE = 1
HS_NOALLOC_MAX_JOINTS = 1 << 19  # joints the static workspace of hs_pose_sample_backward_noalloc holds

SYMBOLS = ("hs_version", "hs_last_error", "hs_context_create", "hs_context_destroy",
           "hs_plan_create", "hs_plan_create_instanced", "hs_plan_destroy", "hs_plan_get_info", "hs_pose_sample",
           "hs_scan_forward", "hs_skin", "hs_scan_backward", "hs_graph_create_forward",
           "hs_graph_create_forward_n", "hs_graph_launch", "hs_graph_destroy", "hs_mesh_create",
           "hs_mesh_destroy", "hs_skin_vertices", "hs_pose_sample_backward", "hs_scan_skin_vertices",
           "hs_effector_loss_grad", "hs_effectors_create", "hs_effectors_destroy", "hs_effectors_sparse",
           "hs_effector_backward", "hs_effector_step", "hs_plan_status", "hs_plan_set_wait_limit",
           "hs_plan_debug_break_parent", "hs_pose_sample_backward_noalloc", "hs_context_load_tuning",
           "hs_context_save_tuning", "hs_stream_probe")


class HSError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hs status {status}: {message}")
        self.status = status


class hs_batch(ctypes.Structure):
    _fields_ = [("num_characters", ctypes.c_int64), ("num_joints", ctypes.c_int64),
                ("joint_offsets", ctypes.c_void_p), ("parents", ctypes.c_void_p)]


class hs_skeleton_set(ctypes.Structure):
    _fields_ = [("num_skeletons", ctypes.c_int32), ("num_joints", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("parents", ctypes.c_void_p)]


class hs_mesh_batch(ctypes.Structure):
    _fields_ = [("vertex_offsets", ctypes.c_void_p), ("mesh_first", ctypes.c_void_p), ("num_rows", ctypes.c_int64),
                ("positions", ctypes.c_void_p), ("joints", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class hs_plan_opts(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("tile_joints", ctypes.c_int32),
                ("waves_per_tile", ctypes.c_int32), ("grid_tiles", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("chain_units", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("adjoint", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("adjoint_blocks_per_wave", ctypes.c_int32)]


class hs_plan_info(ctypes.Structure):
    _fields_ = [("num_characters", ctypes.c_int64), ("num_joints", ctypes.c_int64),
                ("tiled_joints", ctypes.c_int64), ("multipass_joints", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("max_character", ctypes.c_int32),
                ("num_tiles", ctypes.c_int32), ("tile_joints", ctypes.c_int32),
                ("waves_per_tile", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("multipass_rounds", ctypes.c_int32), ("max_block_chain", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("max_anchors", ctypes.c_int32),
                ("adjoint_blocks_per_wave", ctypes.c_int32), ("chain_joints", ctypes.c_int64)]


class hs_clip_lib(ctypes.Structure):
    _fields_ = [("num_clips", ctypes.c_int32), ("num_keys", ctypes.c_int32),
                ("joints_per_clip", ctypes.c_int32), ("fps", ctypes.c_float),
                ("key_quat", ctypes.c_void_p), ("key_trans", ctypes.c_void_p)]


class hs_clip_params(ctypes.Structure):
    _fields_ = [("clip_a", ctypes.c_void_p), ("clip_b", ctypes.c_void_p),
                ("time", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class hs_pose_src(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("quat", ctypes.c_void_p), ("trans", ctypes.c_void_p),
                ("scale", ctypes.c_void_p), ("clips", ctypes.POINTER(hs_clip_lib)),
                ("params", ctypes.POINTER(hs_clip_params))]


_lib = None


def library_path():
    return LIB


def load_library():
    """Load ``libhs.so``; raises if it has not been built.  (Inside
    ``prepare`` the binding's calls are recorded instead of issued.)"""
    global _lib
    if _recorder is not None:
        return _recorder
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"HIP library not built: {LIB} is missing "
                           "(run __graft_entry__.build() or paper_2505_06703_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.hs_version.restype = ctypes.c_char_p
    lib.hs_last_error.restype = ctypes.c_char_p
    lib.hs_context_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.hs_context_destroy.argtypes = [vp]
    lib.hs_context_destroy.restype = None
    lib.hs_stream_probe.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.hs_context_load_tuning.argtypes = [vp, ctypes.c_char_p]
    lib.hs_context_save_tuning.argtypes = [vp, ctypes.c_char_p]
    lib.hs_plan_create.argtypes = [vp, ctypes.POINTER(hs_batch), ctypes.POINTER(hs_plan_opts),
                                   ctypes.POINTER(vp)]
    lib.hs_plan_create_instanced.argtypes = [vp, ctypes.POINTER(hs_skeleton_set), i32, vp,
                                             ctypes.POINTER(hs_plan_opts), ctypes.POINTER(vp)]
    lib.hs_mesh_create.argtypes = [vp, ctypes.POINTER(hs_mesh_batch), ctypes.POINTER(vp)]
    lib.hs_mesh_destroy.argtypes = [vp]
    lib.hs_mesh_destroy.restype = None
    lib.hs_skin_vertices.argtypes = [vp, vp, i32, vp, vp]
    lib.hs_effector_loss_grad.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    lib.hs_effectors_create.argtypes = [vp, i64, vp, ctypes.POINTER(vp)]
    lib.hs_effectors_destroy.argtypes = [vp]
    lib.hs_effectors_destroy.restype = None
    lib.hs_effectors_sparse.argtypes = [vp]
    lib.hs_effectors_sparse.restype = i32
    lib.hs_effector_backward.argtypes = [vp, vp, ctypes.POINTER(hs_pose_src), vp, vp, vp, vp, vp, vp]
    lib.hs_effector_step.argtypes = [vp, vp, ctypes.POINTER(hs_pose_src), vp, vp, vp, vp, vp, vp]
    lib.hs_scan_skin_vertices.argtypes = [vp, ctypes.POINTER(hs_pose_src), vp, vp, i32, vp, vp, vp]
    lib.hs_pose_sample_backward.argtypes = [vp, ctypes.POINTER(hs_clip_lib), ctypes.POINTER(hs_clip_params),
                                            vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hs_pose_sample_backward_noalloc.argtypes = [vp, ctypes.POINTER(hs_clip_lib),
                                                    ctypes.POINTER(hs_clip_params), vp, vp, vp, vp, vp, vp, vp]
    lib.hs_plan_destroy.argtypes = [vp]
    lib.hs_plan_destroy.restype = None
    lib.hs_plan_get_info.argtypes = [vp, ctypes.POINTER(hs_plan_info)]
    lib.hs_plan_status.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(i64), i32]
    lib.hs_plan_set_wait_limit.argtypes = [vp, i32]
    lib.hs_plan_debug_break_parent.argtypes = [vp, i64]
    lib.hs_pose_sample.argtypes = [vp, ctypes.POINTER(hs_clip_lib), ctypes.POINTER(hs_clip_params),
                                   vp, vp, vp]
    lib.hs_scan_forward.argtypes = [vp, ctypes.POINTER(hs_pose_src), vp, vp, vp, vp, i32, u32, vp]
    lib.hs_skin.argtypes = [i64, vp, vp, vp, vp]
    lib.hs_scan_backward.argtypes = [vp, ctypes.POINTER(hs_pose_src), vp, vp, i32, vp, vp, vp, u32, vp]
    lib.hs_graph_create_forward.argtypes = [vp, ctypes.POINTER(hs_pose_src), vp, vp, vp, ctypes.POINTER(vp)]
    lib.hs_graph_create_forward_n.argtypes = [vp, i32, ctypes.POINTER(hs_pose_src), ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.hs_graph_launch.argtypes = [vp, vp]
    lib.hs_graph_destroy.argtypes = [vp]
    lib.hs_graph_destroy.restype = None
    for name in ("hs_context_create", "hs_plan_create", "hs_plan_get_info", "hs_pose_sample",
                 "hs_scan_forward", "hs_skin", "hs_scan_backward", "hs_graph_create_forward",
                 "hs_graph_launch", "hs_plan_status", "hs_plan_set_wait_limit", "hs_plan_debug_break_parent"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status):
    if status != HS_OK:
        raise HSError(status, load_library().hs_last_error().decode())


_recorder = None


class _Recorder:
    """Stands in for the library inside ``prepare``: keeps each C call and
    its marshalled arguments and reports success."""

    def __init__(self, lib):
        self.lib = lib
        self.calls = []

    def __getattr__(self, name):
        fn = getattr(self.lib, name)

        def record(*args):
            self.calls.append((fn, args))
            return HS_OK
        return record


class PreparedCall:
    """One library call with its arguments marshalled once: calling the
    object issues the same C call again (the same buffers, the same stream)
    and raises HSError if it fails.  For loops that repeat a call on fixed
    buffers, where the binding's per-call checks cost more host time than
    the call itself."""

    def __init__(self, fn, args, keep):
        self._fn = fn
        self._args = args
        self._keep = keep  # the tensors and structures the arguments point into

    def __call__(self):
        status = self._fn(*self._args)
        if status != HS_OK:
            _check(status)


def prepare(binding, *args, **kwargs):
    """Check and marshal one call of a binding function (``hs_scan_forward``,
    ``hs_effector_step``, ...) without issuing it.  Returns ``(call, result)``:
    ``call()`` issues the C call with exactly these arguments, ``result`` is
    what the binding function returns (the output tensors it was given or
    allocated).  The stream is the one current now unless ``stream`` is
    given.  Not thread-safe: no other thread may call the binding meanwhile."""
    global _recorder
    lib = load_library()
    rec = _Recorder(lib)
    _recorder = rec
    try:
        result = binding(*args, **kwargs)
    finally:
        _recorder = None
    if len(rec.calls) != 1:
        raise ValueError(f"{getattr(binding, '__name__', binding)} makes {len(rec.calls)} library calls, not one")
    fn, cargs = rec.calls[0]
    return PreparedCall(fn, cargs, (args, kwargs, result)), result


def hs_version():
    return load_library().hs_version().decode()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, name, shape, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device=0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.hs_context_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)

    def load_tuning(self, path):
        """Merge a JSON tuning cache file into this context (``hs_context_load_tuning``)."""
        _check(load_library().hs_context_load_tuning(self.handle, os.fsencode(path)))

    def save_tuning(self, path):
        """Write this context's tuning cache as JSON (``hs_context_save_tuning``)."""
        _check(load_library().hs_context_save_tuning(self.handle, os.fsencode(path)))

    def close(self):
        if self.handle:
            load_library().hs_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device=None):
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


class Plan:
    """Topology analysis of a CSR batch (see ``hs_plan_create``)."""

    def __init__(self, offsets, parents, ctx=None, strategy=HS_STRATEGY_AUTO, tile_joints=0,
                 waves_per_tile=0, grid_tiles=0, autotune=False, chain_units=False, algorithm=HS_ALG_SCAN,
                 adjoint=HS_ADJ_AUTO, schedule=HS_SCHED_AUTO, adjoint_blocks_per_wave=0,
                 skeletons=None):
        self.ctx = ctx or default_context()
        off = np.ascontiguousarray(np.asarray(offsets.cpu() if isinstance(offsets, torch.Tensor) else offsets,
                                              dtype=np.int64))
        par = np.ascontiguousarray(np.asarray(parents.cpu() if isinstance(parents, torch.Tensor) else parents,
                                              dtype=np.int32))
        if off.ndim != 1 or off.size < 1:
            raise ValueError("offsets must be 1-D with C+1 entries")
        self.num_characters = off.size - 1
        self.num_joints = par.size
        batch = hs_batch(self.num_characters, self.num_joints, off.ctypes.data, par.ctypes.data)
        opts = hs_plan_opts(strategy, tile_joints, waves_per_tile, grid_tiles, int(bool(autotune)),
                            int(bool(chain_units)), int(algorithm), int(adjoint), int(schedule),
                            int(adjoint_blocks_per_wave))
        h = ctypes.c_void_p()
        if skeletons is None:
            _check(load_library().hs_plan_create(self.ctx.handle, ctypes.byref(batch), ctypes.byref(opts),
                                                 ctypes.byref(h)))
            self.bind_rows = self.num_joints
        else:
            soff, spar, sid = skeletons
            sk = hs_skeleton_set(soff.size - 1, spar.size, soff.ctypes.data, spar.ctypes.data)
            _check(load_library().hs_plan_create_instanced(self.ctx.handle, ctypes.byref(sk), sid.size,
                                                           sid.ctypes.data, ctypes.byref(opts), ctypes.byref(h)))
            self.bind_rows = spar.size  # inverse binds: one row per skeleton joint
        self.handle = h

    @classmethod
    def instanced(cls, skel_offsets, skel_parents, skeleton_id, **kw):
        """Plan for characters that are copies of shared skeletons (see
        ``hs_plan_create_instanced``): character c is skeleton
        ``skeleton_id[c]``; inverse binds are then given per skeleton joint."""
        soff = np.ascontiguousarray(np.asarray(skel_offsets, dtype=np.int64))
        spar = np.ascontiguousarray(np.asarray(skel_parents, dtype=np.int32))
        sid = np.ascontiguousarray(np.asarray(skeleton_id, dtype=np.int32))
        if soff.ndim != 1 or soff.size < 1 or spar.ndim != 1 or sid.ndim != 1:
            raise ValueError("skeleton offsets, parents and ids must be 1-D")
        if sid.size and (sid.min() < 0 or sid.max() >= soff.size - 1):
            raise ValueError("skeleton_id out of range")
        sizes = np.diff(soff)
        off = np.concatenate([[0], np.cumsum(sizes[sid])]).astype(np.int64)
        par = np.concatenate([spar[soff[k]:soff[k + 1]] for k in sid]) if sid.size else np.zeros(0, np.int32)
        return cls(off, par, skeletons=(soff, spar, sid), **kw)

    def status(self, clear=False):
        """Synchronise and read the plan's device status word
        (``hs_plan_status``): returns ``(status, bits, joint)`` -- the
        hs_status (HS_OK, or HS_ERR_DEVICE when a bit is set), the HS_DEV_*
        bits and the lowest joint that failed the topology check (-1 if
        none).  Does not raise on HS_ERR_DEVICE."""
        bits, joint = ctypes.c_uint32(), ctypes.c_int64()
        rc = load_library().hs_plan_status(self.handle, ctypes.byref(bits), ctypes.byref(joint), int(bool(clear)))
        if rc not in (HS_OK, HS_ERR_DEVICE):
            _check(rc)
        return rc, bits.value, joint.value

    def set_wait_limit(self, polls):
        """Polls after which a kernel's bounded wait gives up (``hs_plan_set_wait_limit``)."""
        _check(load_library().hs_plan_set_wait_limit(self.handle, int(polls)))

    def debug_break_parent(self, joint):
        """Corrupt one entry of the plan's device parent table (``hs_plan_debug_break_parent``)."""
        _check(load_library().hs_plan_debug_break_parent(self.handle, int(joint)))

    @property
    def info(self):
        inf = hs_plan_info()
        _check(load_library().hs_plan_get_info(self.handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in hs_plan_info._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load_library().hs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hs_plan_create(offsets, parents, **kw):
    return Plan(offsets, parents, **kw)


class ClipLibrary:
    """Device-resident clip library: key_quat [K,T,J,4], key_trans [K,T,J,3]."""

    def __init__(self, key_quat, key_trans, fps=30.0):
        K, T, J, _ = key_quat.shape
        self.key_quat = _need(key_quat, "key_quat", (K, T, J, 4))
        self.key_trans = _need(key_trans, "key_trans", (K, T, J, 3))
        self.fps = float(fps)
        self.c = hs_clip_lib(K, T, J, self.fps, key_quat.data_ptr(), key_trans.data_ptr())


def _clip_params(plan, clip_a, clip_b, time, weight):
    C = plan.num_characters
    _need(clip_a, "clip_a", (C,), torch.int32)
    _need(clip_b, "clip_b", (C,), torch.int32)
    _need(time, "time", (C,))
    _need(weight, "weight", (C,))
    return hs_clip_params(clip_a.data_ptr(), clip_b.data_ptr(), time.data_ptr(), weight.data_ptr())


def hs_pose_sample(plan, clips, clip_a, clip_b, time, weight, quat_out=None, trans_out=None, stream=None):
    """Simulation step: sample and blend two clips per character -> (quat [N,4], trans [N,3])."""
    N = plan.num_joints
    dev = clips.key_quat.device
    q = torch.empty((N, 4), device=dev, dtype=torch.float32) if quat_out is None else _need(quat_out, "quat_out", (N, 4))
    t = torch.empty((N, 3), device=dev, dtype=torch.float32) if trans_out is None else _need(trans_out, "trans_out", (N, 3))
    params = _clip_params(plan, clip_a, clip_b, time, weight)
    _check(load_library().hs_pose_sample(plan.handle, ctypes.byref(clips.c), ctypes.byref(params),
                                         _ptr(q), _ptr(t), _stream(stream)))
    return q, t


def sample_backward_workspace(plan, device):
    """Workspace for ``hs_pose_sample_backward`` ([N,2,4] fp32): with it
    each joint's reverse step runs once."""
    return torch.empty((plan.num_joints, 2, 4), device=device, dtype=torch.float32)


def hs_pose_sample_backward(plan, clips, clip_a, clip_b, time, weight, grad_quat, grad_trans,
                            want_keys=True, workspace=None, stream=None):
    """Reverse mode of the Simulation step -> (grad_key_quat [K,T,J,4],
    grad_key_trans [K,T,J,3], grad_time [C], grad_weight [C]); the key
    gradients are None when ``want_keys`` is false.  ``workspace``: None
    or ``sample_backward_workspace(plan, device)``."""
    N, C = plan.num_joints, plan.num_characters
    _need(grad_quat, "grad_quat", (N, 4))
    _need(grad_trans, "grad_trans", (N, 3))
    dev = clips.key_quat.device
    gkq = torch.empty_like(clips.key_quat) if want_keys else None
    gkt = torch.empty_like(clips.key_trans) if want_keys else None
    gtime = torch.empty((C,), device=dev, dtype=torch.float32)
    gw = torch.empty((C,), device=dev, dtype=torch.float32)
    if workspace is not None:
        _need(workspace, "workspace", (N, 2, 4))
    params = _clip_params(plan, clip_a, clip_b, time, weight)
    _check(load_library().hs_pose_sample_backward(plan.handle, ctypes.byref(clips.c), ctypes.byref(params),
                                                  _ptr(grad_quat), _ptr(grad_trans), _ptr(gkq), _ptr(gkt),
                                                  _ptr(gtime), _ptr(gw), _ptr(workspace), _stream(stream)))
    return gkq, gkt, gtime, gw


def hs_pose_sample_backward_noalloc(plan, clips, clip_a, clip_b, time, weight, grad_quat, grad_trans,
                                    want_keys=True, out=None, stream=None):
    """``hs_pose_sample_backward`` on the library's static device workspace
    (the C call allocates nothing; plans of at most
    ``HS_NOALLOC_MAX_JOINTS`` joints).  ``out``: None, or preallocated
    (grad_key_quat, grad_key_trans, grad_time, grad_weight) tensors, the key
    gradients None when ``want_keys`` is false."""
    N, C = plan.num_joints, plan.num_characters
    _need(grad_quat, "grad_quat", (N, 4))
    _need(grad_trans, "grad_trans", (N, 3))
    if out is None:
        dev = clips.key_quat.device
        out = (torch.empty_like(clips.key_quat) if want_keys else None,
               torch.empty_like(clips.key_trans) if want_keys else None,
               torch.empty((C,), device=dev, dtype=torch.float32),
               torch.empty((C,), device=dev, dtype=torch.float32))
    gkq, gkt, gtime, gw = out
    if gkq is not None:
        _need(gkq, "grad_key_quat", tuple(clips.key_quat.shape))
    if gkt is not None:
        _need(gkt, "grad_key_trans", tuple(clips.key_trans.shape))
    _need(gtime, "grad_time", (C,))
    _need(gw, "grad_weight", (C,))
    params = _clip_params(plan, clip_a, clip_b, time, weight)
    _check(load_library().hs_pose_sample_backward_noalloc(plan.handle, ctypes.byref(clips.c),
                                                          ctypes.byref(params), _ptr(grad_quat),
                                                          _ptr(grad_trans), _ptr(gkq), _ptr(gkt),
                                                          _ptr(gtime), _ptr(gw), _stream(stream)))
    return gkq, gkt, gtime, gw


def hs_stream_probe(quat, trans, scale, table, out=None, stream=None):
    """The forward's HBM traffic without its arithmetic (``hs_stream_probe``):
    returns out [n,4,4]."""
    n = quat.shape[0]
    _need(quat, "quat", (n, 4))
    _need(trans, "trans", (n, 3))
    _need(scale, "scale", (n, 3))
    _need(table, "table", (n,), torch.int32)
    if out is None:
        out = torch.empty((n, 4, 4), device=quat.device, dtype=torch.float32)
    _need(out, "out", (n, 4, 4))
    _check(load_library().hs_stream_probe(n, _ptr(quat), _ptr(trans), _ptr(scale), _ptr(table), _ptr(out),
                                          _stream(stream)))
    return out


def _trs_src(plan, quat, trans, scale):
    N = plan.num_joints
    _need(quat, "quat", (N, 4))
    _need(trans, "trans", (N, 3))
    if scale is not None:
        _need(scale, "scale", (N, 3))
    return hs_pose_src(HS_POSE_TRS, quat.data_ptr(), trans.data_ptr(),
                       None if scale is None else scale.data_ptr(), None, None)


def hs_scan_forward(plan, quat=None, trans=None, scale=None, *, clips=None, clip_a=None, clip_b=None,
                    time=None, weight=None, global_out=None, want_global=True, inv_bind=None,
                    skin_out=None, ckpt_out=None, ckpt_k=0, validate=False, stream=None, device=None):
    """Hierarchy-Scan with optional fused skin and checkpoints.

    Poses come from ``quat``/``trans``/``scale`` (TRS) or from ``clips`` and
    the per-character clip parameters (fused Simulation step).  Returns
    ``(global [N,4,4] or None, skin [N,4,4] or None)``.
    """
    N = plan.num_joints
    if clips is not None:
        params = _clip_params(plan, clip_a, clip_b, time, weight)
        src = hs_pose_src(HS_POSE_CLIPS, None, None, None, ctypes.pointer(clips.c), ctypes.pointer(params))
        dev = clips.key_quat.device
    else:
        src = _trs_src(plan, quat, trans, scale)
        dev = quat.device
    if global_out is None and want_global:
        global_out = torch.empty((N, 4, 4), device=dev, dtype=torch.float32)
    elif global_out is not None:
        _need(global_out, "global_out", (N, 4, 4))
    if inv_bind is not None:
        _need(inv_bind, "inv_bind", (plan.bind_rows, 4, 4))
        if skin_out is None:
            skin_out = torch.empty((N, 4, 4), device=dev, dtype=torch.float32)
        else:
            _need(skin_out, "skin_out", (N, 4, 4))
    if ckpt_out is not None:
        _need(ckpt_out, "ckpt_out", (N, 12))
    _check(load_library().hs_scan_forward(plan.handle, ctypes.byref(src), _ptr(global_out), _ptr(inv_bind),
                                          _ptr(skin_out), _ptr(ckpt_out), int(ckpt_k),
                                          HS_FLAG_VALIDATE if validate else 0, _stream(stream)))
    return global_out, skin_out


def hs_skin(global_, inv_bind, skin_out=None, stream=None):
    """Bind MeshPose step: skin_j = global_j @ inv_bind_j (full 4x4)."""
    n = global_.shape[0]
    _need(global_, "global", (n, 4, 4))
    _need(inv_bind, "inv_bind", (n, 4, 4))
    if skin_out is None:
        skin_out = torch.empty_like(global_)
    _need(skin_out, "skin_out", (n, 4, 4))
    _check(load_library().hs_skin(n, _ptr(global_), _ptr(inv_bind), _ptr(skin_out), _stream(stream)))
    return skin_out


class Mesh:
    """Meshes of a plan's characters (see ``hs_mesh_create``): character c's
    vertices are output rows ``vertex_offsets[c]`` .. ``vertex_offsets[c+1]-1``
    and read mesh rows from ``mesh_first[c]`` on (host arrays; the library
    copies them)."""

    def __init__(self, plan, vertex_offsets, mesh_first, positions, joints, weights):
        voff = np.ascontiguousarray(np.asarray(vertex_offsets, np.int64))
        mf = np.ascontiguousarray(np.asarray(mesh_first, np.int32))
        pos = np.ascontiguousarray(np.asarray(positions, np.float32))
        jt = np.ascontiguousarray(np.asarray(joints, np.int32))
        wt = np.ascontiguousarray(np.asarray(weights, np.float32))
        rows = pos.shape[0]
        if pos.shape != (rows, 3) or jt.shape != (rows, 4) or wt.shape != (rows, 4):
            raise ValueError("positions, joints and weights must be [rows,3], [rows,4], [rows,4]")
        if voff.shape != (plan.num_characters + 1,) or mf.shape != (plan.num_characters,):
            raise ValueError("vertex_offsets and mesh_first must have C+1 and C entries")
        self.num_vertices = int(voff[-1])
        mb = hs_mesh_batch(voff.ctypes.data, mf.ctypes.data, rows, pos.ctypes.data, jt.ctypes.data, wt.ctypes.data)
        h = ctypes.c_void_p()
        _check(load_library().hs_mesh_create(plan.handle, ctypes.byref(mb), ctypes.byref(h)))
        self.handle = h
        self.num_joints = plan.num_joints

    def close(self):
        if getattr(self, "handle", None):
            load_library().hs_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hs_skin_vertices(mesh, skin, method=HS_SKIN_LINEAR, out=None, stream=None):
    """Skinned vertex positions [V,3] from the skin matrices [N,4,4]."""
    _need(skin, "skin", (mesh.num_joints, 4, 4))
    if out is None:
        out = torch.empty((mesh.num_vertices, 3), device=skin.device)
    _need(out, "out", (mesh.num_vertices, 3))
    _check(load_library().hs_skin_vertices(mesh.handle, _ptr(skin), int(method), _ptr(out), _stream(stream)))
    return out


def hs_scan_skin_vertices(plan, mesh, inv_bind, quat=None, trans=None, scale=None, *, clips=None, clip_a=None,
                          clip_b=None, time=None, weight=None, method=HS_SKIN_LINEAR, vertices_out=None,
                          skin_out=None, stream=None):
    """Poses, scan, skin matrices and vertex skinning in one pass per tile
    (``hs_scan_skin_vertices``) -> vertices [V,3] (and ``skin_out`` if given)."""
    N = plan.num_joints
    if clips is not None:
        params = _clip_params(plan, clip_a, clip_b, time, weight)
        src = hs_pose_src(HS_POSE_CLIPS, None, None, None, ctypes.pointer(clips.c), ctypes.pointer(params))
        dev = clips.key_quat.device
    else:
        src = _trs_src(plan, quat, trans, scale)
        dev = quat.device
    _need(inv_bind, "inv_bind", (plan.bind_rows, 4, 4))
    if vertices_out is None:
        vertices_out = torch.empty((mesh.num_vertices, 3), device=dev, dtype=torch.float32)
    _need(vertices_out, "vertices_out", (mesh.num_vertices, 3))
    if skin_out is not None:
        _need(skin_out, "skin_out", (N, 4, 4))
    _check(load_library().hs_scan_skin_vertices(plan.handle, ctypes.byref(src), _ptr(inv_bind), mesh.handle,
                                                int(method), _ptr(vertices_out), _ptr(skin_out), _stream(stream)))
    return vertices_out


def hs_effector_loss_grad(global_, effectors, targets, grad_global, stream=None):
    """dLoss/dG of sum_e |b_e - y_e|^2 written into the effector rows of
    ``grad_global`` (whose other entries the caller keeps zero)."""
    N = global_.shape[0]
    _need(global_, "global", (N, 4, 4))
    _need(grad_global, "grad_global", (N, 4, 4))
    E = effectors.shape[0]
    _need(effectors, "effectors", (E,), torch.int64)
    _need(targets, "targets", (E, 3))
    _check(load_library().hs_effector_loss_grad(N, E, _ptr(effectors), _ptr(global_), _ptr(targets),
                                                _ptr(grad_global), _stream(stream)))
    return grad_global


class Effectors:
    """A fixed set of end-effector joints of a plan (``hs_effectors_create``;
    global joint ids, host array, distinct), for ``hs_effector_backward``."""

    def __init__(self, plan, joint_ids):
        ids = np.ascontiguousarray(np.asarray(joint_ids, np.int64).reshape(-1))
        h = ctypes.c_void_p()
        _check(load_library().hs_effectors_create(plan.handle, ids.shape[0], ids.ctypes.data, ctypes.byref(h)))
        self.handle = h
        self.plan = plan
        self.num_effectors = int(ids.shape[0])

    @property
    def sparse(self):
        """True when the adjoint forms the seeds on chip (no dense dLoss/dG)."""
        return bool(load_library().hs_effectors_sparse(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            load_library().hs_effectors_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hs_effector_backward(plan, effectors, quat, trans, scale, global_, targets, want_scale=True, grad_quat=None,
                         grad_trans=None, grad_scale=None, stream=None):
    """Adjoint of sum_e |b_e - y_e|^2 over ``effectors`` (an ``Effectors``),
    given the forward output ``global_`` [N,4,4] and targets [E,3]: returns
    (grad_quat [N,4], grad_trans [N,3], grad_scale [N,3] or None)."""
    N = plan.num_joints
    src = _trs_src(plan, quat, trans, scale)
    _need(global_, "global", (N, 4, 4))
    _need(targets, "targets", (effectors.num_effectors, 3))
    dev = quat.device
    gq = torch.empty((N, 4), device=dev, dtype=torch.float32) if grad_quat is None else _need(grad_quat, "grad_quat", (N, 4))
    gt = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_trans is None else _need(grad_trans, "grad_trans", (N, 3))
    gs = None
    if want_scale:
        gs = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_scale is None else _need(grad_scale, "grad_scale", (N, 3))
    _check(load_library().hs_effector_backward(plan.handle, effectors.handle, ctypes.byref(src), _ptr(global_),
                                               _ptr(targets), _ptr(gq), _ptr(gt), _ptr(gs), _stream(stream)))
    return gq, gt, gs


def hs_effector_step(plan, effectors, quat, trans, scale, targets, global_out=None, want_scale=True,
                     grad_quat=None, grad_trans=None, grad_scale=None, stream=None):
    """Forward scan and the adjoint of sum_e |b_e - y_e|^2 in one launch
    (``hs_effector_step``; needs ``effectors.sparse``): returns (grad_quat,
    grad_trans, grad_scale or None); G goes to ``global_out`` if given."""
    N = plan.num_joints
    src = _trs_src(plan, quat, trans, scale)
    _need(targets, "targets", (effectors.num_effectors, 3))
    if global_out is not None:
        _need(global_out, "global_out", (N, 4, 4))
    dev = quat.device
    gq = torch.empty((N, 4), device=dev, dtype=torch.float32) if grad_quat is None else _need(grad_quat, "grad_quat", (N, 4))
    gt = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_trans is None else _need(grad_trans, "grad_trans", (N, 3))
    gs = None
    if want_scale:
        gs = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_scale is None else _need(grad_scale, "grad_scale", (N, 3))
    _check(load_library().hs_effector_step(plan.handle, effectors.handle, ctypes.byref(src), _ptr(targets),
                                           _ptr(global_out), _ptr(gq), _ptr(gt), _ptr(gs), _stream(stream)))
    return gq, gt, gs


def hs_scan_backward(plan, quat, trans, scale, grad_global, ckpt=None, ckpt_k=0, want_scale=True,
                     grad_quat=None, grad_trans=None, grad_scale=None, validate=False, stream=None):
    """Adjoint of the scan: returns (grad_quat [N,4], grad_trans [N,3], grad_scale [N,3] or None)."""
    N = plan.num_joints
    src = _trs_src(plan, quat, trans, scale)
    _need(grad_global, "grad_global", (N, 4, 4))
    dev = quat.device
    gq = torch.empty((N, 4), device=dev, dtype=torch.float32) if grad_quat is None else _need(grad_quat, "grad_quat", (N, 4))
    gt = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_trans is None else _need(grad_trans, "grad_trans", (N, 3))
    gs = None
    if want_scale:
        gs = torch.empty((N, 3), device=dev, dtype=torch.float32) if grad_scale is None else _need(grad_scale, "grad_scale", (N, 3))
    if ckpt is not None:
        _need(ckpt, "ckpt", (N, 12))
    _check(load_library().hs_scan_backward(plan.handle, ctypes.byref(src), _ptr(grad_global), _ptr(ckpt),
                                           int(ckpt_k), _ptr(gq), _ptr(gt), _ptr(gs),
                                           HS_FLAG_VALIDATE if validate else 0, _stream(stream)))
    return gq, gt, gs


class ForwardGraph:
    """hs_scan_forward calls captured into one HIP graph
    (``hs_graph_create_forward`` / ``hs_graph_create_forward_n``).

    ``ForwardGraph(plan, quat, trans, scale, global_out=...)`` captures one
    call; ``ForwardGraph.sequence(plan, [kwargs, ...])`` captures several, in
    order (same keyword arguments as the single form).  The arrays are baked
    into the graph: ``launch()`` re-reads the current contents of the same
    inputs and rewrites the same outputs.  The object keeps references to
    them so that they outlive the graph.
    """

    def __init__(self, plan, quat=None, trans=None, scale=None, *, clips=None, clip_a=None, clip_b=None,
                 time=None, weight=None, global_out=None, inv_bind=None, skin_out=None):
        self._create(plan, [dict(quat=quat, trans=trans, scale=scale, clips=clips, clip_a=clip_a, clip_b=clip_b,
                                 time=time, weight=weight, global_out=global_out, inv_bind=inv_bind,
                                 skin_out=skin_out)])

    @classmethod
    def sequence(cls, plan, calls):
        self = cls.__new__(cls)
        self._create(plan, [dict(c) for c in calls])
        return self

    def _create(self, plan, calls):
        N = plan.num_joints
        n = len(calls)
        if n < 1:
            raise ValueError("at least one call to capture")
        srcs = (hs_pose_src * n)()
        gouts, binds, souts = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
        keep = [plan, srcs]
        for i, c in enumerate(calls):
            if c.get("clips") is not None:
                params = _clip_params(plan, c["clip_a"], c["clip_b"], c["time"], c["weight"])
                srcs[i] = hs_pose_src(HS_POSE_CLIPS, None, None, None, ctypes.pointer(c["clips"].c),
                                      ctypes.pointer(params))
                keep.append(params)
            else:
                srcs[i] = _trs_src(plan, c.get("quat"), c.get("trans"), c.get("scale"))
            if c.get("global_out") is not None:
                _need(c["global_out"], "global_out", (N, 4, 4))
            if c.get("inv_bind") is not None:
                _need(c["inv_bind"], "inv_bind", (plan.bind_rows, 4, 4))
                _need(c.get("skin_out"), "skin_out", (N, 4, 4))
            gouts[i], binds[i], souts[i] = (_ptr(c.get("global_out")), _ptr(c.get("inv_bind")),
                                           _ptr(c.get("skin_out")))
            keep.append(c)
        self._keep = keep
        h = ctypes.c_void_p()
        _check(load_library().hs_graph_create_forward_n(plan.handle, n, srcs, gouts, binds, souts, ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(load_library().hs_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            load_library().hs_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

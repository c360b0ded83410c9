"""Thin ctypes binding of libnbt_ig.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/nbt_ig.h with
the same name minus the ``nbt_ig_`` prefix.  Device buffers are torch tensors
(PyTorch-ROCm provides allocation and the current HIP stream); no
computation of the method happens in Python.  Importing this module raises
ImportError when the HIP library has not been built, so nothing can fall
back to another implementation silently.
"""

from __future__ import annotations

import ctypes as C
import weakref
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbt_ig.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc --offload-arch=gfx950)")

# torch (device memory and streams) carries its own HIP runtime; it is loaded first
# so that the library binds to that same runtime instead of a second copy.
import torch as _torch_mod  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
RAY_MISS, RAY_HIT, RAY_END, RAY_EXIT, RAY_INVALID = 0, 1, 2, 3, 4
LAYOUT_LINEAR, LAYOUT_COLUMN4, LAYOUT_COLUMN2, LAYOUT_COLUMN8 = 0, 1, 2, 3
LAYOUT_NAMES = ("linear", "column4", "column2", "column8")
OCCUPIED, FREE, UNKNOWN = 1, 2, 3


class NbtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status


class CameraT(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("tan_half_fov_h", C.c_float),
                ("tan_half_fov_v", C.c_float), ("range", C.c_float)]


class LaunchT(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("tile_w_log2", C.c_int32),
                ("tiles_per_wave", C.c_int32), ("xcd_remap", C.c_int32), ("pipeline_depth", C.c_int32)]


class InsertParamsT(C.Structure):
    _fields_ = [("l_hit", C.c_float), ("l_miss", C.c_float), ("l_min", C.c_float), ("l_max", C.c_float)]


class ClassifyT(C.Structure):
    _fields_ = [("occ_threshold", C.c_float), ("free_threshold", C.c_float)]


_vp = C.c_void_p
_u32 = C.c_uint32


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_sig("nbt_ig_abi_version", C.c_int)
_sig("nbt_ig_status_string", C.c_char_p, C.c_int)
_sig("nbt_ig_last_error", C.c_char_p)
_sig("nbt_ig_ctx_create", C.c_int, C.c_int, C.POINTER(_vp))
_sig("nbt_ig_ctx_destroy", None, _vp)
_sig("nbt_ig_create_map", C.c_int, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_float,
     C.POINTER(C.c_float), C.POINTER(ClassifyT), _vp, C.POINTER(_vp))
_sig("nbt_ig_destroy_map", None, _vp)
_sig("nbt_ig_update_map", C.c_int, _vp, _vp, _vp)
_sig("nbt_ig_insert_default_params", InsertParamsT)
_sig("nbt_ig_insert_workspace_words", C.c_uint64, _vp)
_sig("nbt_ig_insert_scans", C.c_int, _vp, C.POINTER(CameraT), _vp, _vp, _u32, C.POINTER(InsertParamsT),
     _vp, _vp, _vp, C.c_uint64, _vp)
_sig("nbt_ig_map_check", C.c_int, _vp, _vp)
_sig("nbt_ig_map_info", C.c_int, _vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
     C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_size_t))
_sig("nbt_ig_eval_viewpoints", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp, _vp)
_sig("nbt_ig_probe_sink_words", C.c_int, _vp)
_sig("nbt_ig_probe_memory", C.c_int, _vp, C.c_int, _vp, C.c_size_t, _u32, _vp, _vp)
_sig("nbt_ig_probe_mfma", C.c_int, _vp, C.c_int, C.c_int, _u32, _vp, C.POINTER(C.c_double), _vp)
_sig("nbt_ig_eval_viewpoints_noalloc", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp, _vp)
_sig("nbt_ig_eval_trajectories", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _u32, _vp, _vp, _vp, _vp)
_sig("nbt_ig_ctx_set_lds_budget", C.c_int, _vp, C.c_size_t)
_sig("nbt_ig_ctx_info", C.c_int, _vp, C.POINTER(C.c_int), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t))
_sig("nbt_ig_ctx_set_traj_waves", C.c_int, _vp, C.c_int)
_sig("nbt_ig_ctx_set_map_layout", C.c_int, _vp, C.c_int)
_sig("nbt_ig_ctx_get_map_layout", C.c_int, _vp, C.POINTER(C.c_int))
_sig("nbt_ig_map_layout", C.c_int, _vp, C.POINTER(C.c_int))
_sig("nbt_ig_map_set_layout", C.c_int, _vp, C.c_int, _vp)
_sig("nbt_ig_autotune_map", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp, _vp, C.POINTER(LaunchT),
     C.POINTER(C.c_int), C.POINTER(C.c_float))
_sig("nbt_ig_ctx_get_traj_waves", C.c_int, _vp, C.POINTER(C.c_int))
_sig("nbt_ig_trace_rays", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp)
_sig("nbt_ig_trace_viewpoints", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp, _vp, _vp)
_sig("nbt_ig_trace_trajectories", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _u32, _vp, _vp, _vp, _vp, _vp)
_sig("nbt_ig_trace_paths", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _u32, _u32, _vp, _vp, _vp)
_sig("nbt_ig_ctx_set_launch", C.c_int, _vp, C.POINTER(LaunchT))
_sig("nbt_ig_ctx_get_launch", C.c_int, _vp, C.POINTER(LaunchT))
_sig("nbt_ig_batch_create", C.c_int, _vp, C.POINTER(_vp), _u32, C.POINTER(CameraT), _u32, C.POINTER(_vp))
_sig("nbt_ig_batch_destroy", None, _vp)
_sig("nbt_ig_batch_run", C.c_int, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("nbt_ig_batch_set_launch", C.c_int, _vp, C.POINTER(LaunchT))
_sig("nbt_ig_batch_get_launch", C.c_int, _vp, C.POINTER(LaunchT), C.POINTER(_u32))
_sig("nbt_ig_autotune_viewpoints", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _vp, _vp, _vp,
     C.POINTER(LaunchT), C.POINTER(C.c_float))
_sig("nbt_ig_batch_autotune", C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(LaunchT), C.POINTER(C.c_float))
_sig("nbt_ig_batch_autotune_layout", C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_int), C.POINTER(C.c_float))
_sig("nbt_ig_autotune_trajectories", C.c_int, _vp, C.POINTER(CameraT), _vp, _u32, _u32, _vp, _vp, _vp, _vp,
     C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_float))
_sig("nbt_ig_surrogate_create", C.c_int, _vp, C.c_void_p, C.c_size_t, C.POINTER(_vp))
_sig("nbt_ig_surrogate_destroy", None, _vp)
_sig("nbt_ig_surrogate_predict", C.c_int, _vp, _vp, C.POINTER(C.c_float), _vp, _u32, _vp, _vp)
_sig("nbt_ig_surrogate_select", C.c_int, _vp, _vp, C.POINTER(CameraT), C.POINTER(C.c_float), _vp, _u32, _u32,
     _u32, _vp, _vp, _vp)
_sig("nbt_ig_surrogate_features", C.c_int, _vp, _vp, C.POINTER(C.c_float), _vp, _vp, _vp)
_sig("nbt_ig_extract_patch", C.c_int, _vp, C.POINTER(C.c_float), C.c_float, _vp, _vp)
_sig("nbt_ig_eval_cost", C.c_int, _vp, _vp, _vp, _u32, _u32, C.c_float, _vp, _u32, _u32, C.POINTER(C.c_float),
     C.c_float, C.c_float, C.c_float, C.c_float, _vp, _vp, _vp, _vp)
_sig("nbt_ig_top_k", C.c_int, _vp, _vp, _u32, _u32, _vp, _vp, _vp)
_sig("nbt_ig_camera_from_grid", C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
     C.POINTER(CameraT))


def lib():
    return _lib


def abi_version() -> int:
    return _lib.nbt_ig_abi_version()


def status_string(s: int) -> str:
    return _lib.nbt_ig_status_string(s).decode()


def last_error() -> str:
    return _lib.nbt_ig_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise NbtError(rc, f"{status_string(rc)}: {last_error()}")


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def camera(cam) -> CameraT:
    """Accept a CameraT, an object with ``as_tuple()`` or (W, H, tan_h, tan_v, range)."""
    if isinstance(cam, CameraT):
        return cam
    if hasattr(cam, "as_tuple"):
        cam = cam.as_tuple()
    w, h, th, tv, r = cam
    return CameraT(int(w), int(h), float(th), float(tv), float(r))


def camera_from_grid(fov_h, fov_v, d_cam, s_vox, s_g) -> CameraT:
    out = CameraT()
    _check(_lib.nbt_ig_camera_from_grid(fov_h, fov_v, d_cam, s_vox, s_g, C.byref(out)))
    return out


class Context:
    """One device plus the reduction workspace (nbt_ig_ctx)."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(_lib.nbt_ig_ctx_create(int(device), C.byref(h)))
        self.handle = h
        self.device = int(device)
        self._children = weakref.WeakSet()     # maps, batches and surrogates of this context

    def set_launch(self, waves_per_group=4, tile_w_log2=3, tiles_per_wave=0, xcd_remap=0, pipeline_depth=0):
        _check(_lib.nbt_ig_ctx_set_launch(self.handle, C.byref(LaunchT(waves_per_group, tile_w_log2,
                                                                        tiles_per_wave, xcd_remap,
                                                                        pipeline_depth))))

    def get_launch(self):
        l = LaunchT()
        _check(_lib.nbt_ig_ctx_get_launch(self.handle, C.byref(l)))
        return {"waves_per_group": l.waves_per_group, "tile_w_log2": l.tile_w_log2,
                "tiles_per_wave": l.tiles_per_wave, "xcd_remap": l.xcd_remap,
                "pipeline_depth": l.pipeline_depth}

    def set_lds_budget(self, nbytes=0):
        _check(_lib.nbt_ig_ctx_set_lds_budget(self.handle, int(nbytes)))

    def set_map_layout(self, layout):
        """Storage order of maps created from now on: LAYOUT_LINEAR or LAYOUT_COLUMN2/4/8."""
        _check(_lib.nbt_ig_ctx_set_map_layout(self.handle, int(layout)))

    def get_map_layout(self):
        v = C.c_int()
        _check(_lib.nbt_ig_ctx_get_map_layout(self.handle, C.byref(v)))
        return v.value

    def set_traj_waves(self, waves_per_group=8):
        _check(_lib.nbt_ig_ctx_set_traj_waves(self.handle, int(waves_per_group)))

    def get_traj_waves(self):
        w = C.c_int()
        _check(_lib.nbt_ig_ctx_get_traj_waves(self.handle, C.byref(w)))
        return w.value

    def info(self):
        cu, lds, budget = C.c_int(), C.c_size_t(), C.c_size_t()
        _check(_lib.nbt_ig_ctx_info(self.handle, C.byref(cu), C.byref(lds), C.byref(budget)))
        return {"cu_count": cu.value, "lds_per_group": lds.value, "lds_budget": budget.value}

    def close(self):
        """Destroys the context's batches, surrogates and maps still open, then the context."""
        if self.handle:
            kids = list(self._children)
            for kind in (Batch, Surrogate, Map):
                for obj in kids:
                    if isinstance(obj, kind):
                        obj.close()
            _lib.nbt_ig_ctx_destroy(self.handle)
            self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Map:
    """A device-resident encoded occupancy map (nbt_ig_map).

    ``prob`` is float32 [nz, ny, nx]: a torch tensor (host or device) or a
    NumPy array.  The library copies it.
    """

    def __init__(self, ctx: Context, prob, voxel: float, origin, thresholds=(0.5, 0.5), stream=None):
        torch = _torch()
        if not isinstance(prob, torch.Tensor):
            prob = torch.from_numpy(prob)
        if prob.dtype != torch.float32 or prob.dim() != 3:
            raise ValueError("prob must be float32 [nz, ny, nx]")
        prob = prob.contiguous()
        nz, ny, nx = prob.shape
        org = (C.c_float * 3)(*[float(v) for v in origin])
        cls = ClassifyT(float(thresholds[0]), float(thresholds[1]))
        h = _vp()
        self.ctx = ctx
        self.handle = _vp()
        _check(_lib.nbt_ig_create_map(ctx.handle, C.c_void_p(prob.data_ptr()), nx, ny, nz, float(voxel),
                                      org, C.byref(cls), _stream(stream), C.byref(h)))
        self.handle = h
        ctx._children.add(self)
        self.dims = (nx, ny, nz)
        self.voxel = float(voxel)

    def update(self, prob, stream=None):
        """Re-encode in place from a device tensor of the same shape (asynchronous)."""
        torch = _torch()
        if tuple(prob.shape) != (self.dims[2], self.dims[1], self.dims[0]):
            raise ValueError("prob shape differs from the map")
        _check(_lib.nbt_ig_update_map(self.handle, _dev_ptr(prob, torch.float32, "prob"), _stream(stream)))

    def check(self, stream=None):
        _check(_lib.nbt_ig_map_check(self.handle, _stream(stream)))

    def set_layout(self, layout, stream=None):
        """Rewrite the map in another storage order (synchronises the stream)."""
        _check(_lib.nbt_ig_map_set_layout(self.handle, int(layout), _stream(stream)))

    def info(self):
        nx, ny, nz = C.c_int(), C.c_int(), C.c_int()
        vs = C.c_float()
        org = (C.c_float * 3)()
        nb = C.c_size_t()
        _check(_lib.nbt_ig_map_info(self.handle, C.byref(nx), C.byref(ny), C.byref(nz), C.byref(vs),
                                    org, C.byref(nb)))
        lay = C.c_int()
        _check(_lib.nbt_ig_map_layout(self.handle, C.byref(lay)))
        return {"dims": (nx.value, ny.value, nz.value), "voxel": vs.value, "origin": tuple(org),
                "device_bytes": nb.value, "layout": lay.value}

    def close(self):
        if self.handle and self.ctx.handle:
            _lib.nbt_ig_destroy_map(self.handle)
        self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_viewpoints(m: Map, cam, poses, ig_out=None, steps_out=None, stream=None, want_steps=True):
    """Per-perspective IG (float32 [N]) and voxel steps (int64 [N] holding uint64)."""
    torch = _torch()
    n = poses.shape[0]
    dev = poses.device
    if ig_out is None:
        ig_out = torch.empty(n, dtype=torch.float32, device=dev)
    if steps_out is None and want_steps:
        steps_out = torch.empty(n, dtype=torch.int64, device=dev)
    cm = camera(cam)
    _check(_lib.nbt_ig_eval_viewpoints(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), n,
                                       _dev_ptr(ig_out, torch.float32, "ig_out"),
                                       _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream)))
    return ig_out, steps_out


PROBE_STREAM, PROBE_GATHER, PROBE_QUAD_GATHER = 0, 1, 2


def probe_memory(ctx, kind, buf, count, sink=None, stream=None):
    """nbt_ig_probe_memory over the bytes of device tensor ``buf``; returns the sink tensor."""
    torch = _torch()
    if sink is None:
        sink = torch.empty(int(_lib.nbt_ig_probe_sink_words(ctx.handle)), dtype=torch.int32, device=buf.device)
    _check(_lib.nbt_ig_probe_memory(ctx.handle, int(kind), _dev_ptr(buf, None, "buf"),
                                    buf.numel() * buf.element_size(), int(count), _dev_ptr(sink, torch.int32, "sink"),
                                    _stream(stream)))
    return sink


PROBE_MFMA_16X16X32_BF16, PROBE_MFMA_32X32X16_BF16 = 0, 1


def probe_mfma(ctx, kind, waves_per_simd, iters, sink=None, stream=None):
    """nbt_ig_probe_mfma; returns (sink tensor, floating point operations of the launch)."""
    torch = _torch()
    if sink is None:
        sink = torch.empty(int(_lib.nbt_ig_probe_sink_words(ctx.handle)), dtype=torch.int32,
                           device=f"cuda:{ctx.device}")
    flops = C.c_double()
    _check(_lib.nbt_ig_probe_mfma(ctx.handle, int(kind), int(waves_per_simd), int(iters),
                                  _dev_ptr(sink, torch.int32, "sink"), C.byref(flops), _stream(stream)))
    return sink, flops.value


NOALLOC_MAX_VIEWPOINTS = 65536


def eval_viewpoints_noalloc(m: Map, cam, poses, ig_out, steps_out=None, stream=None):
    """nbt_ig_eval_viewpoints_noalloc: as eval_viewpoints, into caller-given outputs, with the
    library's fixed reduction slots (at most NOALLOC_MAX_VIEWPOINTS perspectives; calls that
    overlap on one device race)."""
    torch = _torch()
    cm = camera(cam)
    _check(_lib.nbt_ig_eval_viewpoints_noalloc(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"),
                                               int(poses.shape[0]), _dev_ptr(ig_out, torch.float32, "ig_out"),
                                               _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream)))
    return ig_out, steps_out


def insert_default_params():
    """(l_hit, l_miss, l_min, l_max) the library uses when none are given."""
    p = _lib.nbt_ig_insert_default_params()
    return (p.l_hit, p.l_miss, p.l_min, p.l_max)


def insert_scans(m: Map, cam, poses, depth, logodds, params=None, prob_out=None, workspace=None, stream=None):
    """Depth-image insertion into the log-odds grid ``logodds`` (device float32 [nz, ny, nx],
    updated in place): poses float32 [K, 12], depth float32 [K, H, W] z-depths in metres.
    ``params`` = (l_hit, l_miss, l_min, l_max) or None for the library's defaults.  ``prob_out``
    (device float32 like logodds) receives 1/(1+exp(-L)).  Without ``workspace`` the map keeps
    a zeroed one of its own; calls that share a workspace must not overlap (one stream, or
    synchronise between streams).  Returns logodds."""
    torch = _torch()
    nx, ny, nz = m.dims
    if tuple(logodds.shape) != (nz, ny, nx):
        raise ValueError("logodds shape differs from the map")
    if poses.dim() != 2 or int(poses.shape[1]) != 12:
        raise ValueError("poses must be [K, 12] (row-major camera-to-world rotation, then the centre)")
    k = int(poses.shape[0])
    cm = camera(cam)
    if tuple(depth.shape) != (k, cm.height, cm.width):
        raise ValueError("depth must be [K, height, width]")
    words = int(_lib.nbt_ig_insert_workspace_words(m.handle))
    if workspace is None:
        workspace = getattr(m, "_insert_ws", None)
        if workspace is None or workspace.device != logodds.device:
            workspace = torch.zeros(words, dtype=torch.int32, device=logodds.device)
            m._insert_ws = workspace
            if stream is not None and not isinstance(stream, int):
                # the zero fill ran on torch's current stream; the kernels run on `stream`
                stream.wait_stream(torch.cuda.current_stream(logodds.device))
            elif isinstance(stream, int):
                torch.cuda.current_stream(logodds.device).synchronize()
    prm = None if params is None else C.byref(InsertParamsT(*[float(v) for v in params]))
    _check(_lib.nbt_ig_insert_scans(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"),
                                    _dev_ptr(depth, torch.float32, "depth"), k, prm,
                                    _dev_ptr(logodds, torch.float32, "logodds"),
                                    _dev_ptr(prob_out, torch.float32, "prob_out"),
                                    _dev_ptr(workspace, torch.int32, "workspace"), int(workspace.numel()),
                                    _stream(stream)))
    return logodds


def eval_trajectories(m: Map, cam, poses, stream=None, want_visits=True):
    """Union IG per trajectory: poses float32 [T, L, 12] -> (ig [T], counts [T,4] int32, visits [T] int64
    or None when want_visits is False: the walk then keeps no visit count, which is faster)."""
    torch = _torch()
    T, L = int(poses.shape[0]), int(poses.shape[1])
    dev = poses.device
    ig = torch.empty(T, dtype=torch.float32, device=dev)
    counts = torch.empty((T, 4), dtype=torch.int32, device=dev)
    visits = torch.empty(T, dtype=torch.int64, device=dev) if want_visits else None
    cm = camera(cam)
    _check(_lib.nbt_ig_eval_trajectories(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), T, L,
                                         _dev_ptr(ig, torch.float32, "ig"), _dev_ptr(counts, None, "counts"),
                                         _dev_ptr(visits, None, "visits"), _stream(stream)))
    return ig, counts, visits


def _records(out, shape):
    """nbt_ig_ray_digest records (int32 [R, 8]) as a dict of tensors shaped `shape`."""
    torch = _torch()
    return {
        "hash": out[:, 0:2].contiguous().view(torch.int64).view(*shape),
        "gain": out[:, 2:4].contiguous().view(torch.float64).view(*shape),
        "steps": out[:, 4].view(*shape),
        "stop_lin": out[:, 5].view(*shape),
        "reason": out[:, 6].view(*shape),
        "reserved": out[:, 7].view(*shape),
    }


def trace_rays(m: Map, cam, poses, out=None, stream=None):
    """Per-ray records of the reference walk as a dict of tensors shaped [N, W*H]."""
    torch = _torch()
    cm = camera(cam)
    n = poses.shape[0]
    rays = cm.width * cm.height
    if out is None:
        out = torch.empty((n * rays, 8), dtype=torch.int32, device=poses.device)
    _check(_lib.nbt_ig_trace_rays(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), n,
                                  _dev_ptr(out, torch.int32, "out"), _stream(stream)))
    return _records(out, (n, rays))


def trace_viewpoints(m: Map, cam, poses, want_steps=True, stream=None):
    """The timed per-perspective kernel in its parity instance: (ig [N], steps [N] or None,
    records dict of tensors shaped [N, W*H])."""
    torch = _torch()
    cm = camera(cam)
    n = poses.shape[0]
    rays = cm.width * cm.height
    ig = torch.empty(n, dtype=torch.float32, device=poses.device)
    steps = torch.empty(n, dtype=torch.int64, device=poses.device) if want_steps else None
    out = torch.empty((n * rays, 8), dtype=torch.int32, device=poses.device)
    _check(_lib.nbt_ig_trace_viewpoints(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), n,
                                        _dev_ptr(ig, torch.float32, "ig"), _dev_ptr(steps, torch.int64, "steps"),
                                        _dev_ptr(out, torch.int32, "out"), _stream(stream)))
    return ig, steps, _records(out, (n, rays))


def trace_trajectories(m: Map, cam, poses, want_visits=True, stream=None):
    """The trajectory union kernel in its parity instance: poses [T, L, 12] -> (ig [T],
    counts [T, 4], visits [T] or None, records dict of tensors shaped [T, L, W*H]; the
    record's `reserved` counts visits whose bitset position named another voxel)."""
    torch = _torch()
    T, L = int(poses.shape[0]), int(poses.shape[1])
    cm = camera(cam)
    rays = cm.width * cm.height
    dev = poses.device
    ig = torch.empty(T, dtype=torch.float32, device=dev)
    counts = torch.empty((T, 4), dtype=torch.int32, device=dev)
    visits = torch.empty(T, dtype=torch.int64, device=dev) if want_visits else None
    out = torch.empty((max(T * L * rays, 1), 8), dtype=torch.int32, device=dev)
    _check(_lib.nbt_ig_trace_trajectories(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), T, L,
                                          _dev_ptr(ig, torch.float32, "ig"), _dev_ptr(counts, None, "counts"),
                                          _dev_ptr(visits, None, "visits"), _dev_ptr(out, torch.int32, "out"),
                                          _stream(stream)))
    return ig, counts, visits, _records(out[:T * L * rays], (T, L, rays))


def trace_paths(m: Map, cam, poses, rays_sel, max_len, stream=None):
    """Full voxel sequences for selected (pose, ray) pairs: (lin [count, max_len], len [count])."""
    torch = _torch()
    cm = camera(cam)
    sel = rays_sel.to(device=poses.device, dtype=torch.int32).contiguous()
    count = sel.shape[0]
    lin = torch.full((count, max(int(max_len), 1)), -1, dtype=torch.int32, device=poses.device)
    ln = torch.zeros(count, dtype=torch.int32, device=poses.device)
    _check(_lib.nbt_ig_trace_paths(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"),
                                   poses.shape[0], _dev_ptr(sel, None, "rays"), count, int(max_len),
                                   _dev_ptr(lin, None, "lin"), _dev_ptr(ln, None, "len"), _stream(stream)))
    return lin, ln


def _launch_dict(l):
    return {"waves_per_group": l.waves_per_group, "tile_w_log2": l.tile_w_log2,
            "tiles_per_wave": l.tiles_per_wave, "xcd_remap": l.xcd_remap,
            "pipeline_depth": l.pipeline_depth}


class Batch:
    """Many maps, one persistent hipGraph-launched evaluation (nbt_ig_batch)."""

    def __init__(self, ctx: Context, maps, cam, max_total_viewpoints: int):
        self.ctx = ctx
        self.handle = _vp()
        arr = (_vp * len(maps))(*[m.handle for m in maps])
        h = _vp()
        self._cam = camera(cam)
        _check(_lib.nbt_ig_batch_create(ctx.handle, arr, len(maps), C.byref(self._cam),
                                        int(max_total_viewpoints), C.byref(h)))
        self.handle = h
        self.maps = list(maps)          # keep the maps alive
        ctx._children.add(self)

    def run(self, vp_offsets, poses, ig_out, steps_out=None, stream=None):
        torch = _torch()
        _check(_lib.nbt_ig_batch_run(self.handle, _dev_ptr(vp_offsets, torch.int32, "vp_offsets"),
                                     _dev_ptr(poses, torch.float32, "poses"),
                                     _dev_ptr(ig_out, torch.float32, "ig_out"),
                                     _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream)))

    def set_launch(self, waves_per_group=4, tile_w_log2=3, tiles_per_wave=0, pipeline_depth=0):
        _check(_lib.nbt_ig_batch_set_launch(self.handle, C.byref(LaunchT(waves_per_group, tile_w_log2,
                                                                          tiles_per_wave, 0, pipeline_depth))))

    def get_launch(self):
        l, g = LaunchT(), _u32()
        _check(_lib.nbt_ig_batch_get_launch(self.handle, C.byref(l), C.byref(g)))
        d = _launch_dict(l)
        d["persistent_groups"] = g.value
        return d

    def autotune(self, vp_offsets, poses, ig_out, steps_out=None, stream=None):
        torch = _torch()
        l, ms = LaunchT(), C.c_float()
        _check(_lib.nbt_ig_batch_autotune(self.handle, _dev_ptr(vp_offsets, torch.int32, "vp_offsets"),
                                          _dev_ptr(poses, torch.float32, "poses"),
                                          _dev_ptr(ig_out, torch.float32, "ig_out"),
                                          _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream),
                                          C.byref(l), C.byref(ms)))
        return _launch_dict(l), ms.value

    def autotune_layout(self, vp_offsets, poses, ig_out, steps_out=None, stream=None):
        """Put all maps of the batch in the faster storage order; returns (layout, ms)."""
        torch = _torch()
        lay, ms = C.c_int(), C.c_float()
        _check(_lib.nbt_ig_batch_autotune_layout(self.handle, _dev_ptr(vp_offsets, torch.int32, "vp_offsets"),
                                                 _dev_ptr(poses, torch.float32, "poses"),
                                                 _dev_ptr(ig_out, torch.float32, "ig_out"),
                                                 _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream),
                                                 C.byref(lay), C.byref(ms)))
        return lay.value, ms.value

    def close(self):
        if self.handle and self.ctx.handle:
            _lib.nbt_ig_batch_destroy(self.handle)
        self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_viewpoints(m: Map, cam, poses, ig_out=None, steps_out=None, stream=None):
    """Pick the fastest launch shape for these inputs; the context keeps it."""
    torch = _torch()
    n = poses.shape[0]
    if ig_out is None:
        ig_out = torch.empty(n, dtype=torch.float32, device=poses.device)
    cm = camera(cam)
    l, ms = LaunchT(), C.c_float()
    _check(_lib.nbt_ig_autotune_viewpoints(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), n,
                                           _dev_ptr(ig_out, torch.float32, "ig_out"),
                                           _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream),
                                           C.byref(l), C.byref(ms)))
    return _launch_dict(l), ms.value


def autotune_map(m: Map, cam, poses, ig_out=None, steps_out=None, stream=None):
    """Pick the faster storage order for the map (it is rewritten in it), then the fastest
    launch shape (the context keeps it).  Returns (launch, layout, ms)."""
    torch = _torch()
    n = poses.shape[0]
    if ig_out is None:
        ig_out = torch.empty(n, dtype=torch.float32, device=poses.device)
    cm = camera(cam)
    l, lay, ms = LaunchT(), C.c_int(), C.c_float()
    _check(_lib.nbt_ig_autotune_map(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), n,
                                    _dev_ptr(ig_out, torch.float32, "ig_out"),
                                    _dev_ptr(steps_out, torch.int64, "steps_out"), _stream(stream),
                                    C.byref(l), C.byref(lay), C.byref(ms)))
    return _launch_dict(l), lay.value, ms.value


def autotune_trajectories(m: Map, cam, poses, stream=None, want_visits=False):
    """Pick the storage order of the map (it is rewritten in it) and the trajectory workgroup
    size (the context keeps it) that run eval_trajectories fastest on these poses [T, L, 12]
    (timed without the visit count unless want_visits).  Returns (layout, waves, ms)."""
    torch = _torch()
    T, L = int(poses.shape[0]), int(poses.shape[1])
    dev = poses.device
    ig = torch.empty(T, dtype=torch.float32, device=dev)
    counts = torch.empty((T, 4), dtype=torch.int32, device=dev)
    visits = torch.empty(T, dtype=torch.int64, device=dev) if want_visits else None
    cm = camera(cam)
    lay, w, ms = C.c_int(), C.c_int(), C.c_float()
    _check(_lib.nbt_ig_autotune_trajectories(m.handle, C.byref(cm), _dev_ptr(poses, torch.float32, "poses"), T, L,
                                             _dev_ptr(ig, torch.float32, "ig"), _dev_ptr(counts, None, "counts"),
                                             _dev_ptr(visits, None, "visits"), _stream(stream), C.byref(lay),
                                             C.byref(w), C.byref(ms)))
    return lay.value, w.value, ms.value


def _poi(poi):
    return (C.c_float * 3)(*[float(v) for v in poi])


def extract_patch(m: Map, poi, extent, stream=None):
    """Occupied / unknown fractions [2, 32, 32, 32] around the PoI (float32 device tensor)."""
    torch = _torch()
    out = torch.empty((2, 32, 32, 32), dtype=torch.float32, device="cuda")
    _check(_lib.nbt_ig_extract_patch(m.handle, _poi(poi), float(extent), _dev_ptr(out, torch.float32, "out"),
                                     _stream(stream)))
    return out


class Surrogate:
    """The learned IG surrogate (nbt_ig_surrogate); `weights` is the packed blob (bytes)."""

    def __init__(self, ctx: Context, weights: bytes):
        self.ctx = ctx
        self.handle = _vp()
        h = _vp()
        buf = C.create_string_buffer(bytes(weights), len(weights))
        _check(_lib.nbt_ig_surrogate_create(ctx.handle, C.cast(buf, C.c_void_p), len(weights), C.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def predict(self, m: Map, poi, poses, pred=None, stream=None):
        torch = _torch()
        n = poses.shape[0]
        if pred is None:
            pred = torch.empty(n, dtype=torch.float32, device=poses.device)
        _check(_lib.nbt_ig_surrogate_predict(self.handle, m.handle, _poi(poi), _dev_ptr(poses, torch.float32, "poses"),
                                             n, _dev_ptr(pred, torch.float32, "pred"), _stream(stream)))
        return pred

    def select(self, m: Map, cam, poi, poses, k_rescore=256, k=10, stream=None, idx_out=None, ig_out=None):
        """Best k of the candidates: the surrogate's k_rescore best, rescored exactly (into
        idx_out / ig_out when given)."""
        torch = _torch()
        idx = idx_out if idx_out is not None else torch.empty(k, dtype=torch.int32, device=poses.device)
        ig = ig_out if ig_out is not None else torch.empty(k, dtype=torch.float32, device=poses.device)
        if idx.numel() < k or ig.numel() < k:
            raise ValueError("idx_out and ig_out need k elements")
        cm = camera(cam)
        _check(_lib.nbt_ig_surrogate_select(self.handle, m.handle, C.byref(cm), _poi(poi),
                                            _dev_ptr(poses, torch.float32, "poses"), poses.shape[0], int(k_rescore),
                                            int(k), _dev_ptr(idx, None, "idx"), _dev_ptr(ig, torch.float32, "ig"),
                                            _stream(stream)))
        return idx, ig

    def features(self, m: Map, poi, stream=None, want_patch=True, want_features=True):
        """The patch and the trunk's features (None where not wanted: the call then runs the
        trunk alone)."""
        torch = _torch()
        patch = torch.empty((2, 32, 32, 32), dtype=torch.float32, device="cuda") if want_patch else None
        feat = torch.empty(512, dtype=torch.float32, device="cuda") if want_features else None
        _check(_lib.nbt_ig_surrogate_features(
            self.handle, m.handle, _poi(poi), _dev_ptr(patch, None, "patch") if want_patch else None,
            _dev_ptr(feat, None, "feat") if want_features else None, _stream(stream)))
        return patch, feat

    def close(self):
        if self.handle and self.ctx.handle:
            _lib.nbt_ig_surrogate_destroy(self.handle)
        self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_cost(ctx: Context, id_pos, id_ig, poses, poi, tan_h, tan_v, p=2.0, w_i=1.0, eps=1e-7, stream=None):
    """Planner terms for horizons: id_pos [NB,NP,3], id_ig [NB,NP], poses [H,K,12] (device tensors).
    Returns (G [H,K], O [H,K], cost [H])."""
    torch = _torch()
    nb, np_ = int(id_ig.shape[0]), int(id_ig.shape[1])
    h, k = int(poses.shape[0]), int(poses.shape[1])
    G = torch.empty((h, k), dtype=torch.float32, device=poses.device)
    O = torch.empty((h, k), dtype=torch.float32, device=poses.device)
    cost = torch.empty(h, dtype=torch.float32, device=poses.device)
    _check(_lib.nbt_ig_eval_cost(ctx.handle, _dev_ptr(id_pos, torch.float32, "id_pos"),
                                 _dev_ptr(id_ig, torch.float32, "id_ig"), nb, np_, float(p),
                                 _dev_ptr(poses, torch.float32, "poses"), h, k, _poi(poi), float(tan_h), float(tan_v),
                                 float(w_i), float(eps), _dev_ptr(G, None, "G"), _dev_ptr(O, None, "O"),
                                 _dev_ptr(cost, None, "cost"), _stream(stream)))
    return G, O, cost


def top_k(ctx: Context, values, k, stream=None):
    """(indices int32 [k], values [k]) of the k largest values, ties to the lower index."""
    torch = _torch()
    idx = torch.empty(k, dtype=torch.int32, device=values.device)
    val = torch.empty(k, dtype=torch.float32, device=values.device)
    _check(_lib.nbt_ig_top_k(ctx.handle, _dev_ptr(values, torch.float32, "values"), values.numel(), int(k),
                             _dev_ptr(idx, None, "idx"), _dev_ptr(val, None, "val"), _stream(stream)))
    return idx, val

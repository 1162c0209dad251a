"""Probe-grid ray tracing on MI355X: thin Python binding over libprobetrace.so.

Every step of the trace runs in the HIP library (``csrc/``); this module only marshals
arguments (torch device tensors as raw pointers, the current HIP stream) into the C ABI
declared in ``include/probetrace.h``.  There is no fallback: if the library is missing
or no GPU is visible, the calls raise.

Method: arXiv 2507.14624 (see the header for the passages each entry point follows).
"""
from __future__ import annotations

import ctypes
import math
import os

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprobetrace.so")

PT_MISS, PT_HIT, PT_UNKNOWN = 0, 1, 2
PT_FLAG_PERSISTENT = 1
PT_FLAG_GRAPH = 2
PT_FLAG_NEAREST = 4
PT_FLAG_WIDE = 8
PT_FLAG_START_TEXEL = 16
PT_FLAG_NO_START_TEXEL = 32
PT_FLAG_FP64 = 64
PT_FLAG_SCATTER_PER_TEXEL = 128
PT_FLAG_TRACE_ALL_PROBES = 256

EXPORTED = ("pt_trace_opts_default", "probe_grid_create", "probe_grid_destroy", "probe_grid_read_level",
            "probe_grid_set_coarse", "probe_grid_set_distance", "probe_bake_points",
            "probe_trace", "probe_trace_noalloc", "probe_trace_rays", "probe_trace_backward", "probe_trace_backward_hits",
            "probe_trace_backward_distance", "probe_trace_soft", "probe_trace_soft_backward", "probe_autotune",
            "pt_adam_step", "pt_last_error")


class PtGridDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3),
                ("map_res", ctypes.c_int32), ("mip_levels", ctypes.c_int32), ("scene_min", ctypes.c_float * 3),
                ("scene_max", ctypes.c_float * 3)]


class PtView(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fwd", ctypes.c_float * 3), ("tan_half_fov_y", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class PtTraceOpts(ctypes.Structure):
    _fields_ = [("thickness_rel", ctypes.c_float), ("eye_eps_rel", ctypes.c_float),
                ("background", ctypes.c_float * 3), ("max_probes_per_cell", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("start_level", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class ProbeTraceError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libprobetrace.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.pt_trace_opts_default.argtypes = [ctypes.POINTER(PtTraceOpts)]
    lib.pt_trace_opts_default.restype = None
    lib.probe_grid_create.argtypes = [ctypes.POINTER(PtGridDesc), vp, vp, vp, ctypes.POINTER(vp)]
    lib.probe_grid_destroy.argtypes = [vp]
    lib.probe_grid_destroy.restype = None
    lib.probe_grid_read_level.argtypes = [vp, i32, vp, vp]
    lib.probe_grid_set_coarse.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.probe_bake_points.argtypes = [ctypes.POINTER(PtGridDesc), vp, vp, vp, i64, vp, vp, vp, vp]
    lib.probe_trace.argtypes = [vp, vp, ctypes.POINTER(PtView), i32, vp, vp, vp, vp, ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_trace_noalloc.argtypes = lib.probe_trace.argtypes
    lib.probe_trace_rays.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_trace_backward.argtypes = [vp, ctypes.POINTER(PtView), i32, vp, vp, ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_autotune.argtypes = [vp, vp, ctypes.POINTER(PtView), i32, vp, ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_trace_backward_distance.argtypes = [vp, vp, ctypes.POINTER(PtView), i32, vp, vp, vp,
                                                  ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_grid_set_distance.argtypes = [vp, vp, vp]
    lib.probe_trace_soft.argtypes = [vp, vp, ctypes.POINTER(PtView), i32, ctypes.c_float, vp,
                                     ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_trace_soft_backward.argtypes = [vp, vp, ctypes.POINTER(PtView), i32, ctypes.c_float, vp, vp, vp, vp,
                                              ctypes.POINTER(PtTraceOpts), vp]
    lib.probe_trace_backward_hits.argtypes = [vp, ctypes.POINTER(PtView), i32, vp, vp, vp, vp,
                                              ctypes.POINTER(PtTraceOpts), vp]
    f64 = ctypes.c_double
    lib.pt_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, i32, f64, f64, f64, f64, f64, vp]
    for name in ("probe_grid_create", "probe_grid_read_level", "probe_grid_set_coarse", "probe_bake_points",
                 "probe_trace", "probe_trace_noalloc", "probe_trace_rays", "probe_grid_set_distance",
                 "probe_trace_backward", "probe_trace_backward_hits", "probe_trace_backward_distance",
                 "probe_trace_soft", "probe_trace_soft_backward", "probe_autotune", "pt_adam_step"):
        getattr(lib, name).restype = ctypes.c_int
    lib.pt_last_error.argtypes = []
    lib.pt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = _lib.pt_last_error().decode(errors="replace")
        raise ProbeTraceError(f"probetrace status {status}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ProbeTraceError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ProbeTraceError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ProbeTraceError(f"{name} must be contiguous")
    return t


def trace_opts(thickness_rel=0.0, eye_eps_rel=0.0, background=(0.0, 0.0, 0.0), max_probes_per_cell=8,
               tile=(8, 8), start_level=-1, flags=0) -> PtTraceOpts:
    o = PtTraceOpts()
    load_library().pt_trace_opts_default(ctypes.byref(o))
    o.thickness_rel = float(thickness_rel)
    o.eye_eps_rel = float(eye_eps_rel)
    o.background[:] = [float(c) for c in background]
    o.max_probes_per_cell = int(max_probes_per_cell)
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.start_level = int(start_level)
    o.flags = int(flags)
    return o


def make_views(views) -> ctypes.Array:
    """Views as a ctypes array; each view has pos/right/up/fwd/tan_half_fov_y/width/height."""
    arr = (PtView * len(views))()
    for a, v in zip(arr, views):
        a.pos[:] = [float(c) for c in v.pos]
        a.right[:] = [float(c) for c in v.right]
        a.up[:] = [float(c) for c in v.up]
        a.fwd[:] = [float(c) for c in v.fwd]
        a.tan_half_fov_y = float(v.tan_half_fov_y)
        a.width = int(v.width)
        a.height = int(v.height)
    return arr


def n_rays(views) -> int:
    return int(sum(int(v.width) * int(v.height) for v in views))


class ProbeGrid:
    """Device-resident probe geometry (probe_grid_create / probe_grid_destroy)."""

    def __init__(self, dims, origin, spacing, map_res, mip_levels, scene_min, scene_max, distance, normal_half,
                 stream=None):
        lib = load_library()
        distance = _dev_tensor(distance, torch.float32, "distance")
        normal_half = _dev_tensor(normal_half, torch.float16, "normal (FP16 octahedral u, v)")
        d = PtGridDesc()
        d.dims[:] = [int(x) for x in dims]
        d.origin[:] = [float(x) for x in origin]
        d.spacing[:] = [float(x) for x in spacing]
        d.map_res = int(map_res)
        d.mip_levels = int(mip_levels)
        d.scene_min[:] = [float(x) for x in scene_min]
        d.scene_max[:] = [float(x) for x in scene_max]
        P = d.dims[0] * d.dims[1] * d.dims[2]
        N = d.map_res
        if tuple(distance.shape) != (P, N, N) or tuple(normal_half.shape) != (P, N, N, 2):
            raise ProbeTraceError(f"expected distance [{P},{N},{N}] and normal [{P},{N},{N},2]")
        self.handle = ctypes.c_void_p()
        self.desc = d
        self.P, self.N, self.levels = P, N, d.mip_levels
        self.coarse = None
        self.dims = tuple(d.dims)
        self.device = distance.device
        _check(lib.probe_grid_create(ctypes.byref(d), _ptr(distance), _ptr(normal_half), _stream(stream),
                                     ctypes.byref(self.handle)))
        # the library copies on the stream: keep the inputs alive until it has run
        (stream or torch.cuda.current_stream()).synchronize()

    @classmethod
    def from_probes(cls, probes, device="cuda"):
        """From a baked probe set (numpy arrays, see synth.ProbeSet)."""
        import numpy as np
        dist = torch.from_numpy(np.ascontiguousarray(probes.distance)).to(device)
        nrm = torch.from_numpy(np.ascontiguousarray(probes.normal).view(np.float16)).to(device)
        return cls(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                   probes.scene_max, dist, nrm)

    @classmethod
    def from_two_level(cls, two_level, device="cuda"):
        """Fine grid with its coarse level attached, from a synth.TwoLevel pair."""
        fine = cls.from_probes(two_level.fine, device)
        fine.set_coarse(cls.from_probes(two_level.coarse, device), two_level.plane_off, two_level.ratio)
        return fine

    def set_coarse(self, coarse, plane_off=(0, 0, 0), ratio=(1, 1, 1)):
        """Attach (or, with None, detach) the coarse level of a two-level hierarchy: coarse plane
        k is fine plane plane_off + k * ratio.  Coarse probe p becomes probe self.P + p."""
        lib = load_library()
        off = (ctypes.c_int32 * 3)(*[int(x) for x in plane_off])
        rat = (ctypes.c_int32 * 3)(*[int(x) for x in ratio])
        _check(lib.probe_grid_set_coarse(self.handle, coarse.handle if coarse is not None else None, off, rat))
        self.coarse = coarse  # keeps it alive while attached

    def set_distance(self, distance, stream=None):
        """Replace this grid's distance maps ([P,N,N] FP32 on the device) and rebuild its MIN
        pyramid; the tensor must stay alive until the stream has passed the call."""
        lib = load_library()
        distance = _dev_tensor(distance, torch.float32, "distance")
        _need(distance, self.P * self.N * self.N, "distance")
        _check(lib.probe_grid_set_distance(self.handle, _ptr(distance), _stream(stream)))

    @property
    def P_total(self) -> int:
        """Probes of the radiance layout: the fine ones, then the coarse level's."""
        return self.P + (self.coarse.P if self.coarse is not None else 0)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().probe_grid_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def read_level(self, level: int, stream=None) -> torch.Tensor:
        n = self.N >> level
        out = torch.empty((self.P, n, n), dtype=torch.float32, device=self.device)
        _check(load_library().probe_grid_read_level(self.handle, int(level), _ptr(out), _stream(stream)))
        return out


def probe_bake_points(dims, origin, spacing, map_res, points, colors, normals=None, stream=None):
    """Bake probe maps from a point cloud on the GPU (probe_bake_points).  points, colors,
    normals: [M,3] float32 (device tensors or arrays; normals None = store the probe-to-point
    direction).  Returns device tensors distance [P,N,N] float32, normal [P,N,N,2] float16
    (octahedral u, v), radiance [P,N,N,3] float16."""
    lib = load_library()
    dev = torch.device("cuda")
    pts = _dev_tensor(torch.as_tensor(points, device=dev), torch.float32, "points")
    col = _dev_tensor(torch.as_tensor(colors, device=dev), torch.float32, "colors")
    nrm = None if normals is None else _dev_tensor(torch.as_tensor(normals, device=dev), torch.float32, "normals")
    M = pts.shape[0]
    _need(pts, 3 * M, "points")
    _need(col, 3 * M, "colors")
    _need(nrm, 3 * M, "normals")
    d = PtGridDesc()
    d.dims[:] = [int(x) for x in dims]
    d.origin[:] = [float(x) for x in origin]
    d.spacing[:] = [float(x) for x in spacing]
    d.map_res = int(map_res)
    d.mip_levels = 1
    P, N = d.dims[0] * d.dims[1] * d.dims[2], d.map_res
    dist = torch.empty((P, N, N), dtype=torch.float32, device=dev)
    nrm_out = torch.empty((P, N, N, 2), dtype=torch.float16, device=dev)
    rad = torch.empty((P, N, N, 3), dtype=torch.float16, device=dev)
    _check(lib.probe_bake_points(ctypes.byref(d), _ptr(pts), _ptr(col), _ptr(nrm) if nrm is not None else None,
                                 int(M), _ptr(dist), _ptr(nrm_out), _ptr(rad), _stream(stream)))
    return dist, nrm_out, rad


def _alloc_outputs(rays, device, want_t=True, want_status=True, want_hit=True):
    rgb = torch.empty((rays, 3), dtype=torch.float32, device=device)
    t = torch.empty(rays, dtype=torch.float32, device=device) if want_t else None
    st = torch.empty(rays, dtype=torch.uint8, device=device) if want_status else None
    hit = torch.empty((rays, 2), dtype=torch.int32, device=device) if want_hit else None
    return rgb, t, st, hit


def _need(t, n: int, what: str):
    """The library reads and writes these buffers by plain pointer: check their sizes here."""
    if t is not None and t.numel() != n:
        raise ProbeTraceError(f"{what}: expected {n} elements, got {t.numel()}")


def probe_trace(grid: ProbeGrid, radiance_half, views, opts: PtTraceOpts | None = None, out=None, stream=None,
                want_t=True, want_status=True, want_hit=True):
    """Trace every pixel of ``views``; returns dict(rgb, t, status, hit) of device tensors."""
    lib = load_library()
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    rgb, t, st, hit = out if out is not None else _alloc_outputs(rays, radiance_half.device, want_t, want_status,
                                                                  want_hit)
    for a, k, what in ((rgb, 3, "rgb"), (t, 1, "t"), (st, 1, "status"), (hit, 2, "hit")):
        _need(a, rays * k, what)
    _check(lib.probe_trace(grid.handle, _ptr(radiance_half), va, len(va), _ptr(rgb), _ptr(t), _ptr(st), _ptr(hit),
                           ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return dict(rgb=rgb, t=t, status=st, hit=hit)


def probe_trace_noalloc(grid: ProbeGrid, radiance_half, views, out, opts: PtTraceOpts | None = None, stream=None):
    """probe_trace through the entry point that allocates nothing (its scratch is a fixed
    device array).  ``out`` = (rgb, t, status, hit) device tensors (t, status, hit may be
    None), written in place and returned as a dict."""
    lib = load_library()
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    rgb, t, st, hit = out
    for a, k, what in ((rgb, 3, "rgb"), (t, 1, "t"), (st, 1, "status"), (hit, 2, "hit")):
        _need(a, rays * k, what)
    _check(lib.probe_trace_noalloc(grid.handle, _ptr(radiance_half), va, len(va), _ptr(rgb), _ptr(t), _ptr(st),
                                   _ptr(hit), ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return dict(rgb=rgb, t=t, status=st, hit=hit)


def probe_trace_rays(grid: ProbeGrid, radiance_half, origins, dirs, opts: PtTraceOpts | None = None, stream=None):
    lib = load_library()
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    origins = _dev_tensor(origins, torch.float32, "origins")
    dirs = _dev_tensor(dirs, torch.float32, "dirs")
    n = origins.shape[0]
    _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    _need(origins, 3 * n, "origins")
    _need(dirs, 3 * n, "dirs")
    rgb, t, st, hit = _alloc_outputs(n, origins.device)
    _check(lib.probe_trace_rays(grid.handle, _ptr(radiance_half), _ptr(origins), _ptr(dirs), int(n), _ptr(rgb),
                                _ptr(t), _ptr(st), _ptr(hit), ctypes.byref(opts) if opts is not None else None,
                                _stream(stream)))
    return dict(rgb=rgb, t=t, status=st, hit=hit)


def probe_trace_backward(grid: ProbeGrid, views, grad_rgb, grad_radiance, opts: PtTraceOpts | None = None,
                         stream=None):
    """Accumulate (+=) the radiance gradient of sum(grad_rgb * rgb) into grad_radiance [P,N,N,3] FP32."""
    lib = load_library()
    grad_rgb = _dev_tensor(grad_rgb, torch.float32, "grad_rgb")
    grad_radiance = _dev_tensor(grad_radiance, torch.float32, "grad_radiance")
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _need(grad_rgb, 3 * sum(v.width * v.height for v in va), "grad_rgb")
    _need(grad_radiance, grid.P_total * grid.N * grid.N * 3, "grad_radiance")
    _check(lib.probe_trace_backward(grid.handle, va, len(va), _ptr(grad_rgb), _ptr(grad_radiance),
                                    ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return grad_radiance


def probe_trace_backward_hits(grid: ProbeGrid, views, hit, t, grad_rgb, grad_radiance,
                              opts: PtTraceOpts | None = None, stream=None):
    """probe_trace_backward from the forward's hit [rays,2] int32 and t [rays] outputs (no
    recomputed march); accumulates (+=) into grad_radiance [P_total,N,N,3] FP32."""
    lib = load_library()
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    hit = _dev_tensor(hit, torch.int32, "hit")
    t = _dev_tensor(t, torch.float32, "t")
    grad_rgb = _dev_tensor(grad_rgb, torch.float32, "grad_rgb")
    grad_radiance = _dev_tensor(grad_radiance, torch.float32, "grad_radiance")
    _need(hit, 2 * rays, "hit")
    _need(t, rays, "t")
    _need(grad_rgb, 3 * rays, "grad_rgb")
    _need(grad_radiance, grid.P_total * grid.N * grid.N * 3, "grad_radiance")
    _check(lib.probe_trace_backward_hits(grid.handle, va, len(va), _ptr(hit), _ptr(t), _ptr(grad_rgb),
                                         _ptr(grad_radiance), ctypes.byref(opts) if opts is not None else None,
                                         _stream(stream)))
    return grad_radiance


def probe_trace_backward_distance(grid: ProbeGrid, radiance_half, views, grad_rgb, grad_t, grad_distance,
                                  opts: PtTraceOpts | None = None, stream=None):
    """Accumulate (+=) the gradient of sum(grad_rgb * rgb) + sum(grad_t * t) with respect to
    the stored distances into grad_distance [P_total,N,N] FP32, the classification held
    fixed.  grad_rgb or grad_t may be None (not both)."""
    lib = load_library()
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    grad_distance = _dev_tensor(grad_distance, torch.float32, "grad_distance")
    _need(grad_distance, grid.P_total * grid.N * grid.N, "grad_distance")
    if grad_rgb is not None:
        grad_rgb = _dev_tensor(grad_rgb, torch.float32, "grad_rgb")
        _need(grad_rgb, 3 * rays, "grad_rgb")
        radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
        _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    if grad_t is not None:
        grad_t = _dev_tensor(grad_t, torch.float32, "grad_t")
        _need(grad_t, rays, "grad_t")
    _check(lib.probe_trace_backward_distance(
        grid.handle, _ptr(radiance_half) if grad_rgb is not None else None, va, len(va),
        _ptr(grad_rgb) if grad_rgb is not None else None, _ptr(grad_t) if grad_t is not None else None,
        _ptr(grad_distance), ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return grad_distance


def probe_trace_soft(grid: ProbeGrid, radiance_half, views, sigma: float, opts: PtTraceOpts | None = None,
                     out=None, stream=None):
    """Soft-visibility colour [rays,3] (probe_trace_soft): the candidates of the walk mixed
    by logistic acceptance weights of temperature sigma (relative to the stored distance)."""
    lib = load_library()
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    rgb = out if out is not None else torch.empty((rays, 3), dtype=torch.float32, device=radiance_half.device)
    _need(rgb, 3 * rays, "rgb")
    _check(lib.probe_trace_soft(grid.handle, _ptr(radiance_half), va, len(va), float(sigma), _ptr(rgb),
                                ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return rgb


def probe_trace_soft_backward(grid: ProbeGrid, radiance_half, views, sigma: float, rgb, grad_rgb,
                              grad_distance=None, grad_radiance=None, opts: PtTraceOpts | None = None, stream=None):
    """Adjoint of probe_trace_soft: accumulates (+=) into grad_distance [P_total,N,N] and/or
    grad_radiance [P_total,N,N,3] (FP32); rgb is the forward's output."""
    lib = load_library()
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    P, N = grid.P_total, grid.N
    _need(radiance_half, P * N * N * 3, "radiance")
    rgb = _dev_tensor(rgb, torch.float32, "rgb")
    grad_rgb = _dev_tensor(grad_rgb, torch.float32, "grad_rgb")
    _need(rgb, 3 * rays, "rgb")
    _need(grad_rgb, 3 * rays, "grad_rgb")
    if grad_distance is None and grad_radiance is None:
        raise ProbeTraceError("probe_trace_soft_backward: no gradient requested")
    if grad_distance is not None:
        grad_distance = _dev_tensor(grad_distance, torch.float32, "grad_distance")
        _need(grad_distance, P * N * N, "grad_distance")
    if grad_radiance is not None:
        grad_radiance = _dev_tensor(grad_radiance, torch.float32, "grad_radiance")
        _need(grad_radiance, P * N * N * 3, "grad_radiance")
    _check(lib.probe_trace_soft_backward(grid.handle, _ptr(radiance_half), va, len(va), float(sigma), _ptr(rgb),
                                         _ptr(grad_rgb), _ptr(grad_distance), _ptr(grad_radiance),
                                         ctypes.byref(opts) if opts is not None else None, _stream(stream)))
    return grad_distance, grad_radiance


def probe_autotune(grid: ProbeGrid, radiance_half, views, opts: PtTraceOpts | None = None, stream=None):
    """Time candidate tile shapes and start levels; returns the tuned options."""
    lib = load_library()
    opts = opts if opts is not None else trace_opts()
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    rays = sum(v.width * v.height for v in va)
    radiance_half = _dev_tensor(radiance_half, torch.float16, "radiance (FP16)")
    _need(radiance_half, grid.P_total * grid.N * grid.N * 3, "radiance")
    rgb = torch.empty((rays, 3), dtype=torch.float32, device=radiance_half.device)
    _check(lib.probe_autotune(grid.handle, _ptr(radiance_half), va, len(va), _ptr(rgb), ctypes.byref(opts),
                              _stream(stream)))
    return opts


def adam_step(param, grad, exp_avg, exp_avg_sq, half_out, step: int, lr: float, betas=(0.9, 0.999),
              eps: float = 1e-8, weight_decay: float = 0.0, stream=None):
    """pt_adam_step: one Adam step on FP32 `param` in place (with its moments), writing
    param rounded to FP16 into `half_out` (or nothing if None)."""
    lib = load_library()
    param = _dev_tensor(param, torch.float32, "param")
    n = param.numel()
    grad = _dev_tensor(grad, torch.float32, "grad")
    exp_avg = _dev_tensor(exp_avg, torch.float32, "exp_avg")
    exp_avg_sq = _dev_tensor(exp_avg_sq, torch.float32, "exp_avg_sq")
    for t, what in ((grad, "grad"), (exp_avg, "exp_avg"), (exp_avg_sq, "exp_avg_sq")):
        _need(t, n, what)
    if half_out is not None:
        half_out = _dev_tensor(half_out, torch.float16, "half_out")
        _need(half_out, n, "half_out")
    _check(lib.pt_adam_step(_ptr(param), _ptr(grad), _ptr(exp_avg), _ptr(exp_avg_sq),
                            _ptr(half_out) if half_out is not None else None, int(n), int(step), float(lr),
                            float(betas[0]), float(betas[1]), float(eps), float(weight_decay), _stream(stream)))
    return param


class ProbeTraceFn(torch.autograd.Function):
    """rgb = trace(radiance) with the hit test held fixed.

    forward: the FP32 master radiance is rounded to the FP16 storage the trace reads (or
    `storage`, the caller's FP16 rounding of master, is read as it is);
    backward: probe_trace_backward into a zeroed FP32 buffer, passed straight through the
    FP16 rounding to the master.  keep_hits=True keeps the forward's hit and t outputs (12
    bytes per ray: probe and texel as int32, t as FP32) and runs probe_trace_backward_hits instead of recomputing the trace."""

    @staticmethod
    def forward(ctx, master, grid, views, opts=None, keep_hits=False, storage=None):
        if storage is None:
            storage = master.detach().to(torch.float16).contiguous()
        va = views if isinstance(views, ctypes.Array) else make_views(views)
        res = probe_trace(grid, storage, va, opts, want_t=keep_hits, want_status=False, want_hit=keep_hits)
        ctx.grid, ctx.views, ctx.opts = grid, va, opts
        ctx.shape = master.shape
        ctx.hits = (res["hit"], res["t"]) if keep_hits else None
        return res["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        g = torch.zeros(ctx.shape, dtype=torch.float32, device=grad_rgb.device)
        if ctx.hits is not None:
            probe_trace_backward_hits(ctx.grid, ctx.views, ctx.hits[0], ctx.hits[1], grad_rgb.contiguous().float(), g,
                                      ctx.opts)
        else:
            probe_trace_backward(ctx.grid, ctx.views, grad_rgb.contiguous().float(), g, ctx.opts)
        return g, None, None, None, None, None


class ProbeGeometryFn(torch.autograd.Function):
    """(rgb, t) = trace(distance, radiance) of a single-level grid, with the classification
    held fixed in the backward.

    forward: the grid's distance maps are replaced by `distance` ([P,N,N] FP32; the MIN
    pyramid is rebuilt) and the FP32 master radiance is rounded to FP16 storage;
    backward: probe_trace_backward_distance for the distances (through t and the motion of
    the radiance sample), probe_trace_backward for the radiance (straight through the FP16
    rounding).  t is +inf for rays that are not HIT: a loss on t masks them (they get no
    gradient either way)."""

    @staticmethod
    def forward(ctx, distance, master, grid, views, opts=None):
        if grid.P_total != grid.P:
            raise ProbeTraceError("ProbeGeometryFn: single-level grids only")
        grid.set_distance(distance.detach().contiguous())
        storage = master.detach().to(torch.float16).contiguous()
        va = views if isinstance(views, ctypes.Array) else make_views(views)
        res = probe_trace(grid, storage, va, opts, want_t=True, want_status=False, want_hit=False)
        ctx.grid, ctx.views, ctx.opts, ctx.storage = grid, va, opts, storage
        ctx.dshape, ctx.mshape = distance.shape, master.shape
        return res["rgb"], res["t"]

    @staticmethod
    def backward(ctx, grad_rgb, grad_t):
        gd = gm = None
        dev = ctx.storage.device
        grad_rgb = grad_rgb.contiguous().float() if grad_rgb is not None else None
        grad_t = grad_t.contiguous().float() if grad_t is not None else None
        if ctx.needs_input_grad[0] and (grad_rgb is not None or grad_t is not None):
            gd = torch.zeros(ctx.dshape, dtype=torch.float32, device=dev)
            probe_trace_backward_distance(ctx.grid, ctx.storage, ctx.views, grad_rgb, grad_t, gd, ctx.opts)
        if ctx.needs_input_grad[1] and grad_rgb is not None:
            gm = torch.zeros(ctx.mshape, dtype=torch.float32, device=dev)
            probe_trace_backward(ctx.grid, ctx.views, grad_rgb, gm, ctx.opts)
        return gd, gm, None, None, None


class ProbeSoftFn(torch.autograd.Function):
    """rgb = soft-visibility trace(distance, radiance) of a single-level grid
    (probe_trace_soft), with gradients for the stored distances that move the HIT/UNKNOWN
    decision and for the radiance (probe_trace_soft_backward).

    forward: the grid's distance maps are replaced by `distance` ([P,N,N] FP32; the MIN
    pyramid is rebuilt) and the FP32 master radiance is rounded to FP16 storage;
    backward: the candidates and the fire tests held, the FP16 rounding passed straight
    through to the master."""

    @staticmethod
    def forward(ctx, distance, master, grid, views, sigma, opts=None):
        if grid.P_total != grid.P:
            raise ProbeTraceError("ProbeSoftFn: single-level grids only")
        grid.set_distance(distance.detach().contiguous())
        storage = master.detach().to(torch.float16).contiguous()
        va = views if isinstance(views, ctypes.Array) else make_views(views)
        rgb = probe_trace_soft(grid, storage, va, sigma, opts)
        ctx.grid, ctx.views, ctx.opts, ctx.storage, ctx.sigma = grid, va, opts, storage, float(sigma)
        ctx.dshape, ctx.mshape = distance.shape, master.shape
        ctx.save_for_backward(rgb)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        (rgb,) = ctx.saved_tensors
        dev = ctx.storage.device
        gd = torch.zeros(ctx.dshape, dtype=torch.float32, device=dev) if ctx.needs_input_grad[0] else None
        gm = torch.zeros(ctx.mshape, dtype=torch.float32, device=dev) if ctx.needs_input_grad[1] else None
        if gd is not None or gm is not None:
            probe_trace_soft_backward(ctx.grid, ctx.storage, ctx.views, ctx.sigma, rgb, grad_rgb.contiguous().float(),
                                      gd, gm, ctx.opts)
        return gd, gm, None, None, None, None

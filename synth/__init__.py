"""Seeded synthetic inputs: rooms of boxes and spheres, probe bakes and camera views.

This module only makes inputs.  It holds none of the probe-tracing method: the
CPU oracle and the GPU library both consume what it produces and neither is
imported here.  The paper's own inputs (FARO scans of a lab room, Data
Collection / Data Processing sections) are not available, so these seeded
synthetic rooms stand in for them.

Scene recipe (all lengths relative to the probe spacing ``s``):

* room = [0, dims*s]^3, six inward-facing walls with albedo U[0.1,0.9]^3;
* one probe on every point of a regular lattice, ``origin = s/2`` (probe (i,j,k) at
  ``origin + (i,j,k)*s``), so every probe is strictly inside the room;
* K objects, each a box (prob 1/2: centre uniform in the room, two half-extents
  U[0.1,1.5]s and one, on a random axis, U[0.05,0.35]s) or a sphere (radius
  U[0.1,0.4]s), albedo U[0.1,0.9]^3; an object closer than 0.05s to any probe
  centre is redrawn;
* cameras uniform in the room with clearance >= 0.1s from every surface,
  yaw U[0,2pi), pitch U[-30,30] degrees, roll 0, vertical FOV 60 degrees.

Random numbers come from PCG32 (O'Neill 2014, pcg-random.org, the
``pcg32_random_r`` output function with the ``pcg32_srandom_r`` seeding).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_MASK64 = (1 << 64) - 1


class PCG32:
    """PCG32 generator (XSH-RR output, 64-bit LCG state)."""

    MULT = 6364136223846793005

    def __init__(self, initstate: int, initseq: int = 54):
        self.state = 0
        self.inc = ((initseq << 1) | 1) & _MASK64
        self.next_u32()
        self.state = (self.state + initstate) & _MASK64
        self.next_u32()

    def next_u32(self) -> int:
        old = self.state
        self.state = (old * self.MULT + self.inc) & _MASK64
        xorshifted = (((old >> 18) ^ old) >> 27) & 0xFFFFFFFF
        rot = old >> 59
        return ((xorshifted >> rot) | (xorshifted << ((-rot) & 31))) & 0xFFFFFFFF

    def uniform(self, a: float = 0.0, b: float = 1.0) -> float:
        return a + (b - a) * (self.next_u32() / 4294967296.0)

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on [lo, hi] inclusive."""
        return lo + int(self.uniform() * (hi - lo + 1))

    def normal(self) -> float:
        u1 = self.uniform()
        u2 = self.uniform()
        u1 = max(u1, 1e-12)
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


@dataclass
class Scene:
    dims: tuple            # probe grid dims (nx, ny, nz)
    spacing: float
    origin: float          # probe (0,0,0) sits at (origin, origin, origin)
    room_max: np.ndarray   # (3,) room is [0, room_max]
    wall_albedo: np.ndarray  # (6,3)
    obj_type: np.ndarray   # (K,) int32, 0 box, 1 sphere
    obj_param: np.ndarray  # (K,6) float64
    obj_albedo: np.ndarray  # (K,3)
    seed: int = 0
    accel: object = None   # optional _Accel (2D grid over x-y listing boxes per cell)

    @property
    def n_probes(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])

    def probe_positions(self) -> np.ndarray:
        """(P,3) float64, probe index p = i + nx*(j + ny*k)."""
        nx, ny, nz = self.dims
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        pos = np.stack([i, j, k], axis=-1).reshape(-1, 3).astype(np.float64)
        return self.origin + pos * self.spacing

    def with_albedos(self, seed: int) -> "Scene":
        """Same geometry, albedos redrawn from ``seed`` (the differentiable target field)."""
        rng = PCG32(seed)
        walls = np.array([[rng.uniform(0.1, 0.9) for _ in range(3)] for _ in range(6)])
        objs = np.array([[rng.uniform(0.1, 0.9) for _ in range(3)] for _ in range(len(self.obj_type))])
        return Scene(self.dims, self.spacing, self.origin, self.room_max.copy(), walls,
                     self.obj_type.copy(), self.obj_param.copy(), objs.reshape(-1, 3), seed, self.accel)


@dataclass
class View:
    pos: np.ndarray
    right: np.ndarray
    up: np.ndarray
    fwd: np.ndarray
    tan_half_fov_y: float
    width: int
    height: int

    def as_tuple(self):
        return (self.pos, self.right, self.up, self.fwd, self.tan_half_fov_y, self.width, self.height)


def make_scene(seed: int, dims, spacing: float, k_range) -> Scene:
    """Draw a seeded room of boxes and spheres (module docstring recipe)."""
    rng = PCG32(seed)
    dims = tuple(int(d) for d in dims)
    s = float(spacing)
    origin = 0.5 * s
    room_max = np.array(dims, dtype=np.float64) * s
    walls = np.array([[rng.uniform(0.1, 0.9) for _ in range(3)] for _ in range(6)])
    nx, ny, nz = dims
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    probes = origin + s * np.stack([ii, jj, kk], -1).reshape(-1, 3).astype(np.float64)
    K = rng.randint(k_range[0], k_range[1])
    types, params, albs = [], [], []
    for _ in range(K):
        for _attempt in range(2000):
            is_box = rng.uniform() < 0.5
            c = np.array([rng.uniform(0, room_max[a]) for a in range(3)])
            if is_box:
                h = np.array([rng.uniform(0.1, 1.5) * s, rng.uniform(0.1, 1.5) * s, 0.0])
                thin = rng.randint(0, 2)
                h[2] = rng.uniform(0.05, 0.35) * s
                h[[2, thin]] = h[[thin, 2]]
                q = np.abs(probes - c) - h
                outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
                dist = np.where(outside > 0, outside, q.max(axis=1))
                ok = bool(np.all(dist >= 0.05 * s))
                par = np.concatenate([c, h])
            else:
                r = rng.uniform(0.1, 0.4) * s
                ok = bool(np.all(np.linalg.norm(probes - c, axis=1) - r >= 0.05 * s))
                par = np.concatenate([c, [r, 0.0, 0.0]])
            alb = [rng.uniform(0.1, 0.9) for _ in range(3)]
            if ok:
                types.append(0 if is_box else 1)
                params.append(par)
                albs.append(alb)
                break
    return Scene(dims, s, origin, room_max, walls, np.array(types, dtype=np.int32),
                 np.array(params, dtype=np.float64).reshape(-1, 6),
                 np.array(albs, dtype=np.float64).reshape(-1, 3), seed)


class _AccelC(ctypes.Structure):
    _fields_ = [("agx", ctypes.c_int), ("agy", ctypes.c_int), ("acs", ctypes.c_double),
                ("astart", ctypes.c_void_p), ("aitems", ctypes.c_void_p)]


class _Accel:
    """2D uniform grid over the room's x-y extent listing, per cell, the boxes whose
    footprint overlaps it (for scenes of thousands of boxes)."""

    def __init__(self, room_max, obj_param, cs: float = 1.0):
        gx = max(1, int(math.ceil(room_max[0] / cs)))
        gy = max(1, int(math.ceil(room_max[1] / cs)))
        lists = [[] for _ in range(gx * gy)]
        for k, p in enumerate(obj_param):
            x0 = min(max(int(math.floor((p[0] - p[3]) / cs)), 0), gx - 1)
            x1 = min(max(int(math.floor((p[0] + p[3]) / cs)), 0), gx - 1)
            y0 = min(max(int(math.floor((p[1] - p[4]) / cs)), 0), gy - 1)
            y1 = min(max(int(math.floor((p[1] + p[4]) / cs)), 0), gy - 1)
            for j in range(y0, y1 + 1):
                for i in range(x0, x1 + 1):
                    lists[j * gx + i].append(k)
        self.start = np.zeros(gx * gy + 1, dtype=np.int32)
        self.start[1:] = np.cumsum([len(c) for c in lists])
        self.items = np.array([k for c in lists for k in c], dtype=np.int32)
        if self.items.size == 0:
            self.items = np.zeros(1, dtype=np.int32)
        self.c = _AccelC(gx, gy, float(cs), self.start.ctypes.data, self.items.ctypes.data)


def _acc(scene):
    return ctypes.byref(scene.accel.c) if scene.accel is not None else None


def make_city(seed: int, dims, spacing: float, k_range, footprint=(1.0, 4.0), height=(1.0, 12.0)) -> Scene:
    """A seeded city block: K ~ U{k_range} boxes standing on the ground (footprint sides
    U[footprint] x U[footprint], height U[height], centres uniform over the ground, no
    rejection: boxes overlap and may contain probes), albedo U[0.1,0.9]^3, inside a sky
    box [0, dims*s] whose six inward faces are the walls."""
    rng = PCG32(seed)
    dims = tuple(int(d) for d in dims)
    s = float(spacing)
    room_max = np.array(dims, dtype=np.float64) * s
    walls = np.array([[rng.uniform(0.1, 0.9) for _ in range(3)] for _ in range(6)])
    K = rng.randint(k_range[0], k_range[1])
    params, albs = [], []
    for _ in range(K):
        cx, cy = rng.uniform(0, room_max[0]), rng.uniform(0, room_max[1])
        hx = 0.5 * rng.uniform(*footprint) * s
        hy = 0.5 * rng.uniform(*footprint) * s
        hz = 0.5 * rng.uniform(*height) * s
        params.append([cx, cy, hz, hx, hy, hz])
        albs.append([rng.uniform(0.1, 0.9) for _ in range(3)])
    params = np.array(params, dtype=np.float64).reshape(-1, 6)
    sc = Scene(dims, s, 0.5 * s, room_max, walls, np.zeros(K, dtype=np.int32), params,
               np.array(albs, dtype=np.float64).reshape(-1, 3), seed)
    sc.accel = _Accel(room_max, params, cs=s)
    return sc


def _camera_basis(yaw: float, pitch: float):
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    up = np.cross(right, fwd)
    return right, up / np.linalg.norm(up), fwd


def clearance(scene: Scene, pt) -> float:
    lib = _load()
    pt = np.ascontiguousarray(pt, dtype=np.float64)
    return float(lib.synth_clearance(_dp(scene.room_max), int(len(scene.obj_type)),
                                     _ip(scene.obj_type), _dp(scene.obj_param), _dp(pt), _acc(scene)))


def _draw_position(rng: PCG32, scene: Scene, min_clear: float):
    for _ in range(100000):
        p = np.array([rng.uniform(0, scene.room_max[a]) for a in range(3)])
        if clearance(scene, p) >= min_clear:
            return p
    raise RuntimeError("could not place a camera")


FOV_Y_DEG = 60.0


def make_views(scene: Scene, seed: int, n_views: int, width=None, height=None, walk: bool = False,
               w_range=(256, 1920), h_range=(256, 1080), step: float = 0.25):
    """Seeded pinhole views.  ``walk`` makes a random walk (step 0.25, yaw += N(0,15deg)) with
    uneven resolutions drawn from ``w_range`` x ``h_range``; otherwise independent poses at
    ``width`` x ``height``."""
    rng = PCG32(seed, initseq=0x5EED)
    s = scene.spacing
    clear = 0.1 * s
    tanh = math.tan(math.radians(FOV_Y_DEG) / 2)
    views = []
    pos = _draw_position(rng, scene, clear)
    yaw = rng.uniform(0, 2 * math.pi)
    for v in range(n_views):
        if v > 0:
            if walk:
                for _ in range(200):
                    yaw_n = yaw + math.radians(15.0) * rng.normal()
                    cand = pos + step * np.array([math.cos(yaw_n), math.sin(yaw_n), 0.0])
                    if clearance(scene, cand) >= clear:
                        pos, yaw = cand, yaw_n
                        break
                else:
                    yaw = yaw + math.pi
            else:
                pos = _draw_position(rng, scene, clear)
                yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-30.0, 30.0))
        if walk:
            w = rng.randint(w_range[0], w_range[1])
            h = rng.randint(h_range[0], h_range[1])
        else:
            w, h = int(width), int(height)
        right, up, fwd = _camera_basis(yaw, pitch)
        views.append(View(pos.copy(), right, up, fwd, tanh, w, h))
    return views


@dataclass
class ProbeSet:
    """Baked probe maps.  Texel (i, j) of an N x N map has linear index j*N + i."""
    dims: tuple
    origin: np.ndarray      # (3,) float32
    spacing: np.ndarray     # (3,) float32
    N: int
    levels: int
    scene_min: np.ndarray   # (3,) float32
    scene_max: np.ndarray   # (3,) float32
    distance: np.ndarray    # (P,N,N) float32
    normal: np.ndarray      # (P,N,N,2) uint16, FP16 bits of the octahedral (u,v) of the normal
    radiance: np.ndarray    # (P,N,N,3) uint16, FP16 bits of RGB
    extra: dict = field(default_factory=dict)

    @property
    def n_probes(self) -> int:
        return int(self.distance.shape[0])

    def radiance_f32(self) -> np.ndarray:
        return self.radiance.view(np.float16).astype(np.float32)


def grid_positions(dims, origin: float, spacing: float) -> np.ndarray:
    """(P,3) float64 positions of a probe grid, p = i + nx*(j + ny*k)."""
    nx, ny, nz = (int(d) for d in dims)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return float(origin) + float(spacing) * np.stack([i, j, k], axis=-1).reshape(-1, 3).astype(np.float64)


def bake(scene: Scene, N: int, levels: int, nthreads: int | None = None, normals: str = "geometric",
         grid=None) -> ProbeSet:
    """Bake every probe of ``scene`` at N x N texels (centre-ray nearest surface).

    normals: "geometric" stores the surface's outward normal; "incoming" stores, as the
    paper's probe data generation literally does, the direction from the probe to the
    stored point (for a centre-ray bake, the texel's own centre direction, whose octahedral
    coordinates are the texel centre)."""
    if normals not in ("geometric", "incoming"):
        raise ValueError(normals)
    lib = _load()
    # grid = (dims, origin, spacing) of another probe grid in the same scene (default: the
    # scene's own); a probe inside a box sees D = 0 everywhere
    gdims, gorg, gsp = grid if grid is not None else (scene.dims, scene.origin, scene.spacing)
    pos = np.ascontiguousarray(grid_positions(gdims, gorg, gsp))
    P = len(pos)
    dist = np.empty((P, N, N), dtype=np.float32)
    nrm = np.empty((P, N, N, 2), dtype=np.float32)
    rad = np.empty((P, N, N, 3), dtype=np.float32)
    sid = np.empty((P, N, N), dtype=np.int32)
    nt = nthreads or min(16, os.cpu_count() or 1)
    lib.synth_bake(_dp(scene.room_max), _dp(scene.wall_albedo), int(len(scene.obj_type)),
                   _ip(scene.obj_type), _dp(scene.obj_param), _dp(scene.obj_albedo), P, _dp(pos), int(N),
                   _fp(dist), _fp(nrm), _fp(rad), _ip(sid), int(nt), _acc(scene))
    if normals == "incoming":
        c = (-1.0 + (2.0 * np.arange(N) + 1.0) / N).astype(np.float32)
        nrm[..., 0] = c[None, None, :]
        nrm[..., 1] = c[None, :, None]
    f32 = lambda v: np.array(v, dtype=np.float32)
    return ProbeSet(
        dims=tuple(int(d) for d in gdims), origin=f32([gorg] * 3), spacing=f32([gsp] * 3), N=int(N),
        levels=int(levels), scene_min=f32([0, 0, 0]), scene_max=f32(scene.room_max),
        distance=dist, normal=nrm.astype(np.float16).view(np.uint16),
        radiance=rad.astype(np.float16).view(np.uint16), extra=dict(surface_id=sid))


def sample_points(scene: Scene, n: int, seed: int):
    """A seeded synthetic point cloud standing in for the paper's scans (Data Collection):
    ``n`` points uniform by area over every surface (room walls, box faces, spheres), each
    with the surface's outward normal and the bake's shaded colour.  Points hidden inside
    other objects are kept (a projection onto a probe keeps the nearest point per texel, so
    they never win against the visible surface in front of them).  Random numbers: numpy's
    PCG64 seeded with ``seed``.  Returns float32 arrays points [n,3], colours [n,3],
    normals [n,3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = scene.room_max
    faces = []  # (centre, half-extent vector u, half-extent vector v, outward normal, albedo)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (0, 1):
            ctr = R / 2.0
            ctr = ctr.copy()
            ctr[a] = R[a] * side
            u = np.zeros(3); u[b] = R[b] / 2
            v = np.zeros(3); v[c] = R[c] / 2
            nrm = np.zeros(3); nrm[a] = 1.0 if side == 0 else -1.0  # walls face inward
            faces.append((ctr, u, v, nrm, scene.wall_albedo[2 * a + side]))
    spheres = []
    for k, (t, p) in enumerate(zip(scene.obj_type, scene.obj_param)):
        if t == 0:
            for a in range(3):
                b, c = (a + 1) % 3, (a + 2) % 3
                for sgn in (-1.0, 1.0):
                    ctr = p[:3].copy()
                    ctr[a] += sgn * p[3 + a]
                    u = np.zeros(3); u[b] = p[3 + b]
                    v = np.zeros(3); v[c] = p[3 + c]
                    nrm = np.zeros(3); nrm[a] = sgn
                    faces.append((ctr, u, v, nrm, scene.obj_albedo[k]))
        else:
            spheres.append((p[:3], p[3], scene.obj_albedo[k]))
    area = [4.0 * np.linalg.norm(f[1]) * np.linalg.norm(f[2]) for f in faces] + \
           [4.0 * math.pi * r * r for _, r, _ in spheres]
    area = np.array(area)
    which = rng.choice(len(area), size=n, p=area / area.sum())
    pts = np.empty((n, 3)); nrm = np.empty((n, 3)); alb = np.empty((n, 3))
    nf = len(faces)
    for i, f in enumerate(faces):
        m = which == i
        k = int(m.sum())
        if k:
            st = rng.uniform(-1.0, 1.0, size=(k, 2))
            pts[m] = f[0] + st[:, :1] * f[1] + st[:, 1:] * f[2]
            nrm[m] = f[3]
            alb[m] = f[4]
    for j, (c, r, a) in enumerate(spheres):
        m = which == nf + j
        k = int(m.sum())
        if k:
            d = rng.normal(size=(k, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts[m] = c + r * d
            nrm[m] = d
            alb[m] = a
    light = np.array(_LIGHT) / np.linalg.norm(_LIGHT)
    col = alb * (0.3 + 0.7 * np.maximum(nrm @ light, 0.0))[:, None]
    return pts.astype(np.float32), col.astype(np.float32), nrm.astype(np.float32)


_LIGHT = (0.3, 0.5, 0.8)  # the bake's light direction (before normalisation)


def cast(scene: Scene, origins: np.ndarray, dirs: np.ndarray):
    """Analytic nearest hit: returns t (inf if none), normal (n,3), albedo (n,3), surface id."""
    lib = _load()
    o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    t = np.empty(n, dtype=np.float64)
    nn = np.empty((n, 3), dtype=np.float64)
    alb = np.empty((n, 3), dtype=np.float64)
    ids = np.empty(n, dtype=np.int32)
    lib.synth_cast(_dp(scene.room_max), _dp(scene.wall_albedo), int(len(scene.obj_type)), _ip(scene.obj_type),
                   _dp(scene.obj_param), _dp(scene.obj_albedo), ctypes.c_int64(n), _dp(o), _dp(d), _dp(t),
                   _dp(nn), _dp(alb), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _acc(scene))
    return t, nn, alb, ids


# ---------------------------------------------------------------------------------------------
# Workload presets: the five synthetic configurations.
# ---------------------------------------------------------------------------------------------
CONFIGS = {
    "tiny": dict(seed=0, dims=(2, 2, 2), spacing=0.5, N=64, levels=4, k_range=(3, 6),
                 views=dict(seed=100, n=1, width=128, height=128)),
    "single": dict(seed=1, dims=(8, 8, 4), spacing=1.0, N=128, levels=5, k_range=(20, 40),
                   views=dict(seed=101, n=1, width=1920, height=1080)),
    "batched": dict(seed=1, dims=(8, 8, 4), spacing=1.0, N=128, levels=5, k_range=(20, 40),
                    views=dict(seed=2, n=64, walk=True)),
    "diff": dict(seed=3, dims=(16, 16, 8), spacing=1.0, N=256, levels=6, k_range=(20, 40),
                 target_seed=4, views=dict(seed=103, n=32, width=512, height=512)),
    # the paper's map configuration: a few probes (2x2x1 over a 4 x 4 x 2 room) with 2048^2
    # maps and a pyramid down to the 128^2 low-resolution map (5 levels)
    "paper": dict(seed=8, dims=(2, 2, 1), spacing=2.0, N=2048, levels=5, k_range=(6, 12),
                  views=dict(seed=108, n=1, width=1920, height=1080)),
    # two-level hierarchy over a city block: fine 64x64x16 probes (spacing 1) and coarse
    # 16x16x4 (spacing 4) whose planes are every 4th fine plane from the second
    "large": dict(seed=5, dims=(64, 64, 16), spacing=1.0, coarse_dims=(16, 16, 4), plane_off=1, ratio=4,
                  N=128, levels=5, k_range=(2000, 5000), height=(1.0, 12.0),
                  views=dict(seed=105, n=8, width=3840, height=2160)),
    # the same recipe on a 16x16x8 block (test size)
    "large_small": dict(seed=6, dims=(16, 16, 8), spacing=1.0, coarse_dims=(4, 4, 2), plane_off=1, ratio=4,
                        N=32, levels=3, k_range=(120, 300), height=(1.0, 6.0),
                        views=dict(seed=106, n=2, width=160, height=96)),
}


@dataclass
class TwoLevel:
    """A fine and a coarse probe set over one scene; coarse plane a of each axis is fine
    plane plane_off + a * ratio.  Coarse probe p is probe fine.n_probes + p of the pair."""
    fine: ProbeSet
    coarse: ProbeSet
    plane_off: tuple
    ratio: tuple

    @property
    def n_probes(self) -> int:
        return self.fine.n_probes + self.coarse.n_probes

    def radiance(self) -> np.ndarray:
        """[P_fine + P_coarse][N][N][3] FP16 bits, fine first."""
        return np.concatenate([self.fine.radiance, self.coarse.radiance])


def workload(name: str, N: int | None = None, levels: int | None = None, nthreads: int | None = None,
             n_views: int | None = None, size=None):
    """Build (scene, probes, views) for a named preset; N/levels/n_views/size override for tests."""
    cfg = CONFIGS[name]
    if "coarse_dims" in cfg:
        return workload_two_level(name, N, levels, nthreads, n_views, size)
    scene = make_scene(cfg["seed"], cfg["dims"], cfg["spacing"], cfg["k_range"])
    probes = bake(scene, N or cfg["N"], levels or cfg["levels"], nthreads)
    vc = cfg["views"]
    nv = n_views or vc["n"]
    if vc.get("walk"):
        views = make_views(scene, vc["seed"], nv, walk=True)
    else:
        w, h = size if size else (vc["width"], vc["height"])
        views = make_views(scene, vc["seed"], nv, w, h)
    return scene, probes, views


def workload_two_level(name: str, N=None, levels=None, nthreads=None, n_views=None, size=None):
    """(scene, TwoLevel, views) for a two-level preset (city block)."""
    cfg = CONFIGS[name]
    scene = make_city(cfg["seed"], cfg["dims"], cfg["spacing"], cfg["k_range"], height=cfg["height"])
    N, levels = N or cfg["N"], levels or cfg["levels"]
    fine = bake(scene, N, levels, nthreads)
    off, r, s = cfg["plane_off"], cfg["ratio"], cfg["spacing"]
    coarse = bake(scene, N, levels, nthreads, grid=(cfg["coarse_dims"], scene.origin + off * s, r * s))
    vc = cfg["views"]
    w, h = size if size else (vc["width"], vc["height"])
    views = make_views(scene, vc["seed"], n_views or vc["n"], w, h)
    return scene, TwoLevel(fine, coarse, (off,) * 3, (r,) * 3), views


# ---------------------------------------------------------------------------------------------
# native helper
# ---------------------------------------------------------------------------------------------
_lib = None


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def build_native(force: bool = True) -> str:
    src = os.path.join(_HERE, "bake.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_native(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        F = ctypes.POINTER(ctypes.c_float)
        I = ctypes.POINTER(ctypes.c_int32)
        V = ctypes.c_void_p
        lib.synth_bake.argtypes = [D, D, ctypes.c_int, I, D, D, ctypes.c_int, D, ctypes.c_int, F, F, F, I,
                                   ctypes.c_int, V]
        lib.synth_bake.restype = ctypes.c_int
        lib.synth_cast.argtypes = [D, D, ctypes.c_int, I, D, D, ctypes.c_int64, D, D, D, D, D, I, V]
        lib.synth_cast.restype = ctypes.c_int
        lib.synth_clearance.argtypes = [D, ctypes.c_int, I, D, D, V]
        lib.synth_clearance.restype = ctypes.c_double
        _lib = lib
    return _lib

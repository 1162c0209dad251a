"""CPU oracle for probe-grid ray tracing -- TEST INFRASTRUCTURE ONLY.

A plain, slow, double-precision implementation of what the GPU library computes.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import it; the product path never does, and it shares no code with the GPU
library.  The ray march itself lives in ``oracle.c`` (plain C, double); this module
builds the min pyramid, generates camera rays and marshals arrays.

Paper passages followed (arXiv 2507.14624):

* camera rays (X, w) and the radiance identity L_o(X, w1) = L_p(w2): Overview;
* octahedral encode/decode: Overview (octahedral mapping figure);
* low-resolution maps derived from the high-resolution ones: Implementation
  Details > Probe Data Generation (read as a 2x2 MIN pyramid);
* per-probe tracing, HIT/MISS/UNKNOWN: Methodology > Ray Tracing Using One Probe
  and the appendix algorithms;
* closest-first probes and the grid iterator: Methodology > Ray Trace Using
  Multiple Probes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MISS, HIT, UNKNOWN = 0, 1, 2

MG_FIRE, MG_DDA, MG_START, MG_OCTANT, MG_CELL = 1, 2, 4, 8, 16
MG_CAGE, MG_EYE, MG_CLASS, MG_THIT, MG_HIER = 32, 64, 128, 256, 512
MARGIN_BITS = {MG_FIRE: "fire", MG_DDA: "dda", MG_START: "start", MG_OCTANT: "octant", MG_CELL: "cell",
               MG_CAGE: "cage", MG_EYE: "eye", MG_CLASS: "class", MG_THIT: "thit", MG_HIER: "hier"}

DEFAULT_DELTA = 1e-5


class _Grid(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("N", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("smin", ctypes.c_double * 3), ("smax", ctypes.c_double * 3),
                ("dist", ctypes.c_void_p), ("nrm", ctypes.c_void_p), ("rad", ctypes.c_void_p),
                ("mips", ctypes.c_void_p), ("mip_off", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("thickness_rel", ctypes.c_double), ("eye_eps_rel", ctypes.c_double),
                ("background", ctypes.c_double * 3), ("delta", ctypes.c_double),
                ("max_probes_per_cell", ctypes.c_int32), ("check_hier", ctypes.c_int32),
                ("top_level", ctypes.c_int32), ("nthreads", ctypes.c_int32), ("nearest", ctypes.c_int32),
                ("soft", ctypes.c_int32)]


class _SoftOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("count", "probe", "texel", "a", "t", "rin", "rk", "c", "taps", "wts", "dtdr", "drgbdt", "rgb",
                 "trans", "margin")]


class _Out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("status", "t", "rgb", "probe", "texel", "margin", "tests", "normals", "flat_tests", "rank",
                 "taps", "wts", "score", "work", "dtdr", "drgbdt", "kink", "tcond")]


def build_native(force: bool = True) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-pthread", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_native(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_trace.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Opts), ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Out)]
        lib.oracle_trace.restype = ctypes.c_int
        lib.oracle_oct_encode.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_oct_decode.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_texel_sequence.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]
        lib.oracle_texel_sequence.restype = ctypes.c_int
        lib.oracle_bilinear_taps.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p]
        lib.oracle_cell_walk.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_cell_walk.restype = ctypes.c_int
        lib.oracle_cage_order.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_cage_order.restype = ctypes.c_int
        lib.oracle_trace_soft.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.POINTER(_Opts),
                                          ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(_SoftOut)]
        lib.oracle_trace_soft.restype = ctypes.c_int
        lib.oracle_half_to_double.argtypes = [ctypes.c_uint16]
        lib.oracle_half_to_double.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------------------------
# Min pyramid (Implementation Details > Probe Data Generation: coarse maps from fine ones)
# ---------------------------------------------------------------------------------------------
def min_mips(distance: np.ndarray, levels: int) -> list:
    """Level l texel (i,j) = min of level l-1 texels (2i..2i+1, 2j..2j+1); NaN = no data."""
    out = [np.ascontiguousarray(distance, dtype=np.float32)]
    for _ in range(1, levels):
        d = out[-1]
        P, n, _ = d.shape
        q = d.reshape(P, n // 2, 2, n // 2, 2)
        out.append(np.fmin(np.fmin(q[:, :, 0, :, 0], q[:, :, 0, :, 1]),
                           np.fmin(q[:, :, 1, :, 0], q[:, :, 1, :, 1])).astype(np.float32))
    return out


class Grid:
    """Probe grid as the oracle sees it (numpy arrays kept alive here)."""

    def __init__(self, dims, origin, spacing, N, levels, scene_min, scene_max, distance, normal_bits,
                 radiance):
        self.dims = tuple(int(d) for d in dims)
        if min(self.dims) < 1 or (np.prod(self.dims) >= 8 and min(self.dims) < 2):
            # 8 or more probes form a grid (every axis >= 2); fewer are traced all together
            raise ValueError(f"probe layout {self.dims}: 8 or more probes need at least 2 per axis")
        self.N = int(N)
        self.levels = int(levels)
        self.origin = np.asarray(origin, dtype=np.float64)
        self.spacing = np.asarray(spacing, dtype=np.float64)
        self.scene_min = np.asarray(scene_min, dtype=np.float64)
        self.scene_max = np.asarray(scene_max, dtype=np.float64)
        self.distance = np.ascontiguousarray(distance, dtype=np.float32)
        self.normal_bits = np.ascontiguousarray(normal_bits, dtype=np.uint16)
        self.set_radiance(radiance)
        pyr = min_mips(self.distance, self.levels)
        self.mip_levels = pyr
        off = [0] * self.levels
        chunks = []
        pos = 0
        for l in range(1, self.levels):
            off[l] = pos
            chunks.append(pyr[l].ravel())
            pos += pyr[l].size
        self.mips = np.ascontiguousarray(np.concatenate(chunks) if chunks else np.zeros(1, np.float32))
        self.mip_off = np.array(off, dtype=np.int64)

    @classmethod
    def from_probes(cls, probes, radiance=None):
        rad = probes.radiance.view(np.float16).astype(np.float32) if radiance is None else radiance
        return cls(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                   probes.scene_max, probes.distance, probes.normal, rad)

    def set_radiance(self, radiance):
        """Radiance [P][N][N][3]: FP16 bits (uint16) or real values."""
        r = np.asarray(radiance)
        if r.dtype == np.uint16:
            r = r.view(np.float16)
        self.radiance = np.ascontiguousarray(r, dtype=np.float32)

    def probe_position(self, p: int) -> np.ndarray:
        nx, ny, _ = self.dims
        ijk = np.array([p % nx, (p // nx) % ny, p // (nx * ny)], dtype=np.float64)
        return self.origin + ijk * self.spacing

    def _struct(self) -> _Grid:
        g = _Grid()
        g.dims[:] = self.dims
        g.N = self.N
        g.levels = self.levels
        g.origin[:] = list(self.origin)
        g.spacing[:] = list(self.spacing)
        g.smin[:] = list(self.scene_min)
        g.smax[:] = list(self.scene_max)
        g.dist = self.distance.ctypes.data
        g.nrm = self.normal_bits.ctypes.data
        g.rad = self.radiance.ctypes.data
        g.mips = self.mips.ctypes.data
        g.mip_off = self.mip_off.ctypes.data
        return g


# ---------------------------------------------------------------------------------------------
# Camera rays (Overview: a ray (X, w) per pixel)
# ---------------------------------------------------------------------------------------------
def view_rays(pos, right, up, fwd, tan_half_fov_y, width, height, pixels=None):
    """Pinhole rays in double from the FP32 view parameters.

    Pixel (x, y), row 0 at the top:  w = normalize(fwd + a right + b up) with
    a = (2(x+1/2)/W - 1)(W/H) tan, b = (1 - 2(y+1/2)/H) tan.  ``pixels`` is an optional
    array of linear pixel indices y*W + x (default: all, row-major)."""
    f32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)
    pos, right, up, fwd = f32(pos), f32(right), f32(up), f32(fwd)
    th = float(np.float32(tan_half_fov_y))
    W, H = int(width), int(height)
    idx = np.arange(W * H, dtype=np.int64) if pixels is None else np.asarray(pixels, dtype=np.int64)
    x = (idx % W).astype(np.float64)
    y = (idx // W).astype(np.float64)
    a = (2.0 * (x + 0.5) / W - 1.0) * (W / H) * th
    b = (1.0 - 2.0 * (y + 0.5) / H) * th
    d = fwd[None, :] + a[:, None] * right[None, :] + b[:, None] * up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(pos, d.shape).copy()
    return o, d


# ---------------------------------------------------------------------------------------------
# Tracing
# ---------------------------------------------------------------------------------------------
def default_opts(N: int, **kw) -> dict:
    o = dict(thickness_rel=8.0 / N, eye_eps_rel=1e-6, background=(0.0, 0.0, 0.0), delta=DEFAULT_DELTA,
             max_probes_per_cell=8, check_hier=1, top_level=-1, nthreads=os.cpu_count() or 1, nearest=False,
             soft=False)
    o.update(kw)
    return o


class _Level2(ctypes.Structure):
    _fields_ = [("coarse", ctypes.c_void_p), ("plane_off", ctypes.c_int32 * 3), ("ratio", ctypes.c_int32 * 3)]


def trace(grid: Grid, origins: np.ndarray, dirs: np.ndarray, coarse=None, **kw) -> dict:
    """Trace rays; returns per-ray arrays (status, t, rgb, probe, texel, margin, tests,
    normals, flat_tests, rank, taps, wts, score, work, dtdr, drgbdt, kink, tcond).  ``score`` is the smallest gap/error-scale
    ratio over the ray's decisions; ``margin`` has a bit per decision kind with ratio <= delta;
    ``work`` counts probe traces, pieces marched and cells visited."""
    lib = _load()
    o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    opts = default_opts(grid.N, **kw)
    oo = _Opts()
    oo.thickness_rel = float(opts["thickness_rel"])
    oo.eye_eps_rel = float(opts["eye_eps_rel"])
    oo.background[:] = [float(c) for c in opts["background"]]
    oo.delta = float(opts["delta"])
    oo.max_probes_per_cell = int(opts["max_probes_per_cell"])
    oo.check_hier = int(opts["check_hier"])
    oo.top_level = int(opts["top_level"])
    oo.nthreads = int(opts["nthreads"])
    oo.nearest = int(bool(opts["nearest"]))
    oo.soft = int(bool(opts["soft"]))
    res = dict(status=np.empty(n, np.uint8), t=np.empty(n, np.float64), rgb=np.empty((n, 3), np.float64),
               probe=np.empty(n, np.int32), texel=np.empty(n, np.int32), margin=np.empty(n, np.int32),
               tests=np.empty(n, np.int32), normals=np.empty(n, np.int32), flat_tests=np.empty(n, np.int32),
               rank=np.empty(n, np.int32), taps=np.empty((n, 4), np.int32), wts=np.empty((n, 4), np.float64),
               score=np.empty(n, np.float64), work=np.empty((n, 3), np.int32), dtdr=np.empty(n, np.float64),
               drgbdt=np.empty((n, 3), np.float64), kink=np.empty(n, np.int32), tcond=np.empty(n, np.float64))
    out = _Out()
    for k, v in res.items():
        setattr(out, k, v.ctypes.data)
    g = grid._struct()
    if coarse is None:
        lib.oracle_trace(ctypes.byref(g), ctypes.byref(oo), n, _ptr(o), _ptr(d), ctypes.byref(out))
    else:
        # two-level hierarchy: coarse = (coarse Grid, plane_off[3], ratio[3]); coarse plane a
        # is fine plane plane_off + a * ratio; coarse probe p is reported as P_fine + p
        cgrid, off, ratio = coarse
        cs = cgrid._struct()
        L2 = _Level2()
        L2.coarse = ctypes.addressof(cs)
        L2.plane_off[:] = [int(x) for x in off]
        L2.ratio[:] = [int(x) for x in ratio]
        lib.oracle_trace2(ctypes.byref(g), ctypes.byref(L2), ctypes.byref(oo), n, _ptr(o), _ptr(d),
                          ctypes.byref(out))
    return res


def trace_soft(grid: Grid, origins: np.ndarray, dirs: np.ndarray, sigma: float, coarse=None, kcap: int = 64,
               **kw) -> dict:
    """Soft visibility (an extension; the paper's classification is hard): every probe trace
    whose first firing texel faces the ray is a candidate j, in walk order, accepted with
    weight a_j = logistic((r_j (1 + tau) - rho_in,j) / (sigma r_j)); the colour is
    sum_j a_j prod_{i<j} (1 - a_i) c_j + prod_j (1 - a_j) background, the walk stopping once
    the remaining weight is <= 1e-6.  Returns per-ray arrays: count [n] (-1: more than kcap
    candidates), per-candidate probe/texel/a/t/rin/rk/dtdr [n,kcap], c/drgbdt [n,kcap,3],
    taps/wts [n,kcap,4], and rgb [n,3], trans [n] (weight of the background), margin [n]."""
    lib = _load()
    o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    opts = default_opts(grid.N, **kw)
    opts["soft"] = True
    oo = _Opts()
    oo.thickness_rel = float(opts["thickness_rel"])
    oo.eye_eps_rel = float(opts["eye_eps_rel"])
    oo.background[:] = [float(c) for c in opts["background"]]
    oo.delta = float(opts["delta"])
    oo.max_probes_per_cell = int(opts["max_probes_per_cell"])
    oo.check_hier = 0
    oo.top_level = int(opts["top_level"])
    oo.nthreads = int(opts["nthreads"])
    oo.nearest = int(bool(opts["nearest"]))
    oo.soft = 1
    K = int(kcap)
    res = dict(count=np.empty(n, np.int32), probe=np.full((n, K), -1, np.int32), texel=np.full((n, K), -1, np.int32),
               a=np.zeros((n, K)), t=np.zeros((n, K)), rin=np.zeros((n, K)), rk=np.zeros((n, K)),
               c=np.zeros((n, K, 3)), taps=np.zeros((n, K, 4), np.int32), wts=np.zeros((n, K, 4)),
               dtdr=np.zeros((n, K)), drgbdt=np.zeros((n, K, 3)), rgb=np.empty((n, 3)), trans=np.empty(n),
               margin=np.empty(n, np.int32))
    out = _SoftOut()
    for k, v in res.items():
        setattr(out, k, v.ctypes.data)
    g = grid._struct()
    L2 = None
    if coarse is not None:
        cgrid, off, ratio = coarse
        cs = cgrid._struct()
        L2 = _Level2()
        L2.coarse = ctypes.addressof(cs)
        L2.plane_off[:] = [int(x) for x in off]
        L2.ratio[:] = [int(x) for x in ratio]
    rc = lib.oracle_trace_soft(ctypes.byref(g), ctypes.byref(L2) if L2 is not None else None, ctypes.byref(oo),
                               float(sigma), K, n, _ptr(o), _ptr(d), ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_trace_soft: sigma must be > 0 and kcap >= 1")
    res["sigma"] = float(sigma)
    res["tau"] = float(opts["thickness_rel"])
    res["background"] = np.asarray(opts["background"], dtype=np.float64)
    return res


def vjp_soft(grid, result: dict, grad_rgb: np.ndarray):
    """Adjoint of trace_soft's colour (an extension beyond the paper): gradients with respect
    to the stored distances [P,N,N] and the radiance [P,N,N,3], the fire tests and the
    candidates held.  With w_j = a_j prod_{i<j} (1 - a_i), A_j = sum_{k<=j} w_k c_k and g the
    upstream gradient of rgb:
        dL/dx_j   = g . (w_j (1 - a_j) c_j - a_j (rgb - A_j))       (x_j the logistic's argument)
        dL/dr_j  += dL/dx_j * rho_in,j / (sigma r_j^2) + w_j (g . dc_j/dt) dt_j/dr_j
        dL/dRad  += w_j * bilinear weight * g at each of candidate j's taps.
    Accumulated in double."""
    grids = grid if isinstance(grid, (list, tuple)) else (grid,)  # (fine, coarse): probes concatenated
    P = sum(gr.distance.shape[0] for gr in grids)
    N = grids[0].N
    gd = np.zeros(P * N * N, dtype=np.float64)
    grad = np.zeros((P * N * N, 3), dtype=np.float64)
    if np.any(result["count"] < 0):
        raise ValueError("vjp_soft: a ray needed more candidates than kcap")
    g = np.asarray(grad_rgb, dtype=np.float64).reshape(-1, 3)
    rgb = result["rgb"]
    sigma = result["sigma"]
    n, K = result["a"].shape
    Pj = np.ones(n)
    A = np.zeros((n, 3))
    for j in range(K):
        on = result["count"] > j
        if not on.any():
            break
        a = result["a"][on, j]
        c = result["c"][on, j]
        wj = a * Pj[on]
        A[on] += wj[:, None] * c
        dx = np.einsum("ij,ij->i", g[on], wj[:, None] * (1.0 - a)[:, None] * c - a[:, None] * (rgb[on] - A[on]))
        rk = result["rk"][on, j]
        rin = result["rin"][on, j]
        dxdr = np.where(rk > 0.0, rin / (sigma * np.where(rk > 0.0, rk, 1.0) ** 2), 0.0)
        geo = wj * np.einsum("ij,ij->i", g[on], result["drgbdt"][on, j]) * result["dtdr"][on, j]
        # dt/dr is infinite at an exact tangency: such a term is left out
        geo = np.where((wj != 0.0) & np.isfinite(geo), geo, 0.0)
        flat = result["probe"][on, j].astype(np.int64) * (N * N) + result["texel"][on, j]
        np.add.at(gd, flat, dx * dxdr + geo)
        taps = result["probe"][on, j].astype(np.int64)[:, None] * (N * N) + result["taps"][on, j]
        for k in range(4):
            np.add.at(grad, taps[:, k], (wj * result["wts"][on, j, k])[:, None] * g[on])
        Pj[on] *= 1.0 - a
    return gd.reshape(P, N, N), grad.reshape(P, N, N, 3)


def trace_view(grid: Grid, view, pixels=None, **kw) -> dict:
    o, d = view_rays(*view, pixels=pixels)
    return trace(grid, o, d, **kw)


def vjp(grid, result: dict, grad_rgb: np.ndarray) -> np.ndarray:
    """Adjoint of the radiance fetch with the hit test held fixed (an extension beyond the paper, which renders forward only):
    dL/dRad[p][tap][c] = sum over HIT rays of w_tap * dL/drgb[c].  Accumulated in double,
    duplicate taps add up."""
    grids = grid if isinstance(grid, (list, tuple)) else (grid,)  # (fine, coarse): probes concatenated
    P = sum(gr.distance.shape[0] for gr in grids)
    N = grids[0].N
    g = np.zeros((P * N * N, 3), dtype=np.float64)
    hit = result["status"] == HIT
    if not np.any(hit):
        return g.reshape(P, N, N, 3)
    probe = result["probe"][hit].astype(np.int64)
    taps = result["taps"][hit].astype(np.int64)
    wts = result["wts"][hit]
    gr = np.asarray(grad_rgb, dtype=np.float64).reshape(-1, 3)[hit]
    flat = probe[:, None] * (N * N) + taps
    for k in range(4):
        np.add.at(g, flat[:, k], wts[:, k:k + 1] * gr)
    return g.reshape(P, N, N, 3)


def vjp_distance(grid, result: dict, grad_rgb=None, grad_t=None) -> np.ndarray:
    """Adjoint of the stored distances with the classification held fixed (an extension
    beyond the paper, which renders forward only).  A HIT ray depends on the distance r of
    its hit texel only, through the hit distance t: dt/dr is 1 for the eye-aligned lookup,
    0 when the hit is the texel's entry point, r / sqrt(r^2 - d_perp^2) for the root of
    |X - O + t w| = r; the bilinear radiance sample moves with the hit point, d rgb/dt.  So
    dL/dr[p][k] = sum over HIT rays on (p, k) of dt/dr (dL/dt + dL/drgb . drgb/dt), in
    double.  [P][N][N]."""
    grids = grid if isinstance(grid, (list, tuple)) else (grid,)
    P = sum(gr.distance.shape[0] for gr in grids)
    N = grids[0].N
    g = np.zeros(P * N * N, dtype=np.float64)
    hit = result["status"] == HIT
    if not np.any(hit):
        return g.reshape(P, N, N)
    up = np.zeros(int(hit.sum()))
    if grad_t is not None:
        up += np.asarray(grad_t, dtype=np.float64).reshape(-1)[hit]
    if grad_rgb is not None:
        up += np.sum(np.asarray(grad_rgb, dtype=np.float64).reshape(-1, 3)[hit] * result["drgbdt"][hit], axis=1)
    flat = result["probe"][hit].astype(np.int64) * (N * N) + result["texel"][hit].astype(np.int64)
    np.add.at(g, flat, result["dtdr"][hit] * up)
    return g.reshape(P, N, N)


# ---------------------------------------------------------------------------------------------
# Small hooks used by the oracle's own tests
# ---------------------------------------------------------------------------------------------
def oct_encode(d) -> np.ndarray:
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(2, dtype=np.float64)
    lib.oracle_oct_encode(_ptr(d), _ptr(out))
    return out


def oct_decode(uv) -> np.ndarray:
    lib = _load()
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    lib.oracle_oct_decode(_ptr(uv), _ptr(out))
    return out


def texel_sequence(N: int, xp, w, ta: float, tb: float, cap: int = 100000):
    """Flat level-0 texel sequence of the ray X' + t w over [ta, tb] seen from a probe at the
    origin: arrays (ij [n,2], t_in/t_out [n,2], piece [n])."""
    lib = _load()
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    ij = np.empty((cap, 2), np.int32)
    tio = np.empty((cap, 2), np.float64)
    piece = np.empty(cap, np.int32)
    n = lib.oracle_texel_sequence(int(N), _ptr(xp), _ptr(w), float(ta), float(tb), cap, _ptr(ij), _ptr(tio),
                                  _ptr(piece))
    n = min(n, cap)
    return ij[:n].copy(), tio[:n].copy(), piece[:n].copy()


def cell_walk(grid: Grid, X, w, cap: int = 4096):
    """The grid iterator's walk of the ray (X, w) (Ray Trace Using Multiple Probes > Grid
    Iterator): arrays (cells [n,3] int, intervals [n,2] = (ta, tb)) in ray order."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    cells = np.empty((cap, 3), np.int32)
    tab = np.empty((cap, 2), np.float64)
    g = grid._struct()
    n = lib.oracle_cell_walk(ctypes.byref(g), _ptr(X), _ptr(w), cap, _ptr(cells), _ptr(tab))
    n = min(n, cap)
    return cells[:n].copy(), tab[:n].copy()


def cage_order(grid: Grid, cell, X) -> np.ndarray:
    """Probe indices of the cage of `cell` in the order the trace tries them for a ray
    from X (Ray Trace Using Multiple Probes > Less Than 8 Probes)."""
    lib = _load()
    c = np.ascontiguousarray(cell, dtype=np.int32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.empty(8, np.int32)
    g = grid._struct()
    n = lib.oracle_cage_order(ctypes.byref(g), _ptr(c), _ptr(X), _ptr(out))
    return out[:n].copy()


def bilinear_taps(u: float, v: float, N: int):
    lib = _load()
    idx = np.empty(4, np.int32)
    wt = np.empty(4, np.float64)
    lib.oracle_bilinear_taps(float(u), float(v), int(N), _ptr(idx), _ptr(wt))
    return idx, wt


def half_to_double(h: int) -> float:
    return float(_load().oracle_half_to_double(int(h)))


# FP32 operations of one step of the reference schedule (an FMA counts 2, a compare,
# min/max or reciprocal 1):
#   texel test: ray point at the texel exit (3 FMA = 6), squared radial distance (mul +
#     2 FMA = 5), max with the entry value (1), stored value squared and compare (2), next
#     boundary crossing (2 FMA + reciprocal + mul + sign test = 8), min of candidates (2)
#   piece: six linear forms (6 x 5), two motion signs (2 x 3), start texel (3 FMA +
#     reciprocal + 2 mul = 9), two first crossings (2 x 8)
#   probe trace: probe position (3 FMA = 6), relative origin (3), its squared length (5),
#     three octant cuts (3 x 2)
#   cell: three plane crossings (3 x 2) and their minimum (3)
#   HIT: normal decode and facing test (11), larger root (20), hit direction encode (8),
#     bilinear weights (10), 4 taps x 3 channels FMA (24)
#   ray: pinhole direction (25), scene-box exit (9)
FLOPS = dict(test=24, piece=61, probe=20, cell=9, hit=73, ray=34)


def algorithmic_flops(result: dict) -> np.ndarray:
    """Per-ray FP32 operations of the reference schedule (FLOPS table x the oracle's counts)."""
    w = result["work"].astype(np.int64)
    return (FLOPS["test"] * result["tests"].astype(np.int64) + FLOPS["piece"] * w[:, 1]
            + FLOPS["probe"] * w[:, 0] + FLOPS["cell"] * w[:, 2]
            + FLOPS["hit"] * (result["status"] == HIT).astype(np.int64) + FLOPS["ray"])


def algorithmic_bytes(result: dict) -> np.ndarray:
    """Per-ray algorithmic bytes of the reference hierarchical schedule:
    4 B per distance/mip fetch + 4 B per normal fetch + 24 B of radiance taps on HIT
    (4 taps x RGB FP16) + 17 B of output (rgb FP32, t FP32, status u8)."""
    return (4 * result["tests"].astype(np.int64) + 4 * result["normals"].astype(np.int64)
            + 24 * (result["status"] == HIT).astype(np.int64) + 17)

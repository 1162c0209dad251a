"""Probe baking from a point cloud, the oracle's definition (test infrastructure only).

Implementation Details, Probe Data Generation: every point is taken into the probe's frame
and projected onto its octahedral map; a texel keeps the point nearest to the probe; the
distance map holds that distance, the radiance map its colour, and the "normal" map either
the point's surface normal (our reading R1) or, as the paper literally does, the normalised
vector from the probe to the point.

Precision: the paper fixes none.  The nearest point per texel is an integer decision, so
it is taken in the GPU kernel's precision, FP32, with the same operations written out
here in numpy float32 (each numpy float32 operation rounds once, like the kernel's
uncontracted operations):
    O   = fl32(origin + k * spacing)            (one rounding: a fused multiply-add)
    d   = p - O                                 (per axis)
    r2  = (dx*dx + dy*dy) + dz*dz
    L1  = (|dx| + |dy|) + |dz|,  q = d / L1     (IEEE division)
    (u, v) = (qx, qy) if qz >= 0 else ((1 - |qy|) sgn qx, (1 - |qx|) sgn qy)
    i   = clamp(floor((u + 1) * N/2), 0, N-1)   (j from v likewise; texel j*N + i)
The winner of a texel has the smallest r2, ties to the smaller point index.  Outputs:
distance = sqrt(r2) (FP32, correctly rounded), radiance = colour rounded to FP16,
normal = the octahedral (u, v) above of the normal (or of d) rounded to FP16.  A texel no
point projects to has no data: distance NaN, normal (0, 0), radiance 0.  Points at the
probe centre (L1 = 0) have no direction and are skipped.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def _oct_uv(x, y, z):
    L = (np.abs(x) + np.abs(y)) + np.abs(z)
    qx, qy, qz = x / L, y / L, z / L
    sx = np.where(qx >= 0, f32(1), f32(-1))
    sy = np.where(qy >= 0, f32(1), f32(-1))
    u = np.where(qz >= 0, qx, (f32(1) - np.abs(qy)) * sx).astype(f32)
    v = np.where(qz >= 0, qy, (f32(1) - np.abs(qx)) * sy).astype(f32)
    return u, v, L


def probe_origins(dims, origin, spacing) -> np.ndarray:
    """[P,3] float32 probe centres, probe (i,j,k) = i + nx (j + ny k), each coordinate
    origin + k spacing rounded once to FP32."""
    nx, ny, nz = (int(d) for d in dims)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([i, j, k], -1).reshape(-1, 3).astype(np.float64)
    org = np.asarray(origin, np.float32).astype(np.float64)
    spc = np.asarray(spacing, np.float32).astype(np.float64)
    return (idx * spc + org).astype(f32)


def bake_points(dims, origin, spacing, N: int, points, colors, normals=None, probes=None):
    """Bake probes (all, or the indices in ``probes``) from a point cloud.  Returns
    distance [P,N,N] float32, normal [P,N,N,2] uint16 (FP16 bits), radiance [P,N,N,3]
    uint16 (FP16 bits), and the winning point index per texel [P,N,N] int64 (-1: none)."""
    pts = np.ascontiguousarray(points, dtype=f32)
    col = np.ascontiguousarray(colors, dtype=f32)
    nrm = None if normals is None else np.ascontiguousarray(normals, dtype=f32)
    O = probe_origins(dims, origin, spacing)
    sel = np.arange(len(O)) if probes is None else np.asarray(probes)
    P = len(sel)
    M = len(pts)
    hN = f32(N // 2)
    dist = np.full((P, N * N), np.nan, dtype=f32)
    nuv = np.zeros((P, N * N, 2), dtype=np.float16)
    rad = np.zeros((P, N * N, 3), dtype=np.float16)
    win = np.full((P, N * N), -1, dtype=np.int64)
    ids = np.arange(M)
    for a, p in enumerate(sel):
        d = pts - O[p]
        dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
        r2 = (dx * dx + dy * dy) + dz * dz
        u, v, L = _oct_uv(dx, dy, dz)
        ok = L > 0
        i = np.clip(np.floor((u + f32(1)) * hN), 0, N - 1).astype(np.int64)
        j = np.clip(np.floor((v + f32(1)) * hN), 0, N - 1).astype(np.int64)
        tex = j * N + i
        tex, r2s, idx = tex[ok], r2[ok], ids[ok]
        order = np.lexsort((idx, r2s, tex))  # by texel, then r2, then point index
        tex, r2s, idx = tex[order], r2s[order], idx[order]
        first = np.ones(len(tex), bool)
        first[1:] = tex[1:] != tex[:-1]
        t, w, rr = tex[first], idx[first], r2s[first]
        win[a, t] = w
        dist[a, t] = np.sqrt(rr)
        rad[a, t] = col[w].astype(np.float16)
        if nrm is None:
            src = d[w]
        else:
            src = nrm[w]
        nu, nv, _ = _oct_uv(src[:, 0], src[:, 1], src[:, 2])
        nuv[a, t, 0] = nu.astype(np.float16)
        nuv[a, t, 1] = nv.astype(np.float16)
    return (dist.reshape(P, N, N), nuv.view(np.uint16).reshape(P, N, N, 2),
            rad.view(np.uint16).reshape(P, N, N, 3), win.reshape(P, N, N))

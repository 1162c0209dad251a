"""The premises of the cage tables' known-answer rules, checked against the oracle's own walk
(no GPU).  Clear probes: a probe whose smallest stored distance, over the texels a piece in
each octant the cell region admits can reach, exceeds the region's farthest point from the
probe has no level-0 texel that fires along any segment the grid iterator gives that cell.
The rule is restated here from its definition (octant triangles of the octahedral map with
a band across the fold, the neighbouring quadrants' edge texels, the cell region clamped out
to the scene box and the eye) and each certified (ray, cell, probe) is checked on the flat
level-0 texel sequence in double precision: every texel's stored distance is at least the
radial distance at both ends of its span.  Eye cell: every ray's walk starts in the eye's
cell at t = 0, and its first texel there is the texel of the eye's own direction from the
probe, so a probe whose stored distance in that direction lies below the eye's radial
distance (shadow-entry rule) answers UNKNOWN for every ray of the view.  Solid probes: with
every stored distance <= 0 the oracle's walk answers UNKNOWN for every ray, and HIT at
t = 0 for an eye on a probe."""
import numpy as np

import oracle
from conftest import workload


def _octant_minima(D):
    """[P][8] minima, octant o = [x >= 0] + 2 [y >= 0] + 4 [z >= 0]."""
    P, N, _ = D.shape
    h = N // 2
    i = np.arange(N)
    sx = (i >= h).astype(int)
    a = np.where(sx == 1, i - h, h - 1 - i)
    out = np.full((P, 8), np.inf)
    Dn = np.where(np.isnan(D), np.inf, D)
    for o in range(8):
        ox, oy, oz = o & 1, (o >> 1) & 1, o >> 2
        A = a[None, :]          # column (x) index -> a
        B = a[:, None]          # row (y) index -> b
        SX = sx[None, :]
        SY = sx[:, None]
        own = (SX == ox) & (SY == oy)
        edge = ((SX == ox) | (A == 0)) & ((SY == oy) | (B == 0))
        tri = (A + B <= h + 1) if oz else (A + B >= h - 3)
        mask = (own & tri) | (~own & edge)
        out[:, o] = np.where(mask[None], Dn, np.inf).reshape(P, -1).min(1)
    return out


def test_clear_probes_never_fire_on_their_cells():
    scene, probes, views = workload("diff", N=32, levels=3, n_views=1, size=(40, 32))
    og = oracle.Grid.from_probes(probes)
    N, P = probes.N, probes.n_probes
    D = probes.distance.reshape(P, N, N).astype(np.float64)
    om = _octant_minima(D)
    nx, ny, nz = probes.dims
    cmax = np.array(probes.dims) - 2
    org, spc = np.array(probes.origin, float), np.array(probes.spacing, float)
    smin, smax = np.array(probes.scene_min, float), np.array(probes.scene_max, float)
    o, d = oracle.view_rays(*views[0].as_tuple())
    rng = np.random.default_rng(0)
    certified = checked_texels = 0
    for r in rng.choice(len(o), 400, replace=False):
        X, w = o[r], d[r]
        cells, iv = oracle.cell_walk(og, X, w)
        for cell, (ta, tb) in zip(cells, iv):
            lo = org + cell * spc
            hi = lo + spc
            for a in range(3):
                ext = 1e-3 * (smax[a] - smin[a])
                if cell[a] == 0:
                    lo[a] = min(smin[a], X[a], lo[a]) - ext
                if cell[a] == cmax[a]:
                    hi[a] = max(smax[a], X[a], hi[a]) + ext
            for code in range(8):
                pc = cell + np.array([code & 1, (code >> 1) & 1, code >> 2])
                p = pc[0] + nx * (pc[1] + ny * pc[2])
                O = org + pc * spc
                R2 = (np.maximum(np.abs(lo - O), np.abs(hi - O)) ** 2).sum()
                octs = [oo for oo in range(8)
                        if all((hi[a] > O[a]) if (oo >> a) & 1 else (lo[a] < O[a]) for a in range(3))]
                m = min(om[p, oo] for oo in octs)
                if not (m > 0 and m * m > R2 * 1.002001):
                    continue
                certified += 1
                ij, tio, _ = oracle.texel_sequence(N, X - O, w, ta, tb)
                rho = np.linalg.norm((X - O)[None, None, :] + tio[:, :, None] * w[None, None, :], axis=2)
                stored = D[p, ij[:, 1], ij[:, 0]]
                assert np.all(stored >= rho.max(1)), (r, cell, code)
                checked_texels += len(ij)
    assert certified > 300 and checked_texels > 3000, (certified, checked_texels)


def test_eye_cell_probes_behind_the_surface_answer_unknown_for_every_ray():
    # the eye-cell rule: every ray's first piece in the eye's cell starts at the eye, in the
    # eye's octant, so its first texel is the texel of X - O itself; when that texel's stored
    # distance is below |X - O| / (1 + tau), the first fire is behind the surface (UNKNOWN)
    scene, probes, views = workload("single", size=(64, 36))
    og = oracle.Grid.from_probes(probes)
    N, P = probes.N, probes.n_probes
    D = probes.distance.reshape(P, N, N).astype(np.float64)
    tau1 = 1.0 + 8.0 / N
    X = np.asarray(views[0].pos, np.float64)
    org, spc = np.array(probes.origin, float), np.array(probes.spacing, float)
    nx, ny, _ = probes.dims
    cell = np.clip(np.floor((X - org) / spc).astype(int), 0, np.array(probes.dims) - 2)
    o, d = oracle.view_rays(*views[0].as_tuple())
    rng = np.random.default_rng(1)
    rays = rng.choice(len(o), 300, replace=False)
    flagged = 0
    for code in range(8):
        pc = cell + np.array([code & 1, (code >> 1) & 1, code >> 2])
        p = pc[0] + nx * (pc[1] + ny * pc[2])
        xp = X - (org + pc * spc)
        u, v = oracle.oct_encode(xp)
        i, j = (min(int(np.floor((c + 1.0) * 0.5 * N)), N - 1) for c in (u, v))
        r = D[p, j, i]
        rho0 = np.linalg.norm(xp)
        if not (r < rho0 and rho0 > r * tau1):
            continue
        flagged += 1
        for k in rays:
            cells, iv = oracle.cell_walk(og, o[k], d[k])
            assert np.array_equal(cells[0], cell) and iv[0, 0] == 0.0
            ij, tio, _ = oracle.texel_sequence(N, xp, d[k], 0.0, iv[0, 1])
            assert tuple(ij[0]) == (i, j) and tio[0, 0] == 0.0, (p, k, ij[0], (i, j))
    assert flagged >= 2, flagged


def test_solid_probes_answer_unknown_for_every_ray():
    # the solid-probe rule: with every stored distance <= 0, each probe's first texel fires
    # behind the surface, so every ray is UNKNOWN unless the eye sits on a probe (its eye
    # lookup returns the stored 0, a HIT at t = 0)
    scene, probes, views = workload("tiny")
    P, N = probes.n_probes, probes.N
    d0 = np.zeros_like(probes.distance)
    d0[1] = -0.25
    og = oracle.Grid(probes.dims, probes.origin, probes.spacing, N, probes.levels, probes.scene_min,
                     probes.scene_max, d0, probes.normal, probes.radiance.view(np.float16).astype(np.float32))
    o, d = oracle.view_rays(*views[0].as_tuple())
    res = oracle.trace(og, o, d)
    assert np.all(res["status"] == oracle.UNKNOWN)
    # an eye on probe 0
    O = og.probe_position(0)
    res = oracle.trace(og, np.repeat(O[None], len(d), 0), d)
    assert np.all(res["status"] == oracle.HIT) and np.all(res["t"] == 0.0) and np.all(res["probe"] == 0)


def _texel_reach(N, spc, o):
    """[N][N] bound on the radial distance at which a direction of each texel of octant o
    leaves a cell of the spacing with the probe at its corner: min over the axes of
    spacing / |w_i|, |w_i| at its smallest over the texel's corners (the ratio |p_i| / |p| of
    the decoded direction is quasi-concave on a texel inside one octant triangle).  Texels
    across the fold take the cell's diagonal."""
    h = N // 2
    R = float(np.linalg.norm(spc))
    idx = np.arange(N)
    a = np.where(idx >= h, idx - h, h - 1 - idx)
    A, B = a[None, :] + 0 * a[:, None], a[:, None] + 0 * a[None, :]
    oz = o >> 2
    inside = (A + B + 2 <= h) if oz else (A + B >= h)
    m = np.full((N, N, 3), np.inf)
    for da in (0, 1):
        for db in (0, 1):
            au, bv = (A + da) * (2.0 / N), (B + db) * (2.0 / N)
            p = np.stack([au, bv, 1.0 - au - bv], -1) if oz else np.stack([1.0 - bv, 1.0 - au, au + bv - 1.0], -1)
            m = np.minimum(m, np.abs(p) / np.linalg.norm(p, axis=-1, keepdims=True))
    with np.errstate(divide="ignore"):
        r_in = np.min(np.asarray(spc, float)[None, None, :] / m, axis=-1)
    return np.where(inside, np.minimum(r_in, R), R)


def _directional_minima(D, spc):
    """[P][8] minima of D / reach over the texels a piece in each octant reaches (the octant
    triangle, the fold band and the neighbouring quadrants' edge texels, as octmin)."""
    P, N, _ = D.shape
    h = N // 2
    idx = np.arange(N)
    sx = idx >= h
    a = np.where(sx, idx - h, h - 1 - idx)
    A, B = a[None, :], a[:, None]
    SX, SY = sx[None, :], sx[:, None]
    Dn = np.where(np.isnan(D), np.inf, D)
    out = np.full((P, 8), np.inf)
    for o in range(8):
        ox, oy, oz = o & 1, (o >> 1) & 1, o >> 2
        reach = _texel_reach(N, spc, o)
        own = (SX == ox) & (SY == oy)
        edge = ((SX == ox) | (A == 0)) & ((SY == oy) | (B == 0))
        tri = (A + B <= h + 1) if oz else (A + B >= h - 3)
        mask = (own & tri) | (~own & edge)
        out[:, o] = np.where(mask[None], Dn / reach[None], np.inf).reshape(P, -1).min(1)
    return out


def test_texel_reach_bounds_every_direction_of_the_texel():
    # sampled directions of every texel (quadrant x >= 0, y >= 0; both z halves) leave the
    # cell [0, s] no farther than the texel's reach
    N, spc = 16, np.array([1.0, 1.3, 0.8])
    rng = np.random.default_rng(4)
    for o in (3, 7):
        reach = _texel_reach(N, spc, o)
        for j in range(N // 2, N):
            for i in range(N // 2, N):
                uv = (np.array([i, j])[None, :] + rng.uniform(0, 1, size=(64, 2))) * (2.0 / N) - 1.0
                for u, v in uv:
                    z = 1 - abs(u) - abs(v)
                    if (z >= 0) != bool(o >> 2):
                        continue
                    w = np.abs(oracle.oct_decode(np.array([u, v])))
                    w /= np.linalg.norm(w)
                    exit_t = min(spc[k] / w[k] for k in range(3) if w[k] > 0)
                    assert exit_t <= reach[j, i] * (1 + 1e-12), (o, i, j, u, v, exit_t, reach[j, i])


def test_directional_clear_probes_never_fire_on_interior_cells():
    # the directional form of the clear rule on cells away from the grid's boundary (their
    # region is the cell itself, one octant of each corner probe)
    scene, probes, views = workload("diff", N=32, levels=3, n_views=1, size=(40, 32))
    og = oracle.Grid.from_probes(probes)
    N, P = probes.N, probes.n_probes
    D = probes.distance.reshape(P, N, N).astype(np.float64)
    spc = np.array(probes.spacing, float)
    dm = _directional_minima(D, spc)
    om = _octant_minima(D)
    nx, ny, nz = probes.dims
    cmax = np.array(probes.dims) - 2
    org = np.array(probes.origin, float)
    o, d = oracle.view_rays(*views[0].as_tuple())
    rng = np.random.default_rng(2)
    certified = extra = 0
    for r in rng.choice(len(o), 400, replace=False):
        X, w = o[r], d[r]
        cells, iv = oracle.cell_walk(og, X, w)
        for cell, (ta, tb) in zip(cells, iv):
            if not np.all((cell > 0) & (cell < cmax)):
                continue
            for code in range(8):
                pc = cell + np.array([code & 1, (code >> 1) & 1, code >> 2])
                p = pc[0] + nx * (pc[1] + ny * pc[2])
                oct_ = (1 - (code & 1)) + 2 * (1 - ((code >> 1) & 1)) + 4 * (1 - (code >> 2))
                if not dm[p, oct_] > 1.001:
                    continue
                certified += 1
                extra += not (om[p, oct_] > 1.001 * np.linalg.norm(spc))
                O = org + pc * spc
                ij, tio, _ = oracle.texel_sequence(N, X - O, w, ta, tb)
                rho = np.linalg.norm((X - O)[None, None, :] + tio[:, :, None] * w[None, None, :], axis=2)
                assert np.all(D[p, ij[:, 1], ij[:, 0]] >= rho.max(1)), (r, cell, code)
    assert certified > 300 and extra > 20, (certified, extra)

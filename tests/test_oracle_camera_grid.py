"""Pins of the oracle's camera rays, grid iterator and cage order against geometry the
tests compute themselves (no formula of the oracle is retyped here).

* Camera rays (Overview: one ray (X, w) per pixel; pinhole conventions are ours: vertical
  field of view, pixel centres, row 0 at the top): the centre pixel of an odd-sized view
  looks along fwd; the centre rays of the top and bottom rows are 2 atan((1 - 1/H) tan)
  apart, those of the first and last columns 2 atan((1 - 1/W) (W/H) tan); the rays of
  mirrored pixels are mirror images across the plane of fwd and up (or fwd and right).
* Grid iterator (Ray Trace Using Multiple Probes > Grid Iterator): the intervals tile
  [0, t_far] in order; each interval lies in its one cell (every dense sample of the ray
  maps to the reported cell of the interval holding it); consecutive cells are neighbours
  across the planes crossed; the walk crosses each interior plane at most once.
* Cage order (Ray Trace Using Multiple Probes > Less Than 8 Probes: closest to the eye
  first): the probes of a cell's cage sit at the 8 corners of that cell, sorted by distance
  to the eye, ties by corner code dx + 2 dy + 4 dz.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import workload


def _random_basis(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 2] = -q[:, 2]
    return q[:, 0], q[:, 1], q[:, 2]  # right, up, fwd (orthonormal, right-handed)


def _angle(a, b):
    c = np.clip(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)), -1.0, 1.0)
    return math.acos(c)


@pytest.mark.parametrize("W,H,fov_deg,seed", [(101, 75, 60.0, 0), (33, 331, 20.0, 1), (7, 5, 90.0, 2),
                                             (101, 75, 60.0, -1), (9, 1, 45.0, -2)])
def test_camera_rays_from_geometry(W, H, fov_deg, seed):
    if seed >= 0:
        # a random basis rounded to FP32 (the view's precision) is orthonormal to ~1e-7
        rng = np.random.default_rng(seed)
        right, up, fwd = (np.float32(v).astype(np.float64) for v in _random_basis(rng))
        tol = 5e-7
    else:
        # a signed permutation of the axes: exactly orthonormal in FP32
        right, up, fwd = (np.array(v, float) for v in
                          (([0, 0, -1], [1, 0, 0], [0, -1, 0]) if seed == -1 else ([0, 1, 0], [0, 0, 1], [1, 0, 0])))
        tol = 1e-12
    pos = np.array([1.25, -0.5, 3.0])
    th = float(np.float32(math.tan(math.radians(fov_deg) / 2)))
    o, d = oracle.view_rays(pos, right, up, fwd, th, W, H)
    assert o.shape == (W * H, 3) and np.all(o == pos)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    at = lambda x, y: d[y * W + x]
    cx, cy = W // 2, H // 2
    fwd_u = fwd / np.linalg.norm(fwd)
    # odd sizes: the centre pixel looks straight ahead
    assert np.allclose(at(cx, cy), fwd_u, atol=tol)
    # top and bottom row centres span the vertical field of view less one pixel
    vspan = 2 * math.atan((1 - 1 / H) * th)
    assert abs(_angle(at(cx, 0), at(cx, H - 1)) - vspan) < tol
    hspan = 2 * math.atan((1 - 1 / W) * (W / H) * th)
    assert abs(_angle(at(0, cy), at(W - 1, cy)) - hspan) < tol
    # row 0 is the top of the image, column 0 its left edge
    if H > 1:
        assert np.dot(at(cx, 0), up) > 0 > np.dot(at(cx, H - 1), up)
    assert np.dot(at(0, cy), right) < 0 < np.dot(at(W - 1, cy), right)
    # mirror symmetry across the fwd-up plane (x <-> W-1-x) and the fwd-right plane
    for x, y in [(0, 0), (3 % W, 1 % H), (W - 2, H - 1), (cx, 2 % H)]:
        a, b = at(x, y), at(W - 1 - x, y)
        assert abs(np.dot(a, right) + np.dot(b, right)) < tol
        assert abs(np.dot(a, up) - np.dot(b, up)) < tol and abs(np.dot(a, fwd) - np.dot(b, fwd)) < tol
        a, b = at(x, y), at(x, H - 1 - y)
        assert abs(np.dot(a, up) + np.dot(b, up)) < tol
        assert abs(np.dot(a, right) - np.dot(b, right)) < tol
    # square pixels: neighbouring columns and neighbouring rows at the centre subtend the
    # same angle (to first order in the pixel size)
    if H > 1:
        dx = _angle(at(cx, cy), at(cx + 1, cy))
        dy = _angle(at(cx, cy), at(cx, cy + 1))
        assert abs(dx - dy) < 1e-9 + tol
    # a pixel subset is the same rays
    pix = np.array([0, W * H - 1, cy * W + cx, 5 % (W * H)])
    o2, d2 = oracle.view_rays(pos, right, up, fwd, th, W, H, pixels=pix)
    assert np.array_equal(d2, d[pix]) and np.array_equal(o2, o[pix])


def _cell_of(point, origin, spacing, dims):
    q = np.floor((point - origin) / spacing).astype(np.int64)
    return np.clip(q, 0, np.asarray(dims) - 2)


def _tfar(X, w, smin, smax):
    """Exit of the ray from the box [smin, smax] (slab method), enlarged by 1e-4 as the
    trace's range is."""
    t = math.inf
    for a in range(3):
        if w[a] > 0:
            t = min(t, (smax[a] - X[a]) / w[a])
        elif w[a] < 0:
            t = min(t, (smin[a] - X[a]) / w[a])
    return t * (1 + 1e-4)


def _rays_for(probes, scene, rng, n):
    """Ray origins inside the room (some outside the probe hull), directions random,
    axis-aligned and plane-diagonal."""
    room = np.asarray(scene.room_max, dtype=np.float64)
    dirs = [np.array(v, float) for v in
            ([1, 0, 0], [0, -1, 0], [0, 0, 1], [1, 1, 0], [-1, 0, 1], [0, 1, -1], [1, -1, 1])]
    out = []
    for i in range(n):
        X = rng.uniform(0.02 * room, 0.98 * room)
        w = dirs[i % len(dirs)] if i % 3 == 0 else rng.normal(size=3)
        out.append((X, w / np.linalg.norm(w)))
    # rays whose crossings of two or three planes tie exactly (equal offsets from the
    # planes, equal direction components): the walk steps diagonally through the edge
    for k in range(12):
        f = rng.uniform(0.05, 0.95)
        base = np.asarray(probes.origin, dtype=np.float64) + f * np.asarray(probes.spacing, dtype=np.float64)
        X = base.copy()
        w = np.array([1.0, 1.0, rng.uniform(-0.7, 0.7)]) if k % 2 else np.array([1.0, 1.0, 1.0])
        if k % 3 == 2:
            w = -w
            X = X + np.asarray(probes.spacing) * np.minimum(np.asarray(probes.dims) - 2, 1)
        out.append((X, w / np.linalg.norm(w)))
    # a ray starting exactly on a probe plane
    X = rng.uniform(0.1 * room, 0.9 * room)
    X[0] = probes.origin[0] + probes.spacing[0] * min(2, probes.dims[0] - 1)
    out.append((X, np.array([0.3, 0.8, -0.52]) / np.linalg.norm([0.3, 0.8, -0.52])))
    return out


@pytest.mark.parametrize("name,kw", [("single", dict(size=(16, 16))), ("tiny", {})])
def test_grid_iterator_tiles_the_ray_cell_by_cell(name, kw):
    scene, probes, _ = workload(name, **kw)
    g = oracle.Grid.from_probes(probes)
    dims = np.asarray(probes.dims)
    origin = np.asarray(probes.origin, dtype=np.float64)
    spacing = np.asarray(probes.spacing, dtype=np.float64)
    rng = np.random.default_rng(7)
    max_cells = 1 + int(np.sum(dims - 2))
    for X, w in _rays_for(probes, scene, rng, 150):
        cells, tab = oracle.cell_walk(g, X, w)
        tfar = _tfar(X, w, probes.scene_min, probes.scene_max)
        assert len(cells) >= 1
        # the intervals tile [0, t_far] in order
        assert tab[0, 0] == 0.0
        assert abs(tab[-1, 1] - tfar) <= 1e-12 * tfar
        assert np.all(tab[1:, 0] == tab[:-1, 1])
        assert np.all(tab[:, 1] >= tab[:, 0])
        # only a ray starting on a plane and leaving it backwards has an empty interval, the
        # first; a tie of planes is crossed in one step, not through an empty cell
        assert np.all(tab[1:, 1] > tab[1:, 0])
        # each interior plane is crossed at most once
        assert len(cells) <= max_cells
        # consecutive cells are neighbours across the planes crossed (a tie crosses several)
        step = np.diff(cells, axis=0)
        assert np.all(np.abs(step) <= 1) and np.all(np.abs(step).sum(axis=1) >= 1)
        assert np.all((step == 0) | (np.sign(step) == np.sign(w)[None, :]))
        # every dense sample of the ray lies in the cell of the interval holding it
        ts = np.linspace(0.0, tfar, 2001)[1:-1]
        k = np.searchsorted(tab[:, 1], ts, side="left")
        inner = np.abs(ts - tab[np.minimum(k, len(tab) - 1), 1]) > 1e-9 * tfar
        inner &= np.abs(ts - tab[np.minimum(k, len(tab) - 1), 0]) > 1e-9 * tfar
        pts = X[None, :] + ts[:, None] * w[None, :]
        got = np.array([_cell_of(p, origin, spacing, dims) for p in pts])
        assert np.array_equal(got[inner], cells[k[inner]])


def test_grid_iterator_cells_visited_in_order_by_brute_force():
    """Dense sampling of 40 rays of the 1080p room: the distinct cells met along each ray,
    in order, are exactly the walk's cells (those with an interval longer than the
    sampling step)."""
    scene, probes, _ = workload("single", size=(16, 16))
    g = oracle.Grid.from_probes(probes)
    dims = np.asarray(probes.dims)
    origin = np.asarray(probes.origin, dtype=np.float64)
    spacing = np.asarray(probes.spacing, dtype=np.float64)
    rng = np.random.default_rng(11)
    for X, w in _rays_for(probes, scene, rng, 40):
        cells, tab = oracle.cell_walk(g, X, w)
        tfar = tab[-1, 1]
        ts = np.linspace(0.0, tfar, 20001)[:-1]
        pts = X[None, :] + ts[:, None] * w[None, :]
        seq = [tuple(_cell_of(p, origin, spacing, dims)) for p in pts]
        met = [c for i, c in enumerate(seq) if i == 0 or c != seq[i - 1]]
        step = tfar / 20000
        long_enough = [tuple(c) for c, (a, b) in zip(cells, tab) if b - a > 2 * step]
        assert [c for c in met if c in set(long_enough)] == long_enough


def test_cage_order_is_the_cell_corners_closest_first():
    scene, probes, _ = workload("single", size=(16, 16))
    g = oracle.Grid.from_probes(probes)
    pos = synth.grid_positions(probes.dims, float(probes.origin[0]), float(probes.spacing[0]))
    dims = np.asarray(probes.dims)
    origin = np.asarray(probes.origin, dtype=np.float64)
    spacing = np.asarray(probes.spacing, dtype=np.float64)
    rng = np.random.default_rng(3)
    room = np.asarray(scene.room_max, dtype=np.float64)
    for _ in range(300):
        X = rng.uniform(0.0, room)
        cell = _cell_of(X, origin, spacing, dims)
        order = oracle.cage_order(g, cell, X)
        assert len(order) == 8
        corners = {tuple(origin + (cell + np.array(c)) * spacing) for c in itertools.product((0, 1), repeat=3)}
        got = [tuple(pos[p]) for p in order]
        assert set(got) == corners and len(set(order)) == 8
        dist = np.linalg.norm(pos[order] - X, axis=1)
        assert np.all(np.diff(dist) >= 0)
    # at the centre of a cell all 8 corners are equidistant: corner-code order (x fastest)
    cell = np.array([2, 3, 1])
    X = origin + (cell + 0.5) * spacing
    order = oracle.cage_order(g, cell, X)
    want = [tuple(origin + (cell + np.array([c & 1, (c >> 1) & 1, c >> 2])) * spacing) for c in range(8)]
    assert [tuple(pos[p]) for p in order] == want
    # on the cell's x = const mid-plane, pairs tie: the lower code first within each pair
    X = origin + (cell + np.array([0.5, 0.2, 0.1])) * spacing
    order = oracle.cage_order(g, cell, X)
    first = origin + cell * spacing
    assert tuple(pos[order[0]]) == tuple(first) and tuple(pos[order[1]]) == tuple(first + [spacing[0], 0, 0])


def test_cage_order_of_a_small_layout_is_every_probe_closest_first():
    scene, probes, _ = workload("paper", size=(16, 16))
    g = oracle.Grid.from_probes(probes)
    pos = synth.grid_positions(probes.dims, float(probes.origin[0]), float(probes.spacing[0]))
    rng = np.random.default_rng(5)
    for _ in range(50):
        X = rng.uniform(0.0, np.asarray(scene.room_max, dtype=np.float64))
        order = oracle.cage_order(g, [0, 0, 0], X)
        assert sorted(order) == list(range(len(pos)))
        dist = np.linalg.norm(pos[order] - X, axis=1)
        assert np.all(np.diff(dist) >= 0)

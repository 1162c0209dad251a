"""Scenes of fewer than 8 probes (Methodology, Ray Trace Using Multiple Probes: with more
than one but fewer than 8 probes there is no grid iterator; a ray tries the probe closest
to the eye first and falls through to the next closest on MISS or UNKNOWN until every
probe was used).  A single probe is the one-probe trace of the same section.

Pins: the analytic scene (every HIT lies on the true surface within the bound of the
probe representation), the nearest-probe rule checked against positions computed here,
and the mirror symmetry x <-> y of the whole method on mirrored probe data.
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_scene import _check

LAYOUTS = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (2, 2, 1), (3, 1, 1), (3, 2, 1), (1, 1, 2)]

_CACHE = {}


def few_room(dims, N=128, levels=5, size=(120, 80), seed=21):
    """A seeded room sized by `dims` probes (spacing 1) with a few objects, and one view."""
    key = (dims, N, levels, size, seed)
    if key not in _CACHE:
        scene = synth.make_scene(seed, dims, 1.0, (2, 4))
        probes = synth.bake(scene, N, levels)
        views = synth.make_views(scene, seed + 1, 1, *size)
        _CACHE[key] = (scene, probes, views)
    return _CACHE[key]


@pytest.mark.parametrize("dims", LAYOUTS)
def test_few_probe_rooms_against_analytic_scene(dims):
    scene, probes, views = few_room(dims)
    s = _check(scene, probes, views[0])
    assert s["hit"] > 0.3 * s["n"], {k: v for k, v in s.items() if k != "r"}
    assert s["fails"] == 0, {k: v for k, v in s.items() if k != "r"}
    r = s["r"]
    hit = r["status"] == oracle.HIT
    # every probe index reported exists
    assert np.all((r["probe"][hit] >= 0) & (r["probe"][hit] < probes.n_probes))


@pytest.mark.parametrize("dims", [(2, 1, 1), (2, 2, 1), (3, 2, 1), (1, 1, 2)])
def test_one_probe_per_ray_is_the_nearest(dims):
    # with one probe tried per ray, every HIT comes from the probe nearest to the eye
    scene, probes, views = few_room(dims)
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    r = oracle.trace(g, o, d, max_probes_per_cell=1)
    pos = np.stack([g.probe_position(p) for p in range(probes.n_probes)])
    nearest = int(np.argmin(np.linalg.norm(pos - o[0], axis=1)))
    hit = r["status"] == oracle.HIT
    assert hit.any()
    assert np.all(r["probe"][hit] == nearest)
    # and every probe tried resolves at least as many rays
    full = oracle.trace(g, o, d)
    assert np.all(full["status"][hit] == oracle.HIT)
    assert (full["status"] == oracle.HIT).sum() >= hit.sum()


def _mirror_xy(probes):
    """Probe data of the same room mirrored through the plane x = y (axes x and y swapped):
    probe (i, j, k) becomes (j, i, k), texel (i, j) becomes (j, i), an octahedral normal
    (u, v) becomes (v, u)."""
    a, b, c = probes.dims
    N = probes.N
    P = a * b * c
    dist = probes.distance.reshape(P, N, N)
    nrm = probes.normal.reshape(P, N, N, 2)
    rad = probes.radiance.reshape(P, N, N, 3)
    mdist = np.empty_like(dist)
    mnrm = np.empty_like(nrm)
    mrad = np.empty_like(rad)
    pmap = np.empty(P, np.int64)
    for p in range(P):
        i, j, k = p % a, (p // a) % b, p // (a * b)
        q = j + b * (i + a * k)
        pmap[p] = q
        mdist[q] = dist[p].T
        mnrm[q] = nrm[p].transpose(1, 0, 2)[..., ::-1]
        mrad[q] = rad[p].transpose(1, 0, 2)
    sw = lambda v: np.asarray(v)[[1, 0, 2]]
    g = oracle.Grid((b, a, c), sw(probes.origin), sw(probes.spacing), N, probes.levels, sw(probes.scene_min),
                    sw(probes.scene_max), mdist, np.ascontiguousarray(mnrm), np.ascontiguousarray(mrad))
    return g, pmap


@pytest.mark.parametrize("dims", [(2, 1, 1), (3, 2, 1), (3, 1, 1)])
def test_mirror_symmetry(dims):
    scene, probes, views = few_room(dims)
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    r = oracle.trace(g, o, d)
    mg, pmap = _mirror_xy(probes)
    mr = oracle.trace(mg, o[:, [1, 0, 2]], d[:, [1, 0, 2]])
    N = probes.N
    margin = (r["margin"] != 0) | (mr["margin"] != 0)
    assert margin.mean() < 0.1
    keep = ~margin
    assert np.array_equal(r["status"][keep], mr["status"][keep])
    hit = keep & (r["status"] == oracle.HIT)
    assert hit.sum() > 0.3 * len(hit)
    assert np.array_equal(pmap[r["probe"][hit]], mr["probe"][hit])
    tx, ty = r["texel"][hit] % N, r["texel"][hit] // N
    assert np.array_equal(tx * N + ty, mr["texel"][hit])
    assert np.allclose(r["t"][hit], mr["t"][hit], rtol=1e-9, atol=0)
    assert np.allclose(r["rgb"][hit], mr["rgb"][hit], rtol=0, atol=1e-6)


def test_planar_grid_of_eight_or_more_is_rejected():
    scene, probes, views = few_room((2, 1, 1))
    N = probes.N
    with pytest.raises(ValueError):
        oracle.Grid((8, 1, 1), probes.origin, probes.spacing, N, probes.levels, probes.scene_min, probes.scene_max,
                    np.zeros((8, N, N), np.float32), np.zeros((8, N, N, 2), np.uint16),
                    np.zeros((8, N, N, 3), np.float32))

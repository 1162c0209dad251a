"""Two-level probe hierarchy on the oracle (our reading of the paper's hierarchical scene
representation: in each fine cell's interval the fine cage first, then the cage of the
coarse cell holding that fine cell), on a seeded city block of boxes."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from conftest import workload
from test_oracle_scene import _discontinuity_mask, _texel_diameter


def _city():
    return workload("large_small")


def _trace2(tl, o, d, fine=None, coarse=None, **kw):
    og = oracle.Grid.from_probes(fine or tl.fine)
    cg = oracle.Grid.from_probes(coarse or tl.coarse)
    return oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio), **kw), og, cg


def _dead(ps):
    return dataclasses.replace(ps, distance=np.zeros_like(ps.distance))


def test_city_bake_dead_probes_inside_buildings():
    scene, tl, views = _city()
    for ps in (tl.fine, tl.coarse):
        pos = synth.grid_positions(ps.dims, ps.origin[0], ps.spacing[0])
        p = scene.obj_param
        inside = np.array([np.any(np.all(np.abs(x - p[:, :3]) < p[:, 3:], axis=1)) for x in pos])
        dist = ps.distance.reshape(ps.n_probes, -1)
        assert np.all(dist[inside] == 0)
        assert np.all(dist[~inside] > 0)
        assert 0 < inside.mean() < 1


def test_two_level_city_against_analytic_scene():
    # the brute-force bound of the single-level check (test_oracle_scene), on the city at
    # 64^2 maps, with HITs of either level; the same exclusions: grazing rays, texels near a
    # depth jump in the hit probe's map, and camera rays near a silhouette
    scene, tl, views = workload("large_small", N=64, levels=4)
    v = views[0]
    o, d = oracle.view_rays(*v.as_tuple())
    r, og, cg = _trace2(tl, o, d)
    t_true, n_true, alb, ids = synth.cast(scene, o, d)
    assert np.all(np.isfinite(t_true))
    N = tl.fine.N
    tau = 8.0 / N
    theta = _texel_diameter(N, np.arange(N * N))
    dist = np.concatenate([tl.fine.distance, tl.coarse.distance])
    sid = np.concatenate([tl.fine.extra["surface_id"], tl.coarse.extra["surface_id"]])
    pos = np.concatenate([synth.grid_positions(ps.dims, ps.origin[0], ps.spacing[0]) for ps in (tl.fine, tl.coarse)])
    disc = _discontinuity_mask(sid, dist, tau)
    hit = r["status"] == oracle.HIT
    assert hit.mean() > 0.9
    coarse_hit = hit & (r["probe"] >= tl.fine.n_probes)
    assert coarse_hit.sum() > 50  # the coarse level resolves rays the fine cages leave open
    cosw = np.abs(np.sum(n_true * d, 1))
    p = np.where(hit, r["probe"], 0)
    k = np.where(hit, r["texel"], 0)
    rk = dist[p].reshape(len(p), -1)[np.arange(len(p)), k].astype(np.float64)
    excluded = hit & ((cosw < 0.1) | disc[p, k])
    cand = np.nonzero(hit & ~excluded)[0]
    P = o[cand] + t_true[cand, None] * d[cand]
    F = 2.0 * theta[k[cand]] * np.maximum(np.linalg.norm(P - pos[p[cand]], axis=1), rk[cand])
    dd = d[cand]
    a = np.where(np.abs(dd[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(dd, a)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(dd, e1)
    near_edge = np.zeros(len(cand), bool)
    for e in (e1, -e1, e2, -e2):
        t2, _, _, ids2 = synth.cast(scene, o[cand], P + F[:, None] * e - o[cand])
        near_edge |= (ids2 != ids[cand]) & (np.abs(t2 - t_true[cand]) > 4.0 * F / np.maximum(cosw[cand], 0.1))
    excluded[cand[near_edge]] = True
    # unobservable surfaces: the true hit point is seen (same surface id within one texel)
    # by none of the 16 cage probes of the fine cell holding it, so no probe represents it
    # and the ray goes on to a surface behind (probes inside buildings make this happen)
    cand = np.nonzero(hit & ~excluded)[0]
    seen = _observed(tl, o[cand] + t_true[cand, None] * d[cand], ids[cand], sid)
    excluded[cand[~seen]] = True
    assert (~seen).mean() < 0.01
    checked = hit & ~excluded
    bound = 1.5 * rk * (theta[k] + tau) / np.maximum(cosw, 1e-12)
    # a HIT in front of the true surface would be a surface that is not there: none allowed.
    # A HIT behind it means every probe that sees the true surface answered UNKNOWN there
    # (shadow-entry or normal test at the first firing texel) and the ray went on: the
    # method's own leak, which must stay rare.
    early = checked & (r["t"] < t_true - bound)
    late = checked & (r["t"] > t_true + bound)
    assert checked.mean() > 0.5
    assert (checked & coarse_hit).sum() > 100
    assert early.sum() == 0, np.nonzero(early)[0][:10]
    assert late.sum() <= 1e-3 * checked.sum(), (np.nonzero(late)[0][:10], late.sum(), checked.sum())


def _oct_texel(v, N):
    """texel (i, j) of directions v [n,3] (z-folded octahedron), for the observability test"""
    p = v / np.abs(v).sum(1, keepdims=True)
    u, w = p[:, 0].copy(), p[:, 1].copy()
    lo = p[:, 2] < 0
    u[lo] = (1 - np.abs(p[lo, 1])) * np.where(p[lo, 0] >= 0, 1, -1)
    w[lo] = (1 - np.abs(p[lo, 0])) * np.where(p[lo, 1] >= 0, 1, -1)
    return (np.clip(np.floor((u + 1) * N / 2), 0, N - 1).astype(int),
            np.clip(np.floor((w + 1) * N / 2), 0, N - 1).astype(int))


def _observed(tl, pts, true_ids, sid):
    f, c = tl.fine, tl.coarse
    N = f.N
    seen = np.zeros(len(pts), bool)
    fd, cd = np.array(f.dims), np.array(c.dims)
    fcell = np.clip(np.floor((pts - f.origin[0]) / f.spacing[0]), 0, fd - 2).astype(int)
    ccell = np.clip((fcell - np.array(tl.plane_off)) // np.array(tl.ratio), 0, cd - 2)
    S = sid.reshape(sid.shape[0], N, N)
    for base, cell, dims, ps, off in ((0, fcell, fd, f, 0), (0, ccell, cd, c, f.n_probes)):
        for corner in range(8):
            ijk = cell + np.array([corner & 1, (corner >> 1) & 1, corner >> 2])
            p = ijk[:, 0] + dims[0] * (ijk[:, 1] + dims[1] * ijk[:, 2])
            O = ps.origin[0] + ps.spacing[0] * ijk
            ti, tj = _oct_texel(pts - O, N)
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    seen |= S[off + p, np.clip(tj + dj, 0, N - 1), np.clip(ti + di, 0, N - 1)] == true_ids
    return seen


def test_coarse_hits_come_from_the_coarse_cell_of_the_hit_point():
    # with every fine probe dead (D = 0: UNKNOWN everywhere) only coarse probes can HIT, and
    # a HIT in a fine cell's interval comes from a corner of the coarse cell holding it
    scene, tl, views = _city()
    o, d = oracle.view_rays(*views[1].as_tuple())
    r, og, cg = _trace2(tl, o, d, fine=_dead(tl.fine))
    hit = r["status"] == oracle.HIT
    assert hit.mean() > 0.5
    assert np.all(r["probe"][hit] >= tl.fine.n_probes)
    c = tl.coarse
    pts = o[hit] + r["t"][hit, None] * d[hit]
    cdims = np.array(c.dims)
    cell = np.clip(np.floor((pts - c.origin[0]) / c.spacing[0]), 0, cdims - 2).astype(int)
    pc = r["probe"][hit] - tl.fine.n_probes
    pijk = np.stack([pc % cdims[0], (pc // cdims[0]) % cdims[1], pc // (cdims[0] * cdims[1])], 1)
    corner = pijk - cell
    # points on a coarse plane may sit in either neighbouring cell
    onplane = np.abs((pts - c.origin[0]) / c.spacing[0] - np.round((pts - c.origin[0]) / c.spacing[0])) < 1e-6
    ok = np.all(((corner == 0) | (corner == 1)) | onplane, axis=1)
    assert ok.all(), np.nonzero(~ok)[0][:10]


def test_dead_coarse_level_keeps_every_fine_hit():
    scene, tl, views = _city()
    o, d = oracle.view_rays(*views[0].as_tuple())
    one = oracle.trace(oracle.Grid.from_probes(tl.fine), o, d)
    two, og, cg = _trace2(tl, o, d, coarse=_dead(tl.coarse))
    h = one["status"] == oracle.HIT
    assert np.array_equal(two["status"][h], one["status"][h])
    for k in ("probe", "texel", "t"):
        assert np.array_equal(two[k][h], one[k][h]), k
    # a ray the fine grid alone leaves MISS meets the dead coarse probes: UNKNOWN
    m = one["status"] == oracle.MISS
    assert np.all(two["status"][m] == oracle.UNKNOWN)


def test_two_level_vjp_spans_both_levels():
    scene, tl, views = _city()
    o, d = oracle.view_rays(*views[0].as_tuple())
    r, og, cg = _trace2(tl, o, d)
    g = np.random.default_rng(2).normal(size=(len(o), 3))
    got = oracle.vjp((og, cg), r, g)
    assert got.shape[0] == tl.n_probes
    # dot-product identity over the concatenated radiance of both levels
    x = np.random.default_rng(3).normal(size=got.shape)
    rad = x.astype(np.float32)
    og.set_radiance(rad[:tl.fine.n_probes])
    cg.set_radiance(rad[tl.fine.n_probes:])
    rx = oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio))
    lhs = np.sum(rx["rgb"] * g)
    rhs = np.sum(rad.astype(np.float64) * got)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))

"""Probes the per-view cage tables leave out of the hard walk, because their answer is known
for every ray of the view that reaches them (PT_FLAG_TRACE_ALL_PROBES traces them):
UNKNOWN for probes inside solids (every stored distance <= 0) and, in the eye's cell, for
probes whose first texel fires behind the stored surface for the eye itself; MISS for
probes whose nearest stored surface in every octant a piece of the cell can take lies
beyond the cell's farthest point.  Checked here: the same outputs bit for bit either way
on the city block, where most probes of both levels sit inside buildings, in every launch
form and in the adjoints; on the room, the 64-view walk and the paper's 2048^2 maps, where
the eye's cell gives such probes; on the sparse differentiable grid, where many probes are
clear of their cells, also after probe_grid_set_distance moves the surfaces, and for an
eye outside the scene box or on probe planes; a probe the eye sits on is still traced (its
eye lookup is a HIT at t = 0); the flags follow
probe_grid_set_distance (zeroed, negative and NaN maps); and a layout of fewer than 8
probes.  Each default result is also held to the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from conftest import workload
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _np(res):
    return {k: v.cpu().numpy() for k, v in res.items() if v is not None}


def _same(a, b, label):
    for k in ("status", "hit", "t", "rgb"):
        assert np.array_equal(a[k], b[k]), (label, k)


def _solid(ps):
    d = ps.distance.reshape(ps.n_probes, -1)
    return (d <= 0).all(1)


_CACHE = {}


def _city():
    if "city" not in _CACHE:
        pt = _pt()
        scene, tl, views = workload("large_small")
        grid = pt.ProbeGrid.from_two_level(tl)
        rad = torch.from_numpy(tl.radiance().view(np.float16).copy()).cuda()
        og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
        _CACHE["city"] = (scene, tl, views, grid, rad, og, cg)
    return _CACHE["city"]


def _oracle_views(tl, og, cg, views):
    o = np.concatenate([oracle.view_rays(*v.as_tuple())[0] for v in views])
    d = np.concatenate([oracle.view_rays(*v.as_tuple())[1] for v in views])
    return oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio))


def test_city_skip_gives_identical_results_in_every_launch_form():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    assert _solid(tl.fine).mean() > 0.5 and _solid(tl.coarse).mean() > 0.5
    ref = _np(pt.probe_trace(grid, rad, views))
    assert_parity(compare(ref, _oracle_views(tl, og, cg, views)), "city, solid probes left out")
    for flags in (0, pt.PT_FLAG_PERSISTENT, pt.PT_FLAG_GRAPH, pt.PT_FLAG_WIDE):
        for extra in (0, pt.PT_FLAG_TRACE_ALL_PROBES):
            got = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags | extra)))
            _same(got, ref, (flags, extra))
    rays = sum(v.width * v.height for v in views)
    for extra in (0, pt.PT_FLAG_TRACE_ALL_PROBES):
        out = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"),
               torch.empty(rays, dtype=torch.uint8, device="cuda"), torch.empty((rays, 2), dtype=torch.int32,
                                                                                  device="cuda"))
        pt.probe_trace_noalloc(grid, rad, views, out, pt.trace_opts(flags=extra))
        torch.cuda.synchronize()
        got = dict(rgb=out[0].cpu().numpy(), t=out[1].cpu().numpy(), status=out[2].cpu().numpy(),
                   hit=out[3].cpu().numpy())
        _same(got, ref, ("noalloc", extra))


def test_city_adjoints_with_and_without_the_skip():
    # the recomputing adjoints walk the same cage tables: the same HITs, so the same sums up
    # to the order of their FP32 atomics
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    rays = sum(v.width * v.height for v in views)
    g = torch.from_numpy(np.random.default_rng(3).normal(size=(rays, 3)).astype(np.float32)).cuda()
    gt = torch.from_numpy(np.random.default_rng(4).normal(size=rays).astype(np.float32)).cuda()
    P, N = tl.n_probes, tl.fine.N
    out = {}
    for extra in (0, pt.PT_FLAG_TRACE_ALL_PROBES):
        for pers in (0, pt.PT_FLAG_PERSISTENT):
            opts = pt.trace_opts(flags=extra | pers)
            gr = torch.zeros((P, N, N, 3), device="cuda")
            pt.probe_trace_backward(grid, views, g, gr, opts)
            gd = torch.zeros((P, N, N), device="cuda")
            pt.probe_trace_backward_distance(grid, rad, views, g, gt, gd, opts)
            out[(extra, pers)] = (gr.cpu().numpy(), gd.cpu().numpy())
    ref_r, ref_d = out[(0, 0)]
    assert np.count_nonzero(ref_r) > 1000 and np.count_nonzero(ref_d) > 500
    for key, (gr, gd) in out.items():
        for a, b, what in ((gr, ref_r, "radiance"), (gd, ref_d, "distance")):
            err = np.abs(a.astype(np.float64) - b)
            assert (err <= 1e-5 * np.abs(b) + 1e-6).all(), (key, what, err.max())
            assert np.array_equal(a != 0, b != 0), (key, what)


def test_eye_on_a_solid_probe_keeps_its_eye_lookup():
    # a view whose eye sits exactly on a fine probe inside a building: that probe is the
    # first of its cell's cage and its eye lookup returns the stored 0, a HIT at t = 0
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    fine = tl.fine
    solid = np.nonzero(_solid(fine))[0]
    nx, ny, nz = fine.dims
    ijk = np.stack([solid % nx, (solid // nx) % ny, solid // (nx * ny)], 1)
    inner = solid[((ijk > 0) & (ijk < np.array(fine.dims) - 1)).all(1)]
    p = int(inner[len(inner) // 2])
    pos = og.probe_position(p).astype(np.float32).astype(np.float64)
    v = dataclasses.replace(views[0], pos=pos, width=64, height=48)
    a = _np(pt.probe_trace(grid, rad, [v]))
    b = _np(pt.probe_trace(grid, rad, [v], pt.trace_opts(flags=pt.PT_FLAG_TRACE_ALL_PROBES)))
    _same(a, b, "eye on a solid probe")
    assert np.all(a["status"] == oracle.HIT) and np.all(a["t"] == 0.0) and np.all(a["hit"][:, 0] == p)
    assert_parity(compare(a, _oracle_views(tl, og, cg, [v])), "eye on a solid probe")


def test_flags_follow_set_distance():
    pt = _pt()
    scene, probes, views = workload("single", size=(320, 180))
    grid = pt.ProbeGrid.from_probes(probes)
    rad16 = probes.radiance.view(np.float16)
    rad = torch.from_numpy(rad16.copy()).cuda()
    P, N = probes.n_probes, probes.N
    rng = np.random.default_rng(17)
    pick = rng.choice(P, 48, replace=False)
    d2 = probes.distance.copy()
    d2[pick[:32]] = 0.0                       # solid
    d2[pick[32:40]] = -0.25                   # solid (negative distances fire too)
    d2[pick[40:]] = 0.0
    d2[pick[40:], 5, 7] = np.nan              # not solid: a texel without data never fires
    grid.set_distance(torch.from_numpy(d2).cuda())
    fresh = pt.ProbeGrid(probes.dims, probes.origin, probes.spacing, N, probes.levels, probes.scene_min,
                         probes.scene_max, torch.from_numpy(d2).cuda(),
                         torch.from_numpy(probes.normal.view(np.float16)).cuda())
    a = _np(pt.probe_trace(grid, rad, views[:1]))
    _same(a, _np(pt.probe_trace(fresh, rad, views[:1])), "set_distance vs fresh grid")
    _same(a, _np(pt.probe_trace(grid, rad, views[:1], pt.trace_opts(flags=pt.PT_FLAG_TRACE_ALL_PROBES))),
          "set_distance, solid probes traced")
    og = oracle.Grid(probes.dims, probes.origin, probes.spacing, N, probes.levels, probes.scene_min, probes.scene_max,
                     d2, probes.normal, rad16.astype(np.float32))
    orc = oracle.trace_view(og, views[0].as_tuple())
    assert_parity(compare(a, orc), "room with zeroed probes")
    # and back: the original distances clear the flags again
    grid.set_distance(torch.from_numpy(probes.distance.copy()).cuda())
    orig = _np(pt.probe_trace(pt.ProbeGrid.from_probes(probes), rad, views[:1]))
    _same(_np(pt.probe_trace(grid, rad, views[:1])), orig, "restored")
    assert (a["status"] == oracle.UNKNOWN).sum() > (orig["status"] == oracle.UNKNOWN).sum()


def test_fewer_than_8_probes_with_a_solid_probe():
    from test_oracle_few import few_room
    pt = _pt()
    scene, probes, views = few_room((2, 2, 1), size=(160, 100))
    d2 = probes.distance.copy()
    d2[1] = 0.0
    rad16 = probes.radiance.view(np.float16)
    rad = torch.from_numpy(rad16.copy()).cuda()
    grid = pt.ProbeGrid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                        probes.scene_max, torch.from_numpy(d2).cuda(),
                        torch.from_numpy(probes.normal.view(np.float16)).cuda())
    a = _np(pt.probe_trace(grid, rad, views))
    for flags in (pt.PT_FLAG_TRACE_ALL_PROBES, pt.PT_FLAG_PERSISTENT):
        _same(a, _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags))), ("few", flags))
    og = oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                     probes.scene_max, d2, probes.normal, rad16.astype(np.float32))
    assert_parity(compare(a, oracle.trace_view(og, views[0].as_tuple())), "few (2,2,1), probe 1 solid")
    assert np.all(a["hit"][a["status"] == oracle.HIT, 0] != 1)


@pytest.mark.parametrize("name,kw,nviews", [("single", dict(size=(480, 270)), 1), ("batched", {}, 6),
                                            ("paper", dict(size=(480, 270)), 1)])
def test_eye_cell_skip_gives_identical_results(name, kw, nviews):
    # every ray starts in the eye's cell, where the start texel of each cage probe is the
    # same for the whole view: probes whose start texel fires behind the surface are left
    # out; the outputs must be those of tracing them
    pt = _pt()
    scene, probes, views = workload(name, **kw)
    views = views[:nviews]
    grid = pt.ProbeGrid.from_probes(probes)
    rad16 = probes.radiance.view(np.float16)
    rad = torch.from_numpy(rad16.copy()).cuda()
    ref = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_TRACE_ALL_PROBES)))
    for flags in (0, pt.PT_FLAG_PERSISTENT, pt.PT_FLAG_GRAPH):
        _same(_np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags))), ref, (name, flags))
    if nviews == 1 and name == "single":
        og = oracle.Grid.from_probes(probes)
        assert_parity(compare(ref, oracle.trace_view(og, views[0].as_tuple())), f"{name} eye-cell skip")
    # the recomputing adjoint walks the same tables: the same sums up to the order of the
    # FP32 additions, bounded by the sum of the contributions' magnitudes (the adjoint of |g|)
    rays = sum(v.width * v.height for v in views)
    g = torch.from_numpy(np.random.default_rng(5).normal(size=(rays, 3)).astype(np.float32)).cuda()
    grads = []
    for flags, gg in ((0, g), (pt.PT_FLAG_TRACE_ALL_PROBES, g), (pt.PT_FLAG_TRACE_ALL_PROBES, g.abs())):
        gr = torch.zeros((probes.n_probes, probes.N, probes.N, 3), device="cuda")
        pt.probe_trace_backward(grid, views, gg, gr, pt.trace_opts(flags=flags | pt.PT_FLAG_PERSISTENT))
        grads.append(gr.cpu().numpy().astype(np.float64))
    err = np.abs(grads[0] - grads[1])
    assert (err <= 1e-5 * grads[2] + 1e-7).all(), (err / (grads[2] + 1e-7)).max()
    assert np.array_equal(grads[0] != 0, grads[1] != 0)
    assert np.count_nonzero(grads[1]) > 1000


def test_clear_probes_skip_gives_identical_results():
    # the sparse 16x16x8 grid (reduced maps): a large share of its probes are clear of their
    # cells; then the same distances pulled in to half, where far fewer are
    pt = _pt()
    scene, probes, views = workload("diff", N=64, levels=4, n_views=2, size=(160, 128))
    grid = pt.ProbeGrid.from_probes(probes)
    rad16 = probes.radiance.view(np.float16)
    rad = torch.from_numpy(rad16.copy()).cuda()
    rays = sum(v.width * v.height for v in views)
    g = torch.from_numpy(np.random.default_rng(6).normal(size=(rays, 3)).astype(np.float32)).cuda()
    gt = torch.from_numpy(np.random.default_rng(7).normal(size=rays).astype(np.float32)).cuda()
    P, N = probes.n_probes, probes.N
    for scale in (1.0, 0.5):
        if scale != 1.0:
            grid.set_distance(torch.from_numpy((probes.distance * scale).astype(np.float32)).cuda())
        ref = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_TRACE_ALL_PROBES)))
        for flags in (0, pt.PT_FLAG_PERSISTENT, pt.PT_FLAG_GRAPH):
            _same(_np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags))), ref, (scale, flags))
        if scale == 1.0:
            og = oracle.Grid.from_probes(probes)
            o = np.concatenate([oracle.view_rays(*v.as_tuple())[0] for v in views])
            d = np.concatenate([oracle.view_rays(*v.as_tuple())[1] for v in views])
            assert_parity(compare(ref, oracle.trace(og, o, d)), "sparse grid, clear probes left out")
        res = []
        for flags, gg in ((0, g), (pt.PT_FLAG_TRACE_ALL_PROBES, g), (pt.PT_FLAG_TRACE_ALL_PROBES, g.abs())):
            gr = torch.zeros((P, N, N, 3), device="cuda")
            pt.probe_trace_backward(grid, views, gg, gr, pt.trace_opts(flags=flags | pt.PT_FLAG_PERSISTENT))
            gd = torch.zeros((P, N, N), device="cuda")
            pt.probe_trace_backward_distance(grid, rad, views, g, gt, gd, pt.trace_opts(flags=flags))
            res.append((gr.cpu().numpy().astype(np.float64), gd.cpu().numpy().astype(np.float64)))
        # radiance: bounded by the adjoint of |g| (every term positive); distance: its terms
        # carry signed d rgb / d t, so relative to the texel's value and the largest one
        tols = (1e-5 * res[2][0] + 1e-7, 1e-4 * np.abs(res[1][1]) + 1e-6 * np.abs(res[1][1]).max())
        for k in range(2):
            err = np.abs(res[0][k] - res[1][k])
            assert (err <= tols[k]).all(), (scale, k, (err / tols[k]).max())
            assert np.array_equal(res[0][k] != 0, res[1][k] != 0), (scale, k)


def _look_at(pos, target, w, h, tan_half=0.6):
    import synth
    pos, target = np.asarray(pos, np.float64), np.asarray(target, np.float64)
    fwd = target - pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return synth.View(pos.astype(np.float32).astype(np.float64), right, up, fwd, tan_half, w, h)


@pytest.mark.parametrize("where", ["outside_the_box", "on_probe_planes"])
def test_known_answer_skip_with_unusual_eyes(where):
    # eyes the region and octant rules must allow for: outside the scene box (the walk's
    # first cells are clamped and their segments start far from the grid) and exactly on
    # probe planes along x and z (pieces in those planes take the octant across)
    pt = _pt()
    scene, probes, views = workload("diff", N=64, levels=4, n_views=1, size=(64, 64))
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    room = np.asarray(scene.room_max, np.float64)
    if where == "outside_the_box":
        v = _look_at(room + np.array([3.0, 2.0, 1.5]), 0.5 * room, 160, 120)
    else:
        org, spc = np.asarray(probes.origin, np.float64), np.asarray(probes.spacing, np.float64)
        pos = np.array([org[0] + 5 * spc[0], 0.37 * room[1], org[2] + 3 * spc[2]])
        v = _look_at(pos, pos + np.array([0.0, 5.0, 0.0]), 160, 120)
    a = _np(pt.probe_trace(grid, rad, [v]))
    b = _np(pt.probe_trace(grid, rad, [v], pt.trace_opts(flags=pt.PT_FLAG_TRACE_ALL_PROBES)))
    _same(a, b, where)
    orc = oracle.trace_view(oracle.Grid.from_probes(probes), v.as_tuple())
    s = compare(a, orc)
    if where == "outside_the_box":
        assert_parity(s, f"unusual eye: {where}")
    else:
        # an eye on probe planes makes every ray an exact tie of the kind the degenerate-ray
        # tests cover, held to their bar: every disagreement in the margin, at most 1%, and
        # every reported HIT valid
        from degenerate import hit_is_valid
        info = {k: val for k, val in s.items() if k != "disagree_idx"}
        print(f"[parity] unusual eye: {where} {info}", flush=True)
        assert s["disagree_outside_margin"] == 0 and s["disagree"] <= 0.01 * s["n"], info
        o, d = oracle.view_rays(*v.as_tuple())
        assert hit_is_valid(probes, o, d, a["status"], a["hit"], a["t"], 8.0 / probes.N).all()
        assert (a["status"] == oracle.HIT).mean() > 0.5

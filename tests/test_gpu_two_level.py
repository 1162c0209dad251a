"""Two-level probe hierarchy on the GPU (probe_grid_set_coarse) against the oracle's two-level
walk, on a seeded city block (fine 16x16x8 probes, coarse 4x4x2 on every 4th fine plane),
and the 64-bit probe addressing path (PT_FLAG_WIDE), which must give identical results."""
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


_CACHE = {}


def _city(**kw):
    key = tuple(sorted(kw.items()))
    if key not in _CACHE:
        pt = _pt()
        scene, tl, views = workload("large_small", **kw)
        grid = pt.ProbeGrid.from_two_level(tl)
        rad = torch.from_numpy(tl.radiance().view(np.float16).copy()).cuda()
        og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
        _CACHE[key] = (scene, tl, views, grid, rad, og, cg)
    return _CACHE[key]


def _np(res):
    return {k: v.cpu().numpy() for k, v in res.items() if v is not None}


def _oracle_views(tl, og, cg, views, **kw):
    o = np.concatenate([oracle.view_rays(*v.as_tuple())[0] for v in views])
    d = np.concatenate([oracle.view_rays(*v.as_tuple())[1] for v in views])
    return oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio), **kw)


def test_two_level_parity_per_view_launches():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    res = _np(pt.probe_trace(grid, rad, views))
    orc = _oracle_views(tl, og, cg, views)
    s = compare(res, orc)
    assert_parity(s, "city two-level, 2 views")
    coarse = (res["status"] == oracle.HIT) & (res["hit"][:, 0] >= tl.fine.n_probes)
    assert coarse.sum() > 100  # the coarse level resolves rays on the GPU too


def test_two_level_larger_frames_and_nearest():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city(size=(320, 200))
    for flags, kw in ((0, {}), (pt.PT_FLAG_NEAREST, dict(nearest=True))):
        res = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags)))
        assert_parity(compare(res, _oracle_views(tl, og, cg, views, **kw)), f"city 320x200 {kw}")


def test_wide_addressing_gives_identical_results():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    a = _np(pt.probe_trace(grid, rad, views))
    b = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_WIDE)))
    for k in ("status", "hit", "t", "rgb"):
        assert np.array_equal(a[k], b[k]), k
    # and on a single-level grid
    sc, probes, sv = workload("single", size=(240, 135))
    g1 = pt.ProbeGrid.from_probes(probes)
    r1 = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    a = _np(pt.probe_trace(g1, r1, sv))
    b = _np(pt.probe_trace(g1, r1, sv, pt.trace_opts(flags=pt.PT_FLAG_WIDE)))
    for k in ("status", "hit", "t", "rgb"):
        assert np.array_equal(a[k], b[k]), k


def test_two_level_persistent_and_graph_launches_identical():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    ref = _np(pt.probe_trace(grid, rad, views))
    for flags in (pt.PT_FLAG_PERSISTENT, pt.PT_FLAG_GRAPH, pt.PT_FLAG_GRAPH | pt.PT_FLAG_WIDE):
        for rep in range(2):
            got = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags)))
            torch.cuda.synchronize()
            for k in ("status", "hit", "t", "rgb"):
                assert np.array_equal(got[k], ref[k]), (flags, rep, k)


def test_two_level_arbitrary_rays():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    import synth
    rng = np.random.default_rng(4)
    # free-space origins (clearance from every surface) and random directions
    o = []
    while len(o) < 40000:  # enough rays to measure the 1e-4 disagreement rate
        p = rng.uniform([0.2, 0.2, 0.2], scene.room_max - 0.2)
        if synth.clearance(scene, p) > 0.05:
            o.append(p)
    o = np.array(o, np.float32)
    d = rng.normal(size=o.shape).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    res = _np(pt.probe_trace_rays(grid, rad, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()))
    orc = oracle.trace(og, o.astype(np.float64), d.astype(np.float64), coarse=(cg, tl.plane_off, tl.ratio))
    assert_parity(compare(res, orc), "city arbitrary rays")


def test_two_level_backward_matches_oracle_vjp():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    res = _np(pt.probe_trace(grid, rad, views))
    orc = _oracle_views(tl, og, cg, views)
    s = compare(res, orc)
    rng = np.random.default_rng(9)
    g = rng.normal(size=(s["n"], 3)).astype(np.float32)
    g[s["disagree_idx"]] = 0.0
    gg = torch.zeros((tl.n_probes, tl.fine.N, tl.fine.N, 3), device="cuda")
    pt.probe_trace_backward(grid, views, torch.from_numpy(g).cuda(), gg)
    got = gg.cpu().numpy().astype(np.float64)
    # the persistent adjoint over both views, and the adjoint from the forward's stored hits
    # (coarse probes included): the same sums up to the order of the FP32 atomics, so each
    # is held to the oracle with the same per-texel bound
    gp = torch.zeros_like(gg)
    pt.probe_trace_backward(grid, views, torch.from_numpy(g).cuda(), gp, pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT))
    r2 = pt.probe_trace(grid, rad, views)
    gh = torch.zeros_like(gg)
    pt.probe_trace_backward_hits(grid, views, r2["hit"], r2["t"], torch.from_numpy(g).cuda(), gh)
    ref = oracle.vjp((og, cg), orc, g.astype(np.float64))
    wabs = oracle.vjp((og, cg), orc, np.abs(g).astype(np.float64))
    unit = dict(orc)
    unit["wts"] = (orc["wts"] != 0).astype(np.float64)
    gabs = oracle.vjp((og, cg), unit, np.abs(g).astype(np.float64))
    tol = 1e-5 * wabs + 1e-3 * gabs + 1e-8
    for label, x in (("per view", got), ("persistent", gp.cpu().numpy().astype(np.float64)),
                     ("stored hits", gh.cpu().numpy().astype(np.float64))):
        err = np.abs(x - ref)
        print(f"[grad] city two-level {label} max err/tol {(err / tol).max():.3f} nonzero {np.count_nonzero(ref)}",
              flush=True)
        assert not (err > tol).any(), label
    assert np.count_nonzero(ref[tl.fine.n_probes:]) > 100  # coarse texels receive gradient


def test_set_coarse_checks_planes_and_detaches():
    pt = _pt()
    scene, tl, views, grid, rad, og, cg = _city()
    with pytest.raises(pt.ProbeTraceError):
        grid.set_coarse(grid.coarse, (0, 1, 1), tl.ratio)  # coarse planes are not fine plane 0 + 4k
    with pytest.raises(pt.ProbeTraceError):
        grid.set_coarse(grid.coarse, tl.plane_off, (2, 4, 4))
    # the failed calls left the hierarchy as it was
    a = _np(pt.probe_trace(grid, rad, views))
    assert_parity(compare(a, _oracle_views(tl, og, cg, views)), "after rejected re-attach")
    coarse = grid.coarse
    grid.set_coarse(None)
    try:
        one = _np(pt.probe_trace(grid, rad[:tl.fine.n_probes].contiguous(), views))
        o = np.concatenate([oracle.view_rays(*v.as_tuple())[0] for v in views])
        d = np.concatenate([oracle.view_rays(*v.as_tuple())[1] for v in views])
        assert_parity(compare(one, oracle.trace(og, o, d)), "detached: fine level alone")
    finally:
        grid.set_coarse(coarse, tl.plane_off, tl.ratio)

"""probe_trace_noalloc, the entry point that allocates nothing (its scratch is a fixed
device array), against probe_trace through the C ABI: the same per-view kernels, so the
outputs must be equal bit for bit, call after call on one GPU (the fixed array keeps the
previous call's tables, and each call must rewrite what it reads), including a smaller
input after a larger one, another grid, and a two-level hierarchy (both levels' tables).
Its refusals: persistent and graph launch forms, grids with more cells than the array."""
import numpy as np
import pytest
import torch

from conftest import workload

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _outs(rays):
    # filled with values no trace writes, so a ray the call skipped cannot pass
    return (torch.full((rays, 3), -7.0, device="cuda"), torch.full((rays,), -7.0, device="cuda"),
            torch.full((rays,), 255, dtype=torch.uint8, device="cuda"),
            torch.full((rays, 2), -7, dtype=torch.int32, device="cuda"))


def _np(res):
    return {k: v.cpu().numpy() for k, v in res.items()}


def _check_equal(pt, grid, rad, views, opts=None):
    va = pt.make_views(views)
    rays = pt.n_rays(views)
    ref = _np(pt.probe_trace(grid, rad, va, opts))
    got = _np(pt.probe_trace_noalloc(grid, rad, va, _outs(rays), opts))
    torch.cuda.synchronize()
    for k in ("rgb", "t", "status", "hit"):
        assert np.array_equal(got[k], ref[k]), k
    return ref


def test_noalloc_matches_probe_trace_call_after_call():
    pt = _pt()
    import synth
    scene, probes, views = workload("single", size=(240, 135))
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    uneven = [views[0], synth.make_views(scene, 8, 1, 97, 61)[0], synth.make_views(scene, 9, 1, 33, 200)[0]]
    # first call: three views of uneven size; second call: one smaller view of the same grid
    ref = _check_equal(pt, grid, rad, uneven)
    assert (ref["status"] == 1).mean() > 0.5
    _check_equal(pt, grid, rad, [synth.make_views(scene, 10, 1, 50, 40)[0]])
    # other launch options (tile shape, start level, nearest radiance)
    _check_equal(pt, grid, rad, uneven[1:], pt.trace_opts(tile=(4, 16), start_level=2, flags=pt.PT_FLAG_NEAREST))
    # another grid with fewer cells (one cell): the tables are rewritten, not reused
    tscene, tprobes, tviews = workload("tiny")
    tgrid = pt.ProbeGrid.from_probes(tprobes)
    trad = torch.from_numpy(tprobes.radiance.view(np.float16).copy()).cuda()
    _check_equal(pt, tgrid, trad, [synth.make_views(tscene, 3, 1, 64, 48)[0]])
    # and the first grid again
    _check_equal(pt, grid, rad, uneven[:1])


def test_noalloc_two_level_hierarchy():
    pt = _pt()
    scene, tl, views = workload("large_small")
    grid = pt.ProbeGrid.from_two_level(tl)
    rad = torch.from_numpy(tl.radiance().view(np.float16).copy()).cuda()
    ref = _check_equal(pt, grid, rad, views)
    assert (ref["status"] == 1).mean() > 0.5
    _check_equal(pt, grid, rad, views[:1])


def test_noalloc_refusals():
    pt = _pt()
    scene, probes, views = workload("tiny")
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    rays = pt.n_rays(views)
    for flags in (pt.PT_FLAG_PERSISTENT, pt.PT_FLAG_GRAPH):
        with pytest.raises(pt.ProbeTraceError, match="per-view launches only"):
            pt.probe_trace_noalloc(grid, rad, views, _outs(rays), pt.trace_opts(flags=flags))
    # 66^3 probes of 8x8 maps: 65^3 = 274,625 cells, above the 262,144 the array holds
    n, N = 66, 8
    dist = torch.ones((n ** 3, N, N), device="cuda")
    nrm = torch.zeros((n ** 3, N, N, 2), dtype=torch.float16, device="cuda")
    big = pt.ProbeGrid((n, n, n), (0.5,) * 3, (1.0,) * 3, N, 1, (0, 0, 0), (n,) * 3, dist, nrm)
    brad = torch.zeros((n ** 3, N, N, 3), dtype=torch.float16, device="cuda")
    with pytest.raises(pt.ProbeTraceError, match="cells"):
        pt.probe_trace_noalloc(big, brad, views, _outs(rays))
    del big, brad, dist, nrm
    # the library still serves valid calls after the refusals
    _check_equal(pt, grid, rad, views)

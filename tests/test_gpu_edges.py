"""Edge cases of the C ABI on the GPU: views of one pixel, one row and one column, views
whose sides are not multiples of any tile side, such views mixed into one launch; the
largest view side the library accepts and the first one it refuses; empty ray batches;
views that see nothing (every ray a MISS) through the forward and both radiance adjoints."""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import workload
from parity import compare, assert_parity

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


_CACHE = {}


def _room():
    if "room" not in _CACHE:
        pt = _pt()
        scene, probes, views = workload("single", size=(240, 135))
        grid = pt.ProbeGrid.from_probes(probes)
        rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
        _CACHE["room"] = (probes, views[0], grid, rad, oracle.Grid.from_probes(probes))
    return _CACHE["room"]


def _resized(v, w, h):
    return synth.View(v.pos, v.right, v.up, v.fwd, v.tan_half_fov_y, w, h)


def _np(res):
    return {k: x.cpu().numpy() for k, x in res.items() if x is not None}


SIZES = [(1, 1), (1, 37), (129, 1), (65, 3), (7, 9)]


@pytest.mark.parametrize("size", SIZES)
def test_small_and_thin_views_match_oracle(size):
    pt = _pt()
    probes, v0, grid, rad, og = _room()
    v = _resized(v0, *size)
    orc = oracle.trace_view(og, v.as_tuple())
    for label, opts in (("per-view", None), ("persistent", pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)),
                        ("tile 64x1", pt.trace_opts(tile=(64, 1)))):
        res = _np(pt.probe_trace(grid, rad, [v], opts))
        assert res["rgb"].shape == (size[0] * size[1], 3)
        assert_parity(compare(res, orc), f"{size[0]}x{size[1]} {label}")


def test_mixed_view_sizes_in_one_launch():
    # tiny and ragged views between full ones: every launch form gives the same bits, and
    # each view's slice of the concatenated outputs matches the oracle
    pt = _pt()
    probes, v0, grid, rad, og = _room()
    views = [_resized(v0, *s) for s in [(1, 1), (240, 135), (1, 37), (65, 3), (129, 1), (96, 54), (1, 1)]]
    a = _np(pt.probe_trace(grid, rad, views))
    b = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)))
    c = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_GRAPH)))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    off = 0
    for v in views:
        n = v.width * v.height
        sl = {k: x[off:off + n] for k, x in a.items()}
        assert_parity(compare(sl, oracle.trace_view(og, v.as_tuple())), f"{v.width}x{v.height} in batch")
        off += n
    assert off == len(a["status"])


def test_largest_view_side_and_the_first_refused():
    pt = _pt()
    probes, v0, grid, rad, og = _room()
    wide = _resized(v0, 65536, 1)
    res = _np(pt.probe_trace(grid, rad, [wide]))
    pix = np.sort(np.random.default_rng(5).choice(65536, 4000, replace=False))
    assert_parity(compare(res, oracle.trace_view(og, wide.as_tuple(), pixels=pix), sel=pix), "65536x1 sampled")
    tall = _resized(v0, 1, 65536)
    res = _np(pt.probe_trace(grid, rad, [tall], pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)))
    assert_parity(compare(res, oracle.trace_view(og, tall.as_tuple(), pixels=pix), sel=pix), "1x65536 sampled")
    for bad in [(65537, 1), (1, 65537), (0, 4), (4, 0)]:
        with pytest.raises(pt.ProbeTraceError):
            pt.probe_trace(grid, rad, [_resized(v0, *bad)])
    with pytest.raises(pt.ProbeTraceError):
        pt.probe_trace(grid, rad, [synth.View(v0.pos, v0.right, v0.up, v0.fwd, 0.0, 4, 4)])
    # non-finite camera parameters are refused before any launch, for every entry point
    # that takes views
    for field in ("pos", "right", "up", "fwd"):
        for bad in (np.nan, np.inf):
            kw = dict(pos=v0.pos, right=v0.right, up=v0.up, fwd=v0.fwd)
            vec = np.array(kw[field], np.float64)
            vec[1] = bad
            kw[field] = vec
            v = synth.View(kw["pos"], kw["right"], kw["up"], kw["fwd"], v0.tan_half_fov_y, 4, 4)
            with pytest.raises(pt.ProbeTraceError, match="finite"):
                pt.probe_trace(grid, rad, [v])
            with pytest.raises(pt.ProbeTraceError, match="finite"):
                pt.probe_trace_backward(grid, [v], torch.zeros((16, 3), device="cuda"),
                                        torch.zeros((probes.n_probes, probes.N, probes.N, 3), device="cuda"))


def test_empty_ray_batch():
    pt = _pt()
    probes, v0, grid, rad, og = _room()
    z = torch.empty((0, 3), device="cuda")
    res = pt.probe_trace_rays(grid, rad, z, z)
    assert all(x.numel() == 0 for x in res.values() if x is not None)
    torch.cuda.synchronize()


def test_view_that_sees_nothing():
    # an eye outside the scene box looking away from it: every ray leaves at once
    pt = _pt()
    probes, v0, grid, rad, og = _room()
    pos = np.asarray(probes.scene_max, np.float64) + 1.0
    fwd = np.array([1.0, 0.0, 0.0])
    v = synth.View(pos, np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0]), fwd, 0.5, 33, 17)
    bg = (0.25, 0.5, 0.75)
    res = _np(pt.probe_trace(grid, rad, [v], pt.trace_opts(background=bg)))
    orc = oracle.trace_view(og, v.as_tuple())
    assert np.all(orc["status"] == oracle.MISS)
    assert np.all(res["status"] == oracle.MISS)
    assert np.all(np.isinf(res["t"])) and np.all(res["hit"] == -1)
    assert np.array_equal(res["rgb"], np.broadcast_to(np.float32(bg), res["rgb"].shape))
    rays = v.width * v.height
    g = torch.ones((rays, 3), device="cuda")
    gr = torch.zeros((probes.n_probes, probes.N, probes.N, 3), device="cuda")
    pt.probe_trace_backward(grid, [v], g, gr)
    hit = torch.from_numpy(res["hit"]).cuda()
    t = torch.from_numpy(res["t"]).cuda()
    pt.probe_trace_backward_hits(grid, [v], hit, t, g, gr)
    assert torch.count_nonzero(gr).item() == 0

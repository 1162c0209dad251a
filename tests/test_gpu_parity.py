"""Parity of the HIP trace (through the C ABI) against the CPU oracle.

Sizes: the tiny room in full (16,384 rays, several tiles and a ragged tail once cropped),
the 1080p room's scene through a 240x135 view in full, the full 1920x1080 launch (the
benchmark's configuration) on sampled pixels, arbitrary rays (including rays from probe
centres and degenerate directions), and multi-view launches (plain, persistent, graph).
"""
import numpy as np
import pytest
import torch

import oracle
from conftest import workload
from parity import compare, assert_parity

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _gpu_numpy(res):
    return {k: v.cpu().numpy() for k, v in res.items() if v is not None}


_GRIDS = {}


def _grid(name, **kw):
    pt = _pt()
    key = (name, tuple(sorted(kw.items())))
    if key not in _GRIDS:
        scene, probes, views = workload(name, **kw)
        grid = pt.ProbeGrid.from_probes(probes)
        rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
        _GRIDS[key] = (scene, probes, views, grid, rad)
    return _GRIDS[key]


def _oracle_grid(probes):
    return oracle.Grid.from_probes(probes)


def test_pyramid_is_bit_exact():
    pt = _pt()
    scene, probes, views, grid, rad = _grid("single", size=(240, 135))
    ref = oracle.min_mips(probes.distance, probes.levels)
    for l in range(probes.levels):
        got = grid.read_level(l).cpu().numpy()
        assert got.dtype == np.float32
        assert np.array_equal(got.view(np.uint32), ref[l].view(np.uint32)), l


def test_pyramid_nan_and_zero_texels():
    pt = _pt()
    rng = np.random.default_rng(3)
    P, N, L = 8, 32, 4
    dist = rng.uniform(0.1, 3, size=(P, N, N)).astype(np.float32)
    dist[1, 3, 4] = np.nan
    dist[2, :8, :8] = np.nan
    dist[3] = 0.0
    nrm = np.zeros((P, N, N, 2), np.float16)
    g = pt.ProbeGrid((2, 2, 2), (0.25,) * 3, (0.5,) * 3, N, L, (0, 0, 0), (1, 1, 1), torch.from_numpy(dist).cuda(),
                     torch.from_numpy(nrm).cuda())
    ref = oracle.min_mips(dist, L)
    for l in range(L):
        got = g.read_level(l).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref[l].view(np.uint32)), l


def _trace_view(name, view_index=0, pixels=None, opts=None, **kw):
    pt = _pt()
    scene, probes, views, grid, rad = _grid(name, **kw)
    v = views[view_index]
    res = _gpu_numpy(pt.probe_trace(grid, rad, [v], opts))
    orc = oracle.trace_view(_oracle_grid(probes), v.as_tuple(), pixels=pixels)
    return res, orc


def test_parity_tiny_full_view():
    res, orc = _trace_view("tiny")
    assert_parity(compare(res, orc), "tiny 128x128")


def test_parity_room_full_crop_view():
    res, orc = _trace_view("single", size=(240, 135))
    assert_parity(compare(res, orc), "room 240x135")


def test_parity_room_ragged_tiles():
    # a view size that is not a multiple of any tile shape
    res, orc = _trace_view("single", size=(203, 77))
    s = compare(res, orc)
    assert_parity(s, "room 203x77")


@pytest.mark.parametrize("tile", [(8, 8), (16, 4), (32, 2), (64, 1), (4, 16)])
def test_tile_shapes_do_not_change_results(tile):
    pt = _pt()
    scene, probes, views, grid, rad = _grid("single", size=(240, 135))
    a = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]]))
    b = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]], pt.trace_opts(tile=tile)))
    for k in a:
        assert np.array_equal(a[k], b[k]), (tile, k)


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_start_level_does_not_change_results(level):
    pt = _pt()
    scene, probes, views, grid, rad = _grid("single", size=(240, 135))
    a = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]]))
    b = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]], pt.trace_opts(start_level=level)))
    st_same = (a["status"] == b["status"]).mean()
    assert st_same > 1 - 1e-4
    same = (a["status"] == b["status"]) & (a["hit"] == b["hit"]).all(1)
    assert same.mean() > 1 - 1e-4


def test_parity_full_1080p_sampled_pixels():
    # the benchmark's workload in the launch configuration it times (the stored tuned
    # options; the library defaults if none are stored), and the library defaults
    pt = _pt()
    from paper_2507_14624_amd import tuning
    scene, probes, views, grid, rad = _grid("single")
    v = views[0]
    entry = tuning.load("single_1080p")
    rng = np.random.default_rng(7)
    n = v.width * v.height
    pix = np.sort(rng.choice(n, 60000, replace=False))
    orc = oracle.trace_view(_oracle_grid(probes), v.as_tuple(), pixels=pix)
    for label, opts in (("tuned", tuning.apply(pt.trace_opts(), entry) if entry else None), ("defaults", None)):
        res = _gpu_numpy(pt.probe_trace(grid, rad, [v], opts))
        assert_parity(compare(res, orc, sel=pix), f"1920x1080 sampled 60k, {label} launch")


def test_parity_arbitrary_rays_and_probe_centres():
    pt = _pt()
    scene, probes, views, grid, rad = _grid("tiny")
    og = _oracle_grid(probes)
    rng = np.random.default_rng(8)
    n = 4000
    # random rays from free space inside the room, FP32 inputs shared by both sides
    import synth
    o = rng.uniform(0.05, 0.95, size=(3 * n, 3))
    o = o[[synth.clearance(scene, x) > 0.01 for x in o]][:n].astype(np.float32)
    n = len(o)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    # rays from every probe centre through texel centres (eye aligned with the probe)
    P = probes.n_probes
    N = probes.N
    po = np.stack([og.probe_position(p) for p in range(P)]).astype(np.float32)
    ks = rng.choice(N * N, size=(P, 64))
    c = -1 + (2 * np.arange(N) + 1) / N
    de = np.array([oracle.oct_decode(np.array([c[k % N], c[k // N]])) for k in ks.ravel()]).astype(np.float32)
    o = np.concatenate([o, np.repeat(po, 64, axis=0)])
    d = np.concatenate([d, de])
    o[5], d[5] = o[4], 0.0  # degenerate direction
    res = _gpu_numpy(pt.probe_trace_rays(grid, rad, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()))
    keep = np.ones(len(o), bool)
    keep[5] = False
    orc = oracle.trace(og, o[keep].astype(np.float64), d[keep].astype(np.float64))
    assert_parity(compare(res, orc, sel=keep), "arbitrary rays")
    assert res["status"][5] == oracle.MISS and np.isinf(res["t"][5])
    eye = np.arange(n, len(o))
    pe = np.repeat(np.arange(P), 64)
    assert np.all(res["status"][eye] == oracle.HIT)
    assert np.array_equal(res["hit"][eye, 0], pe) and np.array_equal(res["hit"][eye, 1], ks.ravel())
    assert np.array_equal(res["t"][eye], probes.distance.reshape(P, -1)[pe, ks.ravel()])


def test_parity_options():
    pt = _pt()
    scene, probes, views, grid, rad = _grid("tiny")
    og = _oracle_grid(probes)
    v = views[0]
    # the paper-literal variants (two cage probes per cell; no shadow-entry rule, i.e. the
    # appendix classification as printed; the hit texel's own radiance) and plain options
    for kw in (dict(max_probes_per_cell=2), dict(thickness_rel=0.02), dict(thickness_rel=float("inf")),
               dict(background=(0.25, 0.5, 1.0)), dict(nearest=True),
               dict(nearest=True, thickness_rel=float("inf"), max_probes_per_cell=2)):
        gkw = {k: val for k, val in kw.items() if k != "nearest"}
        if kw.get("nearest"):
            gkw["flags"] = pt.PT_FLAG_NEAREST
        res = _gpu_numpy(pt.probe_trace(grid, rad, [v], pt.trace_opts(**gkw)))
        orc = oracle.trace_view(og, v.as_tuple(), **kw)
        assert_parity(compare(res, orc), f"tiny {kw}")
        if kw.get("nearest"):
            # exactly the stored FP16 radiance of the hit texel
            h = res["status"] == oracle.HIT
            R = probes.radiance.view(np.float16).astype(np.float32).reshape(probes.n_probes, -1, 3)
            assert np.array_equal(res["rgb"][h], R[res["hit"][h, 0], res["hit"][h, 1]])


def test_parity_incoming_direction_normal_maps():
    # the literal normal maps of the probe data generation (probe-to-point directions)
    import synth
    pt = _pt()
    scene, probes, views = workload("single", size=(240, 135))
    lit = synth.bake(scene, probes.N, probes.levels, normals="incoming")
    grid = pt.ProbeGrid.from_probes(lit)
    rad = torch.from_numpy(lit.radiance.view(np.float16).copy()).cuda()
    res = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]]))
    orc = oracle.trace_view(_oracle_grid(lit), views[0].as_tuple())
    s = compare(res, orc)
    assert_parity(s, "room 240x135, incoming-direction normals")
    assert 0.05 < s["hit_frac"] < 0.95


def _batch_views(k=6, shrink=8):
    """k views of the batched walk, shrunk (keeping uneven sizes) to keep tests short."""
    import dataclasses
    scene, probes, views = workload("batched", n_views=k)
    return [dataclasses.replace(v, width=max(17, v.width // shrink), height=max(9, v.height // shrink))
            for v in views]


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("single", dict(size=(240, 135))),
                                     ("diff", dict(N=64, levels=4, n_views=2, size=(256, 200)))])
def test_start_texel_test_does_not_change_results(name, kw):
    # deciding pieces whose first texel fires on entry without the march is exact: forced on
    # and forced off give the same bits, per view and persistent
    pt = _pt()
    scene, probes, views, grid, rad = _grid(name, **kw)
    for flags in (0, pt.PT_FLAG_PERSISTENT):
        on = _gpu_numpy(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags | pt.PT_FLAG_START_TEXEL)))
        off = _gpu_numpy(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=flags | pt.PT_FLAG_NO_START_TEXEL)))
        both = _gpu_numpy(pt.probe_trace(grid, rad, views, pt.trace_opts(
            flags=flags | pt.PT_FLAG_START_TEXEL | pt.PT_FLAG_NO_START_TEXEL)))
        for k in on:
            assert np.array_equal(on[k], off[k]), (flags, k)
            assert np.array_equal(both[k], off[k]), (flags, k)
    og = _oracle_grid(probes)
    v = views[0]
    n = v.width * v.height
    assert_parity(compare({k: x[:n] for k, x in on.items()}, oracle.trace_view(og, v.as_tuple())),
                  f"{name} start-texel test on")


def test_multiview_plain_persistent_graph_identical():
    pt = _pt()
    scene, probes, views1, grid, rad = _grid("single", size=(240, 135))
    views = _batch_views(6)
    a = _gpu_numpy(pt.probe_trace(grid, rad, views))
    b = _gpu_numpy(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)))
    c1 = pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_GRAPH))
    c1 = _gpu_numpy(c1)
    c2 = _gpu_numpy(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_GRAPH)))  # replay
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c1[k]), k
        assert np.array_equal(a[k], c2[k]), k
    # and against the oracle, view by view
    og = _oracle_grid(probes)
    off = 0
    for v in views:
        n = v.width * v.height
        orc = oracle.trace_view(og, v.as_tuple())
        sl = {k: x[off:off + n] for k, x in a.items()}
        assert_parity(compare(sl, orc), f"view {v.width}x{v.height}")
        off += n


def test_graph_replays_with_eager_work_between():
    pt = _pt()
    scene, probes, views1, grid, rad = _grid("single", size=(240, 135))
    views = _batch_views(3)
    ref = _gpu_numpy(pt.probe_trace(grid, rad, views))
    out = None
    for rep in range(4):
        r = pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_GRAPH), out=out)
        out = (r["rgb"], r["t"], r["status"], r["hit"])
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        got = _gpu_numpy(r)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (rep, k)
        r["rgb"].fill_(-1.0)  # stale outputs must be overwritten by the next replay


def test_autotune_picks_valid_options_and_results_unchanged():
    pt = _pt()
    scene, probes, views, grid, rad = _grid("single", size=(240, 135))
    o = pt.probe_autotune(grid, rad, [views[0]])
    assert o.tile_w * o.tile_h == 64 and 0 <= o.start_level < probes.levels
    a = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]]))
    b = _gpu_numpy(pt.probe_trace(grid, rad, [views[0]], o))
    same = (a["status"] == b["status"]) & (a["hit"] == b["hit"]).all(1)
    assert same.mean() > 1 - 1e-4

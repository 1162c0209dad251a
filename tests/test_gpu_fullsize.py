"""Parity at the workloads' full sizes, in the launch forms the benchmark uses, on sampled
rays the oracle computes one by one: the batched 64-view walk through one graph-captured
persistent launch, and the differentiable 16x16x8 grid of 256^2 maps (forward and
backward)."""
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


def test_batched_64_views_graph_launch_sampled():
    pt = _pt()
    scene, probes, views = workload("batched")
    assert len(views) == 64
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    res = pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_GRAPH))
    res = {k: v.cpu().numpy() for k, v in res.items()}
    og = oracle.Grid.from_probes(probes)
    rng = np.random.default_rng(11)
    off = 0
    o_all, d_all, sel = [], [], []
    for v in views:
        n = v.width * v.height
        pix = np.sort(rng.choice(n, 500, replace=False))
        o, d = oracle.view_rays(*v.as_tuple(), pixels=pix)
        o_all.append(o)
        d_all.append(d)
        sel.append(off + pix)
        off += n
    assert off == len(res["status"])
    orc = oracle.trace(og, np.concatenate(o_all), np.concatenate(d_all))
    assert_parity(compare(res, orc, sel=np.concatenate(sel)), "batched 64 views, 32k sampled rays")


@pytest.fixture(scope="module")
def diff_grid():
    pt = _pt()
    scene, probes, views = workload("diff", n_views=2)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    return scene, probes, views, grid, rad


def test_differentiable_grid_forward_sampled(diff_grid):
    pt = _pt()
    scene, probes, views, grid, rad = diff_grid
    assert probes.N == 256 and probes.n_probes == 2048 and views[0].width == 512
    res = {k: v.cpu().numpy() for k, v in pt.probe_trace(grid, rad, views).items()}
    rng = np.random.default_rng(12)
    n = views[0].width * views[0].height
    og = oracle.Grid.from_probes(probes)
    for vi, v in enumerate(views):
        pix = np.sort(rng.choice(n, 10000, replace=False))
        orc = oracle.trace_view(og, v.as_tuple(), pixels=pix)
        assert_parity(compare(res, orc, sel=vi * n + pix), f"diff grid view {vi}, 10k sampled rays")


def test_differentiable_grid_backward_sampled(diff_grid):
    # gradient only on sampled rays (zero elsewhere); compare every texel-channel touched
    pt = _pt()
    scene, probes, views, grid, rad = diff_grid
    v = views[0]
    n = v.width * v.height
    rng = np.random.default_rng(13)
    pix = np.sort(rng.choice(n, 20000, replace=False))
    og = oracle.Grid.from_probes(probes)
    orc = oracle.trace_view(og, v.as_tuple(), pixels=pix)
    res = {k: x.cpu().numpy() for k, x in pt.probe_trace(grid, rad, [v]).items()}
    s = compare(res, orc, sel=pix)
    g_s = rng.normal(size=(len(pix), 3)).astype(np.float32).astype(np.float64)
    g_s[s["disagree_idx"]] = 0.0
    g = np.zeros((n, 3), np.float32)
    g[pix] = g_s
    gg = torch.zeros((probes.n_probes, probes.N, probes.N, 3), device="cuda")
    pt.probe_trace_backward(grid, [v], torch.from_numpy(g).cuda(), gg)
    got = gg.cpu().numpy().reshape(-1, 3).astype(np.float64)
    ref = oracle.vjp(og, orc, g_s).reshape(-1, 3)
    wabs = oracle.vjp(og, orc, np.abs(g_s)).reshape(-1, 3)
    unit = dict(orc)
    unit["wts"] = (orc["wts"] != 0).astype(np.float64)
    gabs = oracle.vjp(og, unit, np.abs(g_s)).reshape(-1, 3)
    tol = 1e-5 * wabs + 1e-3 * gabs + 1e-8
    err = np.abs(got - ref)
    print(f"[grad] diff grid: touched {np.count_nonzero(ref)}, max err/tol {(err / tol).max():.3f}", flush=True)
    assert np.count_nonzero(ref) > 10000
    assert not (err > tol).any()

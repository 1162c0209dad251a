"""Gradient through the stored distances on the GPU (probe_trace_backward_distance,
probe_grid_set_distance, ProbeGeometryFn) against the oracle's vjp_distance.

Tolerance per texel:  |g_gpu - g_oracle| <= 1e-3 sum|contribution| + 1e-7, the sum over the
rays hitting that texel: the relative bound the forward allows on rgb.  (The FP32 motion of
the radiance sample loses digits where the hit point moves nearly radially as seen from the
probe and where the four taps' terms cancel; the device code built for the host measures
4e-4 at most, and 2e-4 on dt/dr for grazing roots.)  Left out on both sides (zero upstream
gradient): rays whose
classification differs between GPU and oracle (all inside the float margin, checked by the
forward parity tests), rays with an ill-conditioned hit distance (condition scale above
100 t, or a near-tangent root with dt/dr >= 100), rays
within the margin of switching between the entry-point hit and the root (dt/dr jumps from
0 there), and
rays whose radiance sample sits within 1e-4 texel of a texel-centre line or within 1e-5 of
the octahedral fold, where the sample's derivative jumps and FP32 may take the other side.
"""
import numpy as np
import pytest
import torch

import oracle
from conftest import workload
from parity import compare

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _setup(name="single", seed=0, **kw):
    pt = _pt()
    scene, probes, views = workload(name, **kw)
    grid = pt.ProbeGrid.from_probes(probes)
    rng = np.random.default_rng(seed)
    rad16 = rng.uniform(0.0, 1.0, size=(probes.n_probes, probes.N, probes.N, 3)).astype(np.float16)
    rad = torch.from_numpy(rad16).cuda()
    og = oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                     probes.scene_max, probes.distance, probes.normal, rad16.astype(np.float32))
    return pt, probes, views, grid, rad, og


def _rays(views):
    o_parts, d_parts = [], []
    for v in views:
        o, d = oracle.view_rays(*v.as_tuple())
        o_parts.append(o)
        d_parts.append(d)
    return np.concatenate(o_parts), np.concatenate(d_parts)


def _check(pt, probes, views, grid, rad, og, use_rgb=True, use_t=True, opts=None, nearest=False, coarse=None):
    """coarse: (coarse oracle grid, plane_off, ratio) of a two-level hierarchy (probes then
    only gives N; the gradient spans both levels, fine first)."""
    res = {k: v.cpu().numpy() for k, v in pt.probe_trace(grid, rad, views, opts).items()}
    o, d = _rays(views)
    orc = oracle.trace(og, o, d, nearest=nearest, coarse=coarse)
    Pf = og.distance.shape[0]
    position = (lambda p: og.probe_position(p) if p < Pf else coarse[0].probe_position(p - Pf))
    s = compare(res, orc)
    n = s["n"]
    hit = orc["status"] == oracle.HIT
    keep = np.ones(n, bool)
    keep[s["disagree_idx"]] = False
    # rays whose hit distance or its derivative FP32 cannot resolve to this tolerance: flagged
    # by the oracle, an entry crossing with a condition scale above 100 t, or a near-tangent
    # root (dt/dr = r / sqrt(r^2 - d_perp^2) >= 100)
    keep &= (orc["margin"] & oracle.MG_THIT) == 0
    keep &= ~hit | ((orc["tcond"] <= 100 * orc["t"]) & (orc["dtdr"] < 100))
    keep &= orc["kink"] == 0  # entry point vs root within the margin: dt/dr jumps there
    wts = orc["wts"]
    fx, fy = wts[:, 1] + wts[:, 3], wts[:, 2] + wts[:, 3]
    if not nearest:
        keep &= ~hit | (np.minimum(np.minimum(fx, 1 - fx), np.minimum(fy, 1 - fy)) > 1e-4)
        pos = np.zeros((n, 3))
        pos[hit] = np.stack([position(p) for p in orc["probe"][hit]])
        q = o + np.where(hit, orc["t"], 0.0)[:, None] * d - pos
        keep &= ~hit | (np.abs(q[:, 2]) > 1e-5 * np.abs(q).sum(1))
    rng = np.random.default_rng(7)
    grgb = rng.normal(size=(n, 3)).astype(np.float32) * keep[:, None] if use_rgb else None
    gt = rng.normal(size=n).astype(np.float32) * keep if use_t else None
    gg = torch.zeros((grid.P_total, probes.N, probes.N), dtype=torch.float32, device="cuda")
    pt.probe_trace_backward_distance(grid, rad, views,
                                     torch.from_numpy(grgb).cuda() if use_rgb else None,
                                     torch.from_numpy(gt).cuda() if use_t else None, gg, opts)
    got = gg.cpu().numpy().astype(np.float64)
    g64 = lambda a: None if a is None else a.astype(np.float64)
    grids = (og, coarse[0]) if coarse else og
    ref = oracle.vjp_distance(grids, orc, grad_rgb=g64(grgb), grad_t=g64(gt))
    # sum of |contribution| per texel
    absd = dict(orc)
    absd["dtdr"] = np.abs(orc["dtdr"])
    absd["drgbdt"] = np.abs(orc["drgbdt"])
    mag = oracle.vjp_distance(grids, absd, grad_rgb=None if grgb is None else np.abs(g64(grgb)),
                              grad_t=None if gt is None else np.abs(g64(gt)))
    err = np.abs(got - ref)
    tol = 1e-3 * mag + 1e-7
    bad = err > tol
    print(f"[geo grad] n={n} kept={keep.mean():.4f} disagree={s['disagree']} nonzero={np.count_nonzero(ref)} "
          f"max_err/tol={(err / tol).max():.3f}", flush=True)
    assert not bad.any(), (np.argwhere(bad)[:10], err[bad][:10], tol[bad][:10])
    return got, ref


def test_distance_adjoint_matches_oracle():
    pt, probes, views, grid, rad, og = _setup(size=(240, 135))
    got, ref = _check(pt, probes, views, grid, rad, og)
    assert np.count_nonzero(ref) > 5000


def test_distance_adjoint_persistent_two_views_t_only_and_rgb_only():
    pt, probes, views, grid, rad, og = _setup("diff", N=64, levels=4, n_views=2, size=(96, 80))
    opts = pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)
    _check(pt, probes, views, grid, rad, og, opts=opts)
    got_t, ref_t = _check(pt, probes, views, grid, rad, og, use_rgb=False)
    got_c, ref_c = _check(pt, probes, views, grid, rad, og, use_t=False)
    assert np.count_nonzero(ref_t) > 1000 and np.count_nonzero(ref_c) > 1000


def test_distance_adjoint_per_texel_scatter():
    # the single-channel per-texel reduction (kept for grids of 2^32 - 1 texels or more),
    # forced: the same oracle tolerance as the LDS merge
    pt, probes, views, grid, rad, og = _setup("diff", N=64, levels=4, n_views=2, size=(96, 80))
    _check(pt, probes, views, grid, rad, og, opts=pt.trace_opts(flags=pt.PT_FLAG_SCATTER_PER_TEXEL))
    _check(pt, probes, views, grid, rad, og,
           opts=pt.trace_opts(flags=pt.PT_FLAG_SCATTER_PER_TEXEL | pt.PT_FLAG_PERSISTENT))


def test_nearest_radiance_does_not_move_with_distance():
    pt, probes, views, grid, rad, og = _setup("tiny")
    opts = pt.trace_opts(flags=pt.PT_FLAG_NEAREST)
    rays = views[0].width * views[0].height
    gg = torch.zeros((probes.n_probes, probes.N, probes.N), device="cuda")
    pt.probe_trace_backward_distance(grid, rad, views[:1], torch.ones((rays, 3), device="cuda"), None, gg, opts)
    assert torch.count_nonzero(gg).item() == 0
    _check(pt, probes, views[:1], grid, rad, og, opts=opts, nearest=True)


def test_set_distance_equals_a_fresh_grid():
    pt, probes, views, grid, rad, og = _setup("tiny")
    rng = np.random.default_rng(9)
    d2 = (probes.distance * rng.uniform(0.95, 1.05, size=probes.distance.shape)).astype(np.float32)
    grid.set_distance(torch.from_numpy(d2).cuda())
    fresh = pt.ProbeGrid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                         probes.scene_max, torch.from_numpy(d2).cuda(),
                         torch.from_numpy(probes.normal.view(np.float16)).cuda())
    for l in range(probes.levels):
        assert torch.equal(grid.read_level(l), fresh.read_level(l)), l
    a = pt.probe_trace(grid, rad, views[:1])
    b = pt.probe_trace(fresh, rad, views[:1])
    for k in ("rgb", "status", "hit"):
        assert torch.equal(a[k], b[k]), k


def test_geometry_autograd_function():
    # loss on depth and colour; the autograd gradients equal the direct adjoint calls
    pt, probes, views, grid, rad, og = _setup("tiny")
    dist = torch.from_numpy(probes.distance.copy()).cuda().requires_grad_(True)
    master = rad.float().clone().requires_grad_(True)
    rgb, t = pt.ProbeGeometryFn.apply(dist, master, grid, views[:1])
    hit = torch.isfinite(t)
    loss = (torch.where(hit, t, torch.zeros_like(t)) ** 2).sum() + (rgb ** 2).sum()
    loss.backward()
    gt = torch.where(hit, 2 * t, torch.zeros_like(t)).contiguous()
    grgb = (2 * rgb).detach().contiguous()
    gd = torch.zeros_like(dist)
    pt.probe_trace_backward_distance(grid, rad, views[:1], grgb, gt, gd)
    gm = torch.zeros_like(master)
    pt.probe_trace_backward(grid, views[:1], grgb, gm)
    torch.testing.assert_close(dist.grad, gd, rtol=1e-5, atol=1e-6)
    torch.testing.assert_close(master.grad, gm, rtol=1e-5, atol=1e-6)
    assert torch.count_nonzero(dist.grad).item() > 300


def test_distance_adjoint_two_level_hierarchy():
    # the distance adjoint over both levels of a hierarchy (the city block at reduced size):
    # hits on coarse probes add into the coarse block of the gradient, after the fine one
    pt = _pt()
    scene, tl, views = workload("large_small")
    rng = np.random.default_rng(3)
    rads = [rng.uniform(0.0, 1.0, size=(ps.n_probes, ps.N, ps.N, 3)).astype(np.float16) for ps in (tl.fine, tl.coarse)]
    grid = pt.ProbeGrid.from_two_level(tl)
    rad = torch.from_numpy(np.concatenate(rads)).cuda()
    og, cg = (oracle.Grid.from_probes(ps, radiance=r.astype(np.float32)) for ps, r in zip((tl.fine, tl.coarse), rads))
    got, ref = _check(pt, tl.fine, views, grid, rad, og, coarse=(cg, tl.plane_off, tl.ratio))
    Pf = tl.fine.n_probes
    assert np.count_nonzero(ref[:Pf]) > 500 and np.count_nonzero(ref[Pf:]) > 0

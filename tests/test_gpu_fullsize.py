"""Parity at the workloads' full sizes, in the launch forms the benchmark uses, on sampled
rays the oracle computes one by one: the batched 64-view walk through one graph-captured
persistent launch, and the differentiable 16x16x8 grid of 256^2 maps (forward and
backward; its 32 views in the training step's persistent launch with both radiance
adjoints)."""
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


def test_differentiable_grid_all_views_both_adjoints_sampled(diff_grid):
    # the training configuration: all 32 views of 512^2 in one persistent launch, forward
    # and both radiance adjoints (recomputing, and from the forward's stored hits), with the
    # upstream gradient on 1,000 sampled rays per view, every touched texel-channel held to
    # the oracle's VJP
    import synth
    pt = _pt()
    scene, probes, views2, grid, rad = diff_grid
    vc = synth.CONFIGS["diff"]["views"]
    views = synth.make_views(scene, vc["seed"], vc["n"], vc["width"], vc["height"])
    assert len(views) == 32 and views[0].width == 512
    opts = pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT)
    dev = pt.probe_trace(grid, rad, views, opts)
    res = {k: x.cpu().numpy() for k, x in dev.items()}
    n = views[0].width * views[0].height
    rng = np.random.default_rng(14)
    og = oracle.Grid.from_probes(probes)
    o_all, d_all, sel = [], [], []
    for vi, v in enumerate(views):
        pix = np.sort(rng.choice(n, 1000, replace=False))
        o, d = oracle.view_rays(*v.as_tuple(), pixels=pix)
        o_all.append(o)
        d_all.append(d)
        sel.append(vi * n + pix)
    sel = np.concatenate(sel)
    orc = oracle.trace(og, np.concatenate(o_all), np.concatenate(d_all))
    s = compare(res, orc, sel=sel)
    assert_parity(s, "diff grid, 32 views persistent, 32k sampled rays")
    g_s = rng.normal(size=(len(sel), 3)).astype(np.float32).astype(np.float64)
    g_s[s["disagree_idx"]] = 0.0
    # a ray whose hit distance is ill-conditioned (flagged by the oracle, or a condition scale
    # above 100 t, or a near-tangent root with dt/dr >= 100)
    # has an equally ill-conditioned sample direction, so its bilinear weights are not held
    # to the FP32 bound: it gets no upstream gradient (as in the distance adjoint's test)
    hit_o = orc["status"] == oracle.HIT
    ill = ((orc["margin"] & oracle.MG_THIT) != 0) | (hit_o & ((orc["tcond"] > 100 * orc["t"]) | (orc["dtdr"] >= 100)))
    g_s[ill] = 0.0
    print(f"[grad] diff grid 32 views: {int(ill.sum())} rays with an ill-conditioned hit distance left out",
          flush=True)
    g = np.zeros((32 * n, 3), np.float32)
    g[sel] = g_s
    g_dev = torch.from_numpy(g).cuda()
    shape = (probes.n_probes, probes.N, probes.N, 3)
    ref = oracle.vjp(og, orc, g_s).reshape(-1, 3)
    wabs = oracle.vjp(og, orc, np.abs(g_s)).reshape(-1, 3)
    # FP32 bound on a ray's bilinear weights: the sample direction q = (X - O) + t w loses
    # digits where the hit point lies much closer to the probe than the camera does, by
    # (|X - O| + t) / |q|; in texels (N/2 per unit of the map) that is 4 2^-24 (N/2) times
    # the ratio, and never below the forward's 1e-3
    o, d = np.concatenate(o_all), np.concatenate(d_all)
    hit = orc["status"] == oracle.HIT
    pos = np.zeros_like(o)
    pos[hit] = np.stack([og.probe_position(p) for p in orc["probe"][hit]])
    tt = np.where(hit, orc["t"], 0.0)
    q = o + tt[:, None] * d - pos
    ratio = np.where(hit, (np.linalg.norm(o - pos, axis=1) + tt) / np.maximum(np.linalg.norm(q, axis=1), 1e-30), 0.0)
    wbound = np.maximum(1e-3, 4 * 2.0 ** -24 * (probes.N / 2) * ratio)
    unit = dict(orc)
    unit["wts"] = (orc["wts"] != 0).astype(np.float64)
    gabs = oracle.vjp(og, unit, np.abs(g_s) * wbound[:, None]).reshape(-1, 3)
    tol = 1e-5 * wabs + gabs + 1e-8
    for label in ("recompute", "stored hits"):
        gg = torch.zeros(shape, device="cuda")
        if label == "recompute":
            pt.probe_trace_backward(grid, views, g_dev, gg, opts)
        else:
            pt.probe_trace_backward_hits(grid, views, dev["hit"], dev["t"], g_dev, gg, opts)
        err = np.abs(gg.cpu().numpy().reshape(-1, 3).astype(np.float64) - ref)
        print(f"[grad] diff grid 32 views {label}: touched {np.count_nonzero(ref)}, "
              f"max err/tol {(err / tol).max():.3f}", flush=True)
        if (err > tol).any():
            # the worst texel-channel and the rays that reach it
            wi = int(np.argmax((err / tol).reshape(-1)))
            tex, ch = divmod(wi, 3)
            err, tol, ref, wabs, gabs = (a.reshape(-1) for a in (err, tol, ref, wabs, gabs))
            hit = orc["status"] == oracle.HIT
            flat = orc["probe"].astype(np.int64)[:, None] * probes.N ** 2 + orc["taps"].astype(np.int64)
            rays = np.nonzero(hit[:, None] & (flat == tex) & (orc["wts"] != 0))
            print(f"[grad] worst texel {tex} ch {ch}: got-ref {err[wi]:.3e} tol {tol[wi]:.3e} ref {ref[wi]:.3e} "
                  f"wabs {wabs[wi]:.3e} gabs {gabs[wi]:.3e}", flush=True)
            for ri, k in list(zip(*rays))[:40]:
                pos = og.probe_position(orc["probe"][ri])
                q = o[ri] + orc["t"][ri] * d[ri] - pos
                print(f"  ray {ri} tap {k} w {orc['wts'][ri, k]:.6f} g {g_s[ri, ch]:+.4f} t {orc['t'][ri]:.4f} "
                      f"|X-O| {np.linalg.norm(o[ri] - pos):.4f} |q| {np.linalg.norm(q):.4f} "
                      f"margin {int(orc['margin'][ri])} score {orc['score'][ri]:.2e}", flush=True)
        assert not (err > tol).any(), label
    assert np.count_nonzero(ref) > 100000

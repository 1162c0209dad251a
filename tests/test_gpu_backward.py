"""Radiance adjoint on the GPU (probe_trace_backward, ProbeTraceFn) against the oracle.

Tolerance per texel-channel:  |g_gpu - g_oracle| <= 1e-5 sum|w g| + 1e-3 sum|g| + 1e-8,
where the sums run over the (ray, tap) pairs that touch that texel: the first term is
FP32 atomic accumulation order, the second the single-precision bilinear weights (the
same 1e-3 the forward allows on rgb).  Rays on which GPU and oracle disagree (all inside
the float margin, checked by the forward parity tests) are given zero gradient on both
sides.
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


def _setup(name, **kw):
    pt = _pt()
    scene, probes, views = workload(name, **kw)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    return pt, scene, probes, views, grid, rad


def _check_grad(pt, probes, grid, rad, views, seed=0, nearest=False, flags=0):
    og = oracle.Grid.from_probes(probes)
    flags |= pt.PT_FLAG_NEAREST if nearest else 0
    opts = pt.trace_opts(flags=flags) if flags else None
    dev = pt.probe_trace(grid, rad, views, opts)
    res = {k: v.cpu().numpy() for k, v in dev.items()}
    o_parts, d_parts = [], []
    for v in views:
        o, d = oracle.view_rays(*v.as_tuple())
        o_parts.append(o)
        d_parts.append(d)
    orc = oracle.trace(og, np.concatenate(o_parts), np.concatenate(d_parts), nearest=nearest)
    s = compare(res, orc)
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(s["n"], 3)).astype(np.float32)
    g[s["disagree_idx"]] = 0.0
    gg = torch.zeros((probes.n_probes, probes.N, probes.N, 3), dtype=torch.float32, device="cuda")
    pt.probe_trace_backward(grid, views, torch.from_numpy(g).cuda(), gg, opts)
    got = gg.cpu().numpy().astype(np.float64)
    ref = oracle.vjp(og, orc, g.astype(np.float64))
    wabs = oracle.vjp(og, orc, np.abs(g).astype(np.float64))
    # sum |g| over the (ray, tap) pairs per texel: vjp with unit weights
    unit = dict(orc)
    unit["wts"] = (orc["wts"] != 0).astype(np.float64)
    gabs = oracle.vjp(og, unit, np.abs(g).astype(np.float64))
    tol = 1e-5 * wabs + 1e-3 * gabs + 1e-8
    # the same adjoint from the forward's stored (probe, texel) and t
    gh = torch.zeros_like(gg)
    pt.probe_trace_backward_hits(grid, views, dev["hit"], dev["t"], torch.from_numpy(g).cuda(), gh, opts)
    for label, x in (("recompute", got), ("stored hits", gh.cpu().numpy().astype(np.float64))):
        err = np.abs(x - ref)
        bad = err > tol
        print(f"[grad {label}] n={s['n']} disagree={s['disagree']} max_err={err.max():.3e} "
              f"max_err/tol={(err / tol).max():.3f} nonzero={np.count_nonzero(ref)}", flush=True)
        assert not bad.any(), (label, np.argwhere(bad)[:10])
    assert np.count_nonzero(ref) > 1000
    return got, ref


def test_backward_matches_oracle_vjp_tiny():
    pt, scene, probes, views, grid, rad = _setup("tiny")
    _check_grad(pt, probes, grid, rad, views[:1])


def test_backward_matches_oracle_vjp_room_views():
    pt, scene, probes, views, grid, rad = _setup("diff", N=64, levels=4, n_views=2, size=(96, 80))
    _check_grad(pt, probes, grid, rad, views)


def test_backward_nearest_texel_radiance():
    # one tap per HIT ray: the gradient of a texel is the sum of its rays' grad_rgb
    pt, scene, probes, views, grid, rad = _setup("diff", N=64, levels=4, n_views=2, size=(96, 80))
    _check_grad(pt, probes, grid, rad, views, nearest=True)


def test_backward_persistent_launch_over_uneven_views():
    # the adjoint as one persistent launch over the tiles of all views (the training loop's form)
    import dataclasses
    pt, scene, probes, views, grid, rad = _setup("diff", N=64, levels=4, n_views=3, size=(96, 80))
    views = [views[0], dataclasses.replace(views[1], width=53, height=41), dataclasses.replace(views[2], width=120)]
    _check_grad(pt, probes, grid, rad, views, flags=pt.PT_FLAG_PERSISTENT)


def test_backward_accumulates():
    pt, scene, probes, views, grid, rad = _setup("tiny")
    rays = views[0].width * views[0].height
    g = torch.ones((rays, 3), device="cuda")
    a = torch.zeros((probes.n_probes, probes.N, probes.N, 3), device="cuda")
    pt.probe_trace_backward(grid, views[:1], g, a)
    b = a.clone()
    pt.probe_trace_backward(grid, views[:1], g, b)
    torch.testing.assert_close(b, 2 * a, rtol=1e-5, atol=1e-6)
    # the total equals 3 x number of HIT rays (bilinear weights sum to one)
    st = pt.probe_trace(grid, rad, views[:1])["status"]
    assert abs(a.sum().item() - 3 * (st == 1).sum().item()) < 1e-2 * max(1, (st == 1).sum().item())


def test_dot_product_identity_on_gpu():
    pt, scene, probes, views, grid, rad = _setup("tiny")
    gen = torch.Generator(device="cpu").manual_seed(5)
    x = torch.rand(rad.shape, generator=gen).to(torch.float16).cuda()
    rays = views[0].width * views[0].height
    y = torch.randn((rays, 3), generator=gen).cuda()
    jx = pt.probe_trace(grid, x, views[:1])["rgb"]
    jty = torch.zeros(rad.shape, dtype=torch.float32, device="cuda")
    pt.probe_trace_backward(grid, views[:1], y, jty)
    lhs = (jx.double() * y.double()).sum().item()
    rhs = (x.double() * jty.double()).sum().item()
    assert abs(lhs - rhs) <= 1e-4 * max(1.0, abs(lhs))


def test_autograd_function_and_finite_differences():
    pt, scene, probes, views, grid, rad = _setup("tiny")
    master = rad.float().clone().requires_grad_(True)
    target = torch.rand((views[0].width * views[0].height, 3), device="cuda")
    rgb = pt.ProbeTraceFn.apply(master, grid, views[:1])
    loss = ((rgb - target) ** 2).sum()
    loss.backward()
    g = master.grad.clone()
    # the function's gradient is probe_trace_backward of 2 (rgb - target)
    ref = torch.zeros_like(g)
    pt.probe_trace_backward(grid, views[:1], (2 * (rgb - target)).detach().contiguous(), ref)
    torch.testing.assert_close(g, ref, rtol=1e-5, atol=1e-6)
    # central differences on FP16 storage at the most influential texel-channels
    flat = g.abs().flatten()
    picks = torch.topk(flat, 6).indices.tolist()
    h = 2.0 ** -6
    base = torch.round(master.detach() * 256) / 256  # h-steps exact in FP16
    for idx in picks:
        vals = []
        for s in (1, -1):
            m = base.clone().flatten()
            m[idx] += s * h
            r = pt.probe_trace(grid, m.view_as(base).to(torch.float16), views[:1])["rgb"]
            vals.append(((r.double() - target.double()) ** 2).sum().item())
        fd = (vals[0] - vals[1]) / (2 * h)
        r0 = pt.probe_trace(grid, base.to(torch.float16), views[:1])["rgb"]
        gb = torch.zeros_like(g)
        pt.probe_trace_backward(grid, views[:1], (2 * (r0 - target)).contiguous(), gb)
        an = gb.flatten()[idx].item()
        assert abs(fd - an) <= 2e-3 * max(1.0, abs(an)), (idx, fd, an)


def test_adam_reduces_loss_on_small_differentiable_room():
    pt = _pt()
    scene, probes, views = workload("diff", N=32, levels=3, n_views=4, size=(64, 64))
    target_scene = scene.with_albedos(4)
    import synth
    target_probes = synth.bake(target_scene, probes.N, probes.levels)
    grid = pt.ProbeGrid.from_probes(probes)
    trad = torch.from_numpy(target_probes.radiance.view(np.float16).copy()).cuda()
    with torch.no_grad():
        target = pt.probe_trace(grid, trad, views)["rgb"]
    from paper_2507_14624_amd.differentiable import RadianceFit
    fit = RadianceFit(grid, views, target, init=0.5, lr=1e-2)
    losses = [fit.step().item() for _ in range(30)]
    assert losses[-1] < 0.5 * losses[0], losses
    # the helper's loss is the mean squared error of the traced FP16-rounded master
    rgb = pt.probe_trace(grid, fit.master.detach().to(torch.float16), views)["rgb"]
    torch.testing.assert_close(fit.loss().detach(), ((rgb - target) ** 2).mean(), rtol=1e-6, atol=0)


@pytest.mark.parametrize("name,kw,flags", [("single", dict(size=(240, 135)), 0),
                                           ("diff", dict(N=64, levels=4, n_views=3, size=(96, 80)), 0),
                                           ("tiny", {}, 4),
                                           ("diff", dict(N=64, levels=4, n_views=3, size=(96, 80)), 128),
                                           ("single", dict(size=(240, 135)), 128 | 1)])
def test_backward_from_stored_hits_equals_recompute(name, kw, flags):
    # the adjoint from the forward's (probe, texel) and t outputs rebuilds every sample
    # direction exactly: the same gradient as the recomputing adjoint up to atomic order
    pt, scene, probes, views, grid, rad = _setup(name, **kw)
    opts = pt.trace_opts(flags=flags) if flags else None
    res = pt.probe_trace(grid, rad, views, opts)
    rays = res["rgb"].shape[0]
    gen = torch.Generator(device="cpu").manual_seed(2)
    gr = torch.randn((rays, 3), generator=gen).cuda()
    shape = (probes.n_probes, probes.N, probes.N, 3)
    a = torch.zeros(shape, device="cuda")
    b = torch.zeros(shape, device="cuda")
    pt.probe_trace_backward(grid, views, gr, a, opts)
    pt.probe_trace_backward_hits(grid, views, res["hit"], res["t"], gr, b, opts)
    torch.testing.assert_close(b, a, rtol=1e-5, atol=1e-5)
    assert torch.count_nonzero(a).item() > 1000


def test_autograd_with_stored_hits():
    pt, scene, probes, views, grid, rad = _setup("tiny")
    master = rad.float().clone().requires_grad_(True)
    target = torch.zeros((views[0].width * views[0].height, 3), device="cuda")
    grads = []
    for keep in (False, True):
        master.grad = None
        rgb = pt.ProbeTraceFn.apply(master, grid, views[:1], None, keep)
        ((rgb - target) ** 2).mean().backward()
        grads.append(master.grad.clone())
    torch.testing.assert_close(grads[1], grads[0], rtol=1e-5, atol=1e-7)


def test_stored_hits_outside_the_grid_add_nothing():
    # hit entries that are no forward output (probe beyond the grid, texel beyond the map)
    # contribute nothing and write nowhere: the same gradient as with those rays marked MISS
    pt, scene, probes, views, grid, rad = _setup("tiny")
    res = pt.probe_trace(grid, rad, views[:1])
    rays = res["rgb"].shape[0]
    gen = torch.Generator(device="cpu").manual_seed(8)
    gr = torch.randn((rays, 3), generator=gen).cuda()
    hit = res["hit"].clone()
    bad = torch.arange(0, rays, 97, device="cuda")
    N2 = probes.N * probes.N
    vals = torch.tensor([[probes.n_probes, 0], [probes.n_probes + 5, 3], [2 ** 30, 7], [0, N2], [1, N2 + 11],
                         [0, -5]], dtype=torch.int32, device="cuda")
    hit[bad] = vals[torch.arange(len(bad), device="cuda") % len(vals)]
    miss = res["hit"].clone()
    miss[bad] = -1
    shape = (probes.n_probes, probes.N, probes.N, 3)
    a = torch.zeros(shape, device="cuda")
    b = torch.zeros(shape, device="cuda")
    pt.probe_trace_backward_hits(grid, views[:1], hit, res["t"], gr, a)
    pt.probe_trace_backward_hits(grid, views[:1], miss, res["t"], gr, b)
    torch.testing.assert_close(a, b, rtol=1e-5, atol=1e-5)
    assert torch.count_nonzero(b).item() > 1000


def test_stored_hit_adjoint_with_every_tap_of_a_wave_distinct():
    # One 8x8 tile (one wavefront) whose 64 rays each name a different probe: its 256 taps are
    # 256 distinct texels, the most a wave's merge table ever holds; then the same tile with
    # every ray on one probe and texel (one texel per tap position, heavy merging).  The
    # expected gradient is the plain definition: for each ray, the 4 bilinear taps at the
    # direction X - O + t w of its probe, weighted by the upstream gradient.
    pt, scene, probes, views, grid, rad = _setup("single", size=(64, 64))
    import synth
    v = synth.make_views(scene, 41, 1, 8, 8)[0]
    og = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*v.as_tuple())
    N = probes.N
    rng = np.random.default_rng(5)
    g = rng.normal(size=(64, 3)).astype(np.float32)
    for probes_of_rays in (np.arange(64) * 3 % probes.n_probes, np.full(64, 77)):
        t = rng.uniform(0.5, 3.0, 64).astype(np.float32)
        hit = np.stack([probes_of_rays, rng.integers(0, N * N, 64)], 1).astype(np.int32)
        want = np.zeros((probes.n_probes, N * N, 3))
        for i in range(64):
            p = int(hit[i, 0])
            q = o[i] - og.probe_position(p) + float(t[i]) * d[i]
            u, vv = oracle.oct_encode(q)
            idx, wt = oracle.bilinear_taps(u, vv, N)
            for k in range(4):
                want[p, idx[k]] += wt[k] * g[i].astype(np.float64)
        gh = torch.zeros((probes.n_probes, N, N, 3), device="cuda")
        pt.probe_trace_backward_hits(grid, [v], torch.from_numpy(hit).cuda(), torch.from_numpy(t).cuda(),
                                     torch.from_numpy(g).cuda(), gh)
        got = gh.cpu().numpy().reshape(probes.n_probes, N * N, 3).astype(np.float64)
        assert np.count_nonzero(want) > 0
        assert np.abs(got - want).max() <= 1e-3 * np.abs(g).max(), np.abs(got - want).max()
        assert np.array_equal(got != 0, want != 0)


def test_per_texel_scatter_matches_oracle_vjp():
    # the reduction the library keeps for grids of 2^32 - 1 texels or more, forced on a
    # small grid: the same tolerance against the oracle's VJP as the default LDS merge
    pt, scene, probes, views, grid, rad = _setup("single", size=(160, 90))
    _check_grad(pt, probes, grid, rad, views, flags=pt.PT_FLAG_SCATTER_PER_TEXEL)
    _check_grad(pt, probes, grid, rad, views, flags=pt.PT_FLAG_SCATTER_PER_TEXEL | pt.PT_FLAG_PERSISTENT)


def test_per_texel_scatter_equals_lds_merge():
    # both reductions of the stored-hit adjoint on the differentiable grid, where an 8x8 tile
    # touches ~100 distinct texels: the same sums up to FP32 summation order
    pt, scene, probes, views, grid, rad = _setup("diff", N=64, levels=4, n_views=3, size=(128, 96))
    res = pt.probe_trace(grid, rad, views)
    rays = res["rgb"].shape[0]
    gen = torch.Generator(device="cpu").manual_seed(5)
    gr = torch.randn((rays, 3), generator=gen).cuda()
    shape = (probes.n_probes, probes.N, probes.N, 3)
    a = torch.zeros(shape, device="cuda")
    b = torch.zeros(shape, device="cuda")
    pt.probe_trace_backward_hits(grid, views, res["hit"], res["t"], gr, a, None)
    pt.probe_trace_backward_hits(grid, views, res["hit"], res["t"], gr, b,
                                 pt.trace_opts(flags=pt.PT_FLAG_SCATTER_PER_TEXEL))
    torch.testing.assert_close(b, a, rtol=1e-5, atol=1e-5)
    assert torch.count_nonzero(a).item() > 1000

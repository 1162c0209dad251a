"""pt_adam_step against torch.optim.Adam (its single-tensor form, the textbook update) on
the GPU: parameters and moments over several steps, with and without weight decay, the
FP16 output equal to the parameters' rounding bit for bit, misaligned buffers (the
one-element path) equal to aligned ones, and RadianceFit with the fused step against
RadianceFit with torch's Adam."""
import numpy as np
import pytest
import torch

from conftest import workload

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


@pytest.mark.parametrize("wd", [0.0, 1e-2])
def test_adam_step_matches_torch_adam(wd):
    pt = _pt()
    gen = torch.Generator(device="cpu").manual_seed(5)
    n = 1_000_003  # not a multiple of 4: the last 3 elements take the one-element path
    p0 = torch.rand(n, generator=gen).cuda()
    ref = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd, foreach=False,
                           fused=False)
    p = p0.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    h = torch.empty(n, dtype=torch.float16, device="cuda")
    for step in range(1, 6):
        g = torch.randn(n, generator=gen).cuda()
        ref.grad = g.clone()
        opt.step()
        pt.adam_step(p, g, m, v, h, step, 1e-2, (0.9, 0.999), 1e-8, wd)
        st = opt.state[ref]
        torch.testing.assert_close(m, st["exp_avg"], rtol=1e-6, atol=1e-7)
        torch.testing.assert_close(v, st["exp_avg_sq"], rtol=1e-6, atol=1e-9)
        torch.testing.assert_close(p, ref.detach(), rtol=1e-6, atol=1e-7)
        assert torch.equal(h, p.to(torch.float16)), step


def test_adam_step_misaligned_buffers_and_no_half_output():
    pt = _pt()
    gen = torch.Generator(device="cpu").manual_seed(6)
    n = 4099
    base = [torch.rand(n + 1, generator=gen).cuda() for _ in range(2)]
    g = torch.randn(n + 1, generator=gen).cuda()
    # aligned run
    pa, ma, va = base[0][:n].clone(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    ha = torch.empty(n, dtype=torch.float16, device="cuda")
    # misaligned run: every buffer starts one element into its allocation
    pm = base[1].clone()
    pm[1:] = base[0][:n]
    mm, vm = torch.zeros(n + 1, device="cuda"), torch.zeros(n + 1, device="cuda")
    hm = torch.empty(n + 1, dtype=torch.float16, device="cuda")
    for step in (1, 2, 3):
        pt.adam_step(pa, g[:n].contiguous(), ma, va, ha, step, 3e-3)
        gm = torch.empty(n + 1, device="cuda")
        gm[1:] = g[:n]
        pt.adam_step(pm[1:], gm[1:], mm[1:], vm[1:], hm[1:], step, 3e-3)
    assert torch.equal(pa, pm[1:]) and torch.equal(ma, mm[1:]) and torch.equal(va, vm[1:])
    assert torch.equal(ha, hm[1:])
    # no FP16 output: the same update
    pn, mn, vn = base[0][:n].clone(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for step in (1, 2, 3):
        pt.adam_step(pn, g[:n].contiguous(), mn, vn, None, step, 3e-3)
    assert torch.equal(pn, pa)


def test_adam_step_rejects_bad_arguments():
    pt = _pt()
    p = torch.zeros(8, device="cuda")
    for kw in (dict(step=0), dict(lr=-1.0), dict(betas=(1.0, 0.999)), dict(betas=(0.9, 1.0)), dict(eps=float("nan"))):
        args = dict(step=1, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
        args.update(kw)
        with pytest.raises(pt.ProbeTraceError):
            pt.adam_step(p, p.clone(), p.clone(), p.clone(), None, args["step"], args["lr"], args["betas"],
                         args["eps"])
    with pytest.raises(pt.ProbeTraceError):
        pt.adam_step(p, torch.zeros(7, device="cuda"), p.clone(), p.clone(), None, 1, 1e-3)


def test_radiance_fit_fused_step_matches_torch_adam():
    pt = _pt()
    from paper_2507_14624_amd.differentiable import RadianceFit
    scene, probes, views = workload("tiny")
    grid = pt.ProbeGrid.from_probes(probes)
    trad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    target = pt.probe_trace(grid, trad, views[:1])["rgb"]
    # The two fits' gradients differ in the order of their FP32 atomics, and Adam turns a
    # texel's near-zero gradient into a full-size step whatever its last digits, so the
    # masters are not compared texel by texel: the loss trajectories are (they sum over
    # every ray), and the fused step's FP16 storage must be the master's rounding.
    fits = [RadianceFit(grid, views[:1], target, init=0.3, lr=2e-2, optimizer=o) for o in ("fused", "torch")]
    losses = [[], []]
    for _ in range(4):
        for f, l in zip(fits, losses):
            l.append(f.step().item())
        assert torch.equal(fits[0].storage, fits[0].master.detach().to(torch.float16))
    np.testing.assert_allclose(losses[0], losses[1], rtol=1e-5)
    assert losses[0][-1] < 0.7 * losses[0][0]

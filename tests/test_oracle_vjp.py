"""Pins of the oracle's radiance adjoint and of its float-margin flag.

The forward trace is exactly linear in the stored radiance once the geometry is fixed
(the hit test never reads radiance), so its adjoint is fixed by three facts checked
here: the dot-product identity <J x, y> = <x, J^T y>, exact central differences of a
quadratic loss, and a zero loss when the radiance equals the target.
"""
import numpy as np
import pytest

import oracle
from conftest import workload, fp16_bits


def _setup(name="tiny", pixels=None, **kw):
    scene, probes, views = workload(name, **kw)
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple(), pixels=pixels)
    return scene, probes, g, o, d


def test_dot_product_identity():
    scene, probes, g, o, d = _setup()
    rng = np.random.default_rng(20)
    r = oracle.trace(g, o, d)
    x = rng.uniform(-1, 1, size=g.radiance.shape).astype(np.float32)
    y = rng.uniform(-1, 1, size=(len(o), 3))
    g.set_radiance(x)
    rx = oracle.trace(g, o, d)  # J x (background 0 keeps the map linear)
    lhs = float(np.sum(rx["rgb"] * y))
    jt = oracle.vjp(g, r, y)
    rhs = float(np.sum(x.astype(np.float64) * jt))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    g.set_radiance(probes.radiance)


def test_central_differences_match_vjp():
    # loss = sum (rgb - target)^2 is quadratic in the radiance, so central differences with
    # a step exactly representable in FP16 storage are exact up to rounding
    scene, probes, g, o, d = _setup(pixels=np.arange(0, 128 * 128, 3))
    rng = np.random.default_rng(21)
    # radiance on a 2^-8 grid in [0, 1): base and base +- 2^-6 are all exact in FP16
    base = np.round(probes.radiance.view(np.float16).astype(np.float64) * 256) / 256
    g.set_radiance(fp16_bits(base))
    r0 = oracle.trace(g, o, d)
    target = rng.uniform(0, 1, size=(len(o), 3))
    grad = oracle.vjp(g, r0, 2.0 * (r0["rgb"] - target))
    h = 2.0 ** -6
    # texels actually sampled by the rays, plus one never sampled
    hitp = r0["probe"][r0["status"] == oracle.HIT]
    taps = r0["taps"][r0["status"] == oracle.HIT]
    picks = [(int(hitp[i]), int(taps[i, 0])) for i in rng.choice(len(hitp), 12, replace=False)]
    unseen = np.argwhere(grad.reshape(grad.shape[0], -1, 3).sum(-1) == 0)
    picks.append((int(unseen[0, 0]), int(unseen[0, 1])))
    N = probes.N
    for p, k in picks:
        for c in range(3):
            vals = []
            for s in (+1, -1):
                rad = base.copy()
                rad[p, k // N, k % N, c] += s * h
                g.set_radiance(fp16_bits(rad))
                assert rad[p, k // N, k % N, c] == g.radiance[p, k // N, k % N, c]  # the step is exact in FP16
                rr = oracle.trace(g, o, d)
                assert np.array_equal(rr["status"], r0["status"])  # geometry held fixed
                vals.append(np.sum((rr["rgb"] - target) ** 2))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grad[p, k // N, k % N, c]) <= 1e-9 * max(1.0, abs(fd))
    g.set_radiance(probes.radiance)


def test_zero_loss_at_target_and_gradient_vanishes():
    scene, probes, g, o, d = _setup()
    r = oracle.trace(g, o, d)
    grad = oracle.vjp(g, r, 2.0 * (r["rgb"] - r["rgb"]))
    assert np.all(grad == 0)


def test_vjp_duplicate_taps_accumulate():
    # every HIT ray spreads exactly its own gradient over its taps (weights sum to 1)
    scene, probes, g, o, d = _setup()
    r = oracle.trace(g, o, d)
    y = np.ones((len(o), 3))
    jt = oracle.vjp(g, r, y)
    assert abs(jt.sum() - 3.0 * (r["status"] == oracle.HIT).sum()) < 1e-6


def _rounded_rays(o, d):
    """The same rays with origin and direction rounded to FP32 (a perturbation of the size
    a single-precision implementation makes)."""
    return o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("single", dict(size=(240, 135)))])
def test_margin_flag_covers_perturbed_inputs(name, kw):
    # Rays whose decisions flip when the inputs move by a few dozen single-precision ulps
    # must be flagged: that is what lets a single-precision implementation disagree with
    # the oracle only inside the margin.
    scene, probes, g, o, d = _setup(name, **kw)
    r = oracle.trace(g, o, d)
    rng = np.random.default_rng(22)
    flips = 0
    for eps in (0.0, 1e-6, 3e-6):
        o2, d2 = _rounded_rays(o, d)
        if eps:
            o2 = o * (1 + rng.uniform(-eps, eps, size=o.shape))
            d2 = d * (1 + rng.uniform(-eps, eps, size=d.shape))
        r2 = oracle.trace(g, o2, d2)
        diff = (r["status"] != r2["status"]) | (r["texel"] != r2["texel"]) | (r["probe"] != r2["probe"])
        flips += diff.sum()
        assert np.all((r["margin"][diff] != 0) | (r2["margin"][diff] != 0)), np.nonzero(diff & (r["margin"] == 0))
        # the flipped decisions sit far inside the stated margin
        assert np.all(np.minimum(r["score"][diff], r2["score"][diff]) <= 0.2 * oracle.DEFAULT_DELTA)
    if name == "single":
        assert flips > 0
    assert (r["margin"] != 0).mean() < 0.25

"""The oracle's soft-visibility relaxation (an extension; the paper's HIT/UNKNOWN decision is
hard): every probe trace whose first firing texel faces the ray is a candidate, accepted
with a logistic weight of how far the ray entered that texel behind the stored surface.

Pins (none of them retypes the mixture formula):
* the hard limit: as sigma -> 0 the soft colour is the hard oracle's colour, ray by ray;
* the background enters linearly with the remaining weight: rgb(bg2) - rgb(bg1) =
  trans (bg2 - bg1), and the weights of the candidates and the background sum to one;
* the candidates are the hard method's probe traces: the first candidate accepted with
  weight > 1/2 is the hard HIT (same probe, texel, distance), and every candidate before
  it is a shadow-entry UNKNOWN;
* the colour is linear in the radiance with the candidates fixed: the radiance VJP passes
  the dot-product test against a finite change of the radiance;
* the distance VJP equals central differences of the soft colour in the stored distances
  (double precision, texels of rays with no near decision, step far below every gap).
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def room():
    scene, probes, views = synth.workload("tiny")
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    return probes, g, o, d


def test_hard_limit(room):
    probes, g, o, d = room
    h = oracle.trace(g, o, d, background=(0.2, 0.4, 0.6))
    s = oracle.trace_soft(g, o, d, 1e-4 * 8 / probes.N, background=(0.2, 0.4, 0.6))
    clear = h["margin"] == 0
    assert np.abs(s["rgb"][clear] - h["rgb"][clear]).max() < 1e-9
    # at a moderate temperature the colour moves, but only on rays with a candidate near the
    # shadow-entry threshold
    s2 = oracle.trace_soft(g, o, d, 0.25 * 8 / probes.N, background=(0.2, 0.4, 0.6))
    moved = np.abs(s2["rgb"] - h["rgb"]).max(1) > 1e-3
    assert 0 < moved.mean() < 0.2


def test_background_and_weights(room):
    probes, g, o, d = room
    sig = 0.5 * 8 / probes.N
    s1 = oracle.trace_soft(g, o, d, sig, background=(0.0, 0.0, 0.0))
    s2 = oracle.trace_soft(g, o, d, sig, background=(1.0, 2.0, 3.0))
    assert np.array_equal(s1["count"], s2["count"])
    assert np.allclose(s2["rgb"] - s1["rgb"], s1["trans"][:, None] * np.array([1.0, 2.0, 3.0]), atol=1e-12)
    # weights: a_j prod_{i<j} (1 - a_i), plus the background's, sum to one
    n, K = s1["a"].shape
    total = s1["trans"].copy()
    P = np.ones(n)
    for j in range(K):
        on = s1["count"] > j
        total[on] += s1["a"][on, j] * P[on]
        P[on] *= 1.0 - s1["a"][on, j]
    assert np.allclose(total, 1.0, atol=1e-12)
    assert np.allclose(P, s1["trans"], rtol=1e-12, atol=1e-300)
    assert s1["count"].mean() > 1.5  # at this temperature most rays mix several candidates


def test_candidates_are_the_hard_probe_traces(room):
    probes, g, o, d = room
    h = oracle.trace(g, o, d)
    s = oracle.trace_soft(g, o, d, 0.1 * 8 / probes.N)
    clear = (h["margin"] == 0) & (h["status"] == oracle.HIT)
    checked = 0
    for i in np.nonzero(clear)[0][:3000]:
        m = s["count"][i]
        first = np.nonzero(s["a"][i, :m] > 0.5)[0]
        assert len(first), i
        j = first[0]
        assert s["probe"][i, j] == h["probe"][i] and s["texel"][i, j] == h["texel"][i], i
        assert abs(s["t"][i, j] - h["t"][i]) <= 1e-12 * max(1.0, h["t"][i])
        # the candidates before it entered their texel behind the surface (shadow entry)
        tau = 8.0 / probes.N
        assert np.all(s["rin"][i, :j] > s["rk"][i, :j] * (1 + tau)), i
        checked += 1
    assert checked > 1000


def test_radiance_vjp_dot_product(room):
    probes, g, o, d = room
    sig = 0.5 * 8 / probes.N
    s = oracle.trace_soft(g, o, d, sig)
    rng = np.random.default_rng(3)
    gr = rng.normal(size=(len(o), 3))
    _, grad = oracle.vjp_soft(g, s, gr)
    dR = rng.normal(size=grad.shape) * 1e-3
    g2 = oracle.Grid.from_probes(probes, radiance=g.radiance + dR.astype(np.float32))
    # the float32 perturbation actually applied
    dR32 = g2.radiance.astype(np.float64) - g.radiance.astype(np.float64)
    s2 = oracle.trace_soft(g2, o, d, sig)
    assert np.array_equal(s2["count"], s["count"])
    lhs = np.sum(gr * (s2["rgb"] - s["rgb"]))
    rhs = np.sum(grad * dR32)
    assert abs(lhs - rhs) <= 1e-9 * (abs(rhs) + 1e-12) + 1e-12, (lhs, rhs)


def test_distance_vjp_central_differences(room):
    probes, g, o, d = room
    sig = 0.5 * 8 / probes.N
    h = oracle.trace(g, o, d)
    clear = h["margin"] == 0
    o, d = o[clear][::4], d[clear][::4]
    s = oracle.trace_soft(g, o, d, sig)
    rng = np.random.default_rng(5)
    gr = rng.normal(size=(len(o), 3))
    gd, _ = oracle.vjp_soft(g, s, gr)
    # texels that carry a candidate's distance gradient; perturb each one alone
    N = probes.N
    flat = np.argsort(-np.abs(gd.ravel()))[:12]
    D = probes.distance.astype(np.float64)
    for f in flat:
        p, k = divmod(int(f), N * N)
        r = D.reshape(-1, N * N)[p, k]
        h1 = 8.0 * float(np.spacing(np.float32(r)))  # 8 FP32 ulps: r +- h1, r +- 2 h1 are exact
        vals = []
        for step in (1.0, -1.0, 2.0, -2.0):
            dist = probes.distance.copy()
            dist.reshape(-1, N * N)[p, k] = np.float32(r + step * h1)
            assert float(dist.reshape(-1, N * N)[p, k]) == r + step * h1
            gp = oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                             probes.scene_max, dist, probes.normal, g.radiance)
            sp = oracle.trace_soft(gp, o, d, sig)
            assert np.array_equal(sp["count"], s["count"]), "a candidate set changed"
            vals.append(np.sum(gr * sp["rgb"]))
        c1 = (vals[0] - vals[1]) / (2 * h1)
        c2 = (vals[2] - vals[3]) / (4 * h1)
        fd = (4 * c1 - c2) / 3  # Richardson: O(h^4)
        assert abs(fd - gd.ravel()[f]) <= 1e-7 * abs(gd.ravel()[f]) + 1e-9, (p, k, fd, gd.ravel()[f])

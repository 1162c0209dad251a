"""Paper-literal variants of the method, on the oracle: the hit texel's own radiance (the
appendix algorithms traceOneProbe / highResolutionTracing fetch the colour of the texel the
march stopped at), the printed classification without the shadow-entry rule, the
two-probe limit, and normal maps that hold the probe-to-point direction (Implementation
Details: the "normal" map of the probe data generation)."""
import numpy as np

import oracle
import synth
from conftest import workload


def _grid_rays(name="tiny", **kw):
    scene, probes, views = workload(name, **kw)
    og = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    return scene, probes, og, o, d


def test_nearest_radiance_is_the_hit_texel():
    scene, probes, og, o, d = _grid_rays()
    bil = oracle.trace(og, o, d)
    near = oracle.trace(og, o, d, nearest=True)
    # radiance never changes the geometry
    for k in ("status", "probe", "texel", "t", "margin"):
        assert np.array_equal(bil[k], near[k]), k
    h = near["status"] == oracle.HIT
    assert h.mean() > 0.9
    R = probes.radiance.view(np.float16).astype(np.float64).reshape(probes.n_probes, -1, 3)
    assert np.array_equal(near["rgb"][h], R[near["probe"][h], near["texel"][h]])
    assert np.array_equal(near["taps"][h, 0], near["texel"][h])
    assert np.all(near["wts"][h] == np.array([1.0, 0.0, 0.0, 0.0]))
    # and it differs from the filtered sample somewhere (the variant is not a no-op)
    assert np.abs(near["rgb"][h] - bil["rgb"][h]).max() > 1e-3


def test_nearest_vjp_scatters_each_rays_gradient_to_its_texel():
    scene, probes, og, o, d = _grid_rays()
    near = oracle.trace(og, o, d, nearest=True)
    g = np.random.default_rng(1).normal(size=(len(o), 3))
    got = oracle.vjp(og, near, g).reshape(-1, 3)
    ref = np.zeros_like(got)
    h = near["status"] == oracle.HIT
    np.add.at(ref, near["probe"][h] * probes.N * probes.N + near["texel"][h], g[h])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_incoming_direction_normal_map_is_the_texel_direction():
    scene, probes, views = workload("tiny")
    lit = synth.bake(scene, probes.N, probes.levels, normals="incoming")
    assert np.array_equal(lit.distance, probes.distance)
    uv = lit.normal.view(np.float16).astype(np.float64)
    N = probes.N
    c = -1.0 + (2.0 * np.arange(N) + 1.0) / N
    assert np.array_equal(uv[0, :, :, 0], np.broadcast_to(c[None, :], (N, N)))
    assert np.array_equal(uv[0, :, :, 1], np.broadcast_to(c[:, None], (N, N)))
    # with these maps a HIT needs the ray to move against the probe-to-point direction of
    # the hit texel; every other first fire is UNKNOWN
    og = oracle.Grid.from_probes(lit)
    o, d = oracle.view_rays(*views[0].as_tuple())
    res = oracle.trace(og, o, d)
    h = res["status"] == oracle.HIT
    k = res["texel"][h]
    dirs = np.array([oracle.oct_decode((c[t % N], c[t // N])) for t in k])
    assert len(dirs) > 0 and np.all(np.einsum("ij,ij->i", dirs, d[h]) < 0)
    # the geometric maps resolve more rays than the literal ones on the same room
    geo = oracle.trace(oracle.Grid.from_probes(probes), o, d)
    assert (geo["status"] == oracle.HIT).mean() > h.mean()


def test_paper_classification_without_shadow_rule():
    # tau = +inf: the first fire is HIT whenever its stored normal faces the ray
    scene, probes, og, o, d = _grid_rays()
    lit = oracle.trace(og, o, d, thickness_rel=float("inf"))
    ref = oracle.trace(og, o, d)
    # dropping the rule only turns shadow-entry UNKNOWNs into HITs or later resolutions:
    # a ray the default resolves at some (cell, probe) rank is resolved no later without it
    both = (lit["status"] == oracle.HIT) & (ref["status"] == oracle.HIT)
    assert np.all(lit["rank"][both] <= ref["rank"][both])
    assert (lit["status"] == oracle.HIT).sum() >= (ref["status"] == oracle.HIT).sum()

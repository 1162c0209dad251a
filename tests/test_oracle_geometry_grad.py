"""Gradient through the stored distances (an extension beyond the paper, which renders
forward only): with the classification held fixed, a HIT ray depends on the distance of its
hit texel through the hit distance t, and on t through the position of its bilinear
radiance sample.  oracle.trace returns dt/dr and drgb/dt per ray; oracle.vjp_distance
assembles dL/dr.

Pins: central finite differences of the oracle itself on perturbed FP32 distance maps (two
step sizes; rays whose classification changes under the step are left out), the three
closed-form cases (eye lookup dt/dr = 1 and no radiance motion; entry hit dt/dr = 0; root
dt/dr = r / (q . w) with q the hit point seen from the probe), and the assembly of the
adjoint against a dense Jacobian-vector product.
"""
import numpy as np
import pytest

import oracle
from conftest import workload


def _grid_with(probes, distance, radiance):
    return oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                       probes.scene_max, distance, probes.normal, radiance)


def _random_radiance(probes, seed=0):
    # a radiance field that varies from texel to texel, so the sample's motion shows
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(probes.n_probes, probes.N, probes.N, 3)).astype(np.float32)


def _fd(probes, rad, o, d, flat, eps):
    """Central differences of t and rgb w.r.t. the distances at the flat texel indices,
    perturbed together by the relative step eps (each ray depends on its own texel only)."""
    base = probes.distance.reshape(-1)
    outs = []
    dr = None
    for sgn in (1.0, -1.0):
        dist = base.copy()
        dist[flat] = (base[flat].astype(np.float64) * (1.0 + sgn * eps)).astype(np.float32)
        if dr is None:
            dr = dist[flat].astype(np.float64)
        else:
            dr = dr - dist[flat].astype(np.float64)
        outs.append(oracle.trace(_grid_with(probes, dist.reshape(probes.distance.shape), rad), o, d))
    return outs, dr


def test_hit_distance_and_sample_motion_match_finite_differences(single_small):
    scene, probes, views = single_small
    rad = _random_radiance(probes)
    g = _grid_with(probes, probes.distance, rad)
    o, d = oracle.view_rays(*views[0].as_tuple())
    r = oracle.trace(g, o, d)
    N = probes.N
    ok = (r["status"] == oracle.HIT) & (r["margin"] == 0)
    flat_all = r["probe"].astype(np.int64) * N * N + r["texel"]
    # one ray per hit texel, so that a joint perturbation moves each ray's own texel only
    _, first = np.unique(np.where(ok, flat_all, -1), return_index=True)
    sel = first[ok[first]][:3000]
    o, d = o[sel], d[sel]
    r = {k: v[sel] for k, v in r.items()}
    flat = flat_all[sel]
    fds = []
    for eps in (2.0 ** -12, 2.0 ** -13):
        (rp, rm), dr = _fd(probes, rad, o, d, flat, eps)
        same = np.ones(len(sel), bool)
        for x in (rp, rm):
            same &= (x["status"] == r["status"]) & (x["probe"] == r["probe"]) & (x["texel"] == r["texel"])
            # t(r) is continuous but kinks where the hit switches between the texel's entry
            # point and the root (rho_in = r): such rays are left out too
            same &= (x["dtdr"] == 0) == (r["dtdr"] == 0)
        fds.append((same, (rp["t"] - rm["t"]) / dr, (rp["rgb"] - rm["rgb"]) / dr[:, None]))
    same = fds[0][0] & fds[1][0]
    assert same.mean() > 0.9
    root = same & (r["dtdr"] > 0)
    entry = same & (r["dtdr"] == 0)
    assert root.sum() > 500 and entry.sum() > 50
    # entry hits do not move; root hits move as r / (q . w).  Richardson extrapolation of the
    # two central differences removes their O(eps^2) error (near-tangent roots are curved)
    assert np.all(fds[0][1][entry] == 0.0) and np.all(fds[1][1][entry] == 0.0)
    rich_t = (4.0 * fds[1][1] - fds[0][1]) / 3.0
    rel = np.abs(rich_t[root] - r["dtdr"][root]) / r["dtdr"][root]
    assert rel.max() < 1e-5, rel.max()
    assert np.median(rel) < 1e-10
    # the radiance sample: where both step sizes agree (no texel-centre line or fold crossed)
    want = r["dtdr"][:, None] * r["drgbdt"]
    smooth = root & np.all(np.abs(fds[0][2] - fds[1][2]) <= 1e-3 * (np.abs(fds[1][2]) + 1e-2), axis=1)
    assert smooth.sum() > 0.8 * root.sum()
    rich_c = (4.0 * fds[1][2] - fds[0][2]) / 3.0
    err = np.abs(rich_c[smooth] - want[smooth])
    assert np.all(err <= 1e-4 * (np.abs(want[smooth]) + 1e-2)), err.max()
    assert np.abs(want[smooth]).max() > 1.0  # the field does vary along the hit points


def test_eye_lookup_moves_with_the_stored_distance_only():
    scene, probes, views = workload("tiny")
    rad = _random_radiance(probes, 1)
    g = _grid_with(probes, probes.distance, rad)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(g.probe_position(3), d.shape).copy()
    r = oracle.trace(g, o, d)
    # rays whose first cell holds their stored surface are resolved by the eye lookup of
    # probe 3; the others fall through to other probes in later cells
    hit = (r["status"] == oracle.HIT) & (r["probe"] == 3)
    assert hit.mean() > 0.5
    assert np.all(r["dtdr"][hit] == 1.0)
    assert np.all(r["drgbdt"][hit] == 0.0)
    assert np.array_equal(r["t"][hit], probes.distance.reshape(probes.n_probes, -1)[3, r["texel"][hit]])


def test_root_derivative_closed_form(single_small):
    # dt/dr = r / (q . w): q = X - O + t w is the hit point seen from the probe, and q . w is
    # the square root in the larger root of |X - O + t w| = r
    scene, probes, views = single_small
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple(), pixels=np.arange(0, 240 * 135, 7))
    r = oracle.trace(g, o, d)
    root = (r["status"] == oracle.HIT) & (r["dtdr"] > 0) & (r["margin"] == 0)
    assert root.sum() > 500
    pos = np.stack([g.probe_position(p) for p in r["probe"][root]])
    q = o[root] + r["t"][root, None] * d[root] - pos
    rk = probes.distance.reshape(probes.n_probes, -1)[r["probe"][root], r["texel"][root]].astype(np.float64)
    assert np.allclose(np.linalg.norm(q, axis=1), rk, rtol=1e-12)
    assert np.allclose(r["dtdr"][root], rk / np.sum(q * d[root], axis=1), rtol=1e-9)


def test_distance_adjoint_assembly(tiny):
    # <dL/dr, delta> equals the directional derivative of L = <g_t, t> + <g_rgb, rgb> along
    # delta, summed ray by ray from the per-ray derivatives
    scene, probes, views = tiny
    rad = _random_radiance(probes, 3)
    g = _grid_with(probes, probes.distance, rad)
    o, d = oracle.view_rays(*views[0].as_tuple())
    r = oracle.trace(g, o, d)
    rng = np.random.default_rng(4)
    n = len(o)
    gt = rng.normal(size=n)
    grgb = rng.normal(size=(n, 3))
    adj = oracle.vjp_distance(g, r, grad_rgb=grgb, grad_t=gt)
    assert adj.shape == probes.distance.shape
    delta = rng.normal(size=probes.distance.shape)
    hit = r["status"] == oracle.HIT
    flat = r["probe"][hit].astype(np.int64) * probes.N ** 2 + r["texel"][hit]
    dirderiv = r["dtdr"][hit] * delta.reshape(-1)[flat] * (gt[hit] + np.sum(grgb[hit] * r["drgbdt"][hit], axis=1))
    assert np.isclose(np.sum(adj * delta), dirderiv.sum(), rtol=1e-10)
    # the gradient lives on hit texels only
    touched = np.zeros(adj.size, bool)
    touched[flat] = True
    assert np.all(adj.reshape(-1)[~touched] == 0.0)

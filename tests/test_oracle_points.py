"""Probe baking from a point cloud, the oracle's definition (oracle/points.py): nearest
point per texel (Implementation Details, Probe Data Generation), pinned by closed forms,
an independent double-precision check of the nearest-point property, and the analytic
limit of a dense cloud."""
import numpy as np

import oracle
import synth
from conftest import workload
from oracle.points import bake_points, probe_origins


def _centre_dir(i, j, N):
    return oracle.oct_decode(np.array([-1 + (2 * i + 1) / N, -1 + (2 * j + 1) / N]))


def test_points_on_texel_centres_give_their_distances_and_colours():
    N = 16
    dims, origin, spacing = (1, 1, 1), (0.5, 0.5, 0.5), (1.0, 1.0, 1.0)
    O = probe_origins(dims, origin, spacing).astype(np.float64)
    rng = np.random.default_rng(0)
    pts, cols, want_d, want_c = [], [], {}, {}
    for p in range(1):
        for (i, j) in [(0, 0), (3, 7), (15, 15), (8, 2), (12, 9)]:
            d = _centre_dir(i, j, N)
            r_near, r_far = rng.uniform(0.5, 2.0), rng.uniform(2.5, 4.0)
            for r in (r_far, r_near):  # the far point first: order must not matter
                pts.append(O[p] + r * d)
                c = rng.uniform(0.1, 0.9, 3)
                cols.append(c)
                if r == r_near:
                    want_d[(p, j * N + i)] = r
                    want_c[(p, j * N + i)] = c
    pts, cols = np.array(pts, np.float32), np.array(cols, np.float32)
    dist, nrm, rad, win = bake_points(dims, origin, spacing, N, pts, cols)
    filled = np.isfinite(dist).reshape(1, -1)
    assert filled.sum() == len(want_d)
    for (p, k), r in want_d.items():
        assert abs(dist.reshape(1, -1)[p, k] - r) < 1e-5 * r
        c = rad.reshape(1, -1, 3)[p, k].view(np.float16).astype(np.float64)
        assert np.allclose(c, want_c[(p, k)], atol=1e-3)
    # empty texels: no data
    assert np.all(np.isnan(dist.reshape(1, -1)[~filled]))
    assert np.all(nrm.reshape(1, -1, 2)[~filled] == 0) and np.all(rad.reshape(1, -1, 3)[~filled] == 0)


def test_stored_point_is_the_nearest_in_its_texel_in_double():
    # independent check: bin every point with the double-precision octahedral map of the
    # trace oracle and compare distances in double; points within 1e-5 of a texel edge or
    # of the winner's distance are left out (FP32 may decide those either way)
    scene, probes, views = workload("tiny")
    pts, col, nrm = synth.sample_points(scene, 60000, 11)
    N = 32
    dist, _, _, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    P64 = pts.astype(np.float64)
    for p in range(len(O)):
        d = P64 - O[p]
        r = np.linalg.norm(d, axis=1)
        uv = np.array([oracle.oct_encode(x) for x in d[::7]])  # a subsample keeps it quick
        x, y = (uv[:, 0] + 1) * N / 2, (uv[:, 1] + 1) * N / 2
        i, j = np.clip(np.floor(x), 0, N - 1).astype(int), np.clip(np.floor(y), 0, N - 1).astype(int)
        edge = (np.minimum(x - np.floor(x), np.ceil(x) - x) < 1e-5) | (np.minimum(y - np.floor(y), np.ceil(y) - y) < 1e-5)
        stored = dist[p][j, i].astype(np.float64)
        rs = r[::7]
        ok = edge | (stored <= rs * (1 + 1e-6))
        assert ok.all(), (p, np.nonzero(~ok)[0][:5])
        # and the stored distance is the distance of the stored point
        w = win[p].ravel()
        has = w >= 0
        assert np.allclose(dist[p].ravel()[has], r[w[has]], rtol=1e-6)


def test_dense_cloud_approaches_the_analytic_bake():
    # The centre ray of a texel meets a surface at the analytic distance r_a; a dense cloud
    # has points on that surface next to the hit inside the texel's cone, so the nearest
    # point is at most a fraction of the texel's angular size farther: r <= r_a (1 + 2 theta)
    # wherever the cloud is dense on the footprint (>= 20 expected points in (r_a theta)^2).
    # It may be nearer (another surface poking into the cone), so the bound is one-sided.
    scene, probes, views = workload("tiny")
    n = 400000
    pts, col, nrm = synth.sample_points(scene, n, 12)
    R = scene.room_max
    area = 2 * (R[0] * R[1] + R[1] * R[2] + R[0] * R[2])
    for t, p in zip(scene.obj_type, scene.obj_param):
        area += 8 * (p[3] * p[4] + p[4] * p[5] + p[3] * p[5]) if t == 0 else 4 * np.pi * p[3] ** 2
    N = probes.N
    dist, nuv, rad, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    from test_oracle_scene import _texel_diameter
    theta = _texel_diameter(N, np.arange(N * N))[None, :]
    ra = probes.distance.reshape(len(dist), -1).astype(np.float64)
    rp = dist.reshape(len(dist), -1).astype(np.float64)
    dense = np.isfinite(rp) & (n / area * (ra * theta) ** 2 >= 20)
    assert dense.mean() > 0.8
    assert not (dense & (rp > ra * (1 + 2 * theta))).any()
    assert np.median(np.abs(rp - ra)[dense] / ra[dense]) < 0.02


def test_literal_normal_map_is_the_direction_to_the_stored_point():
    scene, probes, views = workload("tiny")
    pts, col, nrm = synth.sample_points(scene, 50000, 13)
    N = 32
    dist, nuv, rad, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, None)
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    uv = nuv.view(np.float16).astype(np.float64).reshape(len(dist), -1, 2)
    w = win.reshape(len(dist), -1)
    for p in range(len(O)):
        has = np.nonzero(w[p] >= 0)[0][::5]
        for k in has:
            d = pts[w[p, k]].astype(np.float64) - O[p]
            want = oracle.oct_encode(d)
            assert np.allclose(uv[p, k], want, atol=2e-3)
            # inside the texel it was binned to
            i, j = k % N, k // N
            assert -1 + 2 * i / N - 2e-3 <= uv[p, k, 0] <= -1 + 2 * (i + 1) / N + 2e-3
            assert -1 + 2 * j / N - 2e-3 <= uv[p, k, 1] <= -1 + 2 * (j + 1) / N + 2e-3

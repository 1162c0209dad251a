"""Pins of the oracle's octahedral map, min pyramid and bilinear fetch.

The octahedral map (paper: Overview, octahedral mapping figure) sends the unit sphere to
the octahedron |x|+|y|+|z| = 1 and unfolds it into the square [-1,1]^2; its vertices,
edges and folds are fixed by that construction, which these tests check by value.
"""
import numpy as np
import pytest

import oracle


def test_octahedron_vertices_map_to_fixed_points():
    # +z is the centre, the four equator vertices are the edge midpoints of the inner
    # diamond, -z is the square's corners (all four are the same point; with the sign
    # convention s(0) = +1 it lands on (1, 1)).
    cases = {(0, 0, 1): (0, 0), (1, 0, 0): (1, 0), (-1, 0, 0): (-1, 0), (0, 1, 0): (0, 1),
             (0, -1, 0): (0, -1), (0, 0, -1): (1, 1)}
    for d, uv in cases.items():
        np.testing.assert_allclose(oracle.oct_encode(np.array(d, float)), uv, atol=1e-15)
    for c in [(1, 1), (-1, 1), (1, -1), (-1, -1)]:
        np.testing.assert_allclose(oracle.oct_decode(np.array(c, float)), (0, 0, -1), atol=1e-15)


def test_upper_hemisphere_is_inner_diamond_and_l1_scale():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        d = rng.normal(size=3)
        uv = oracle.oct_encode(d)
        inner = abs(uv[0]) + abs(uv[1]) <= 1 + 1e-15
        assert inner == (d[2] >= 0)
        if d[2] >= 0:  # central projection onto the octahedron face: uv = (x, y) / |d|_1
            np.testing.assert_allclose(uv, d[:2] / np.abs(d).sum(), atol=1e-15)
        # quadrant of the map = signs of x and y
        assert np.sign(uv[0]) in (np.sign(d[0]), 0) and np.sign(uv[1]) in (np.sign(d[1]), 0)


def test_round_trips():
    rng = np.random.default_rng(2)
    for _ in range(3000):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        np.testing.assert_allclose(oracle.oct_decode(oracle.oct_encode(d)), d, atol=1e-12)
    for _ in range(3000):
        uv = rng.uniform(-1, 1, size=2)
        np.testing.assert_allclose(oracle.oct_encode(oracle.oct_decode(uv)), uv, atol=1e-12)


def test_fold_edges_identify_mirrored_points():
    # across the square's edge u = 1 the map continues mirrored in v: (1, v) ~ (1, -v),
    # likewise for the other three edges.
    for v in np.linspace(-1, 1, 17):
        np.testing.assert_allclose(oracle.oct_decode(np.array([1.0, v])), oracle.oct_decode(np.array([1.0, -v])),
                                   atol=1e-15)
        np.testing.assert_allclose(oracle.oct_decode(np.array([v, -1.0])), oracle.oct_decode(np.array([-v, -1.0])),
                                   atol=1e-15)


def test_min_pyramid_is_block_minimum():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.1, 5, size=(3, 32, 32)).astype(np.float32)
    d[1, 5, 7] = np.nan  # a texel without data never lowers the minimum
    pyr = oracle.min_mips(d, 4)
    for l in range(1, 4):
        b = 1 << l
        n = 32 >> l
        for p in range(3):
            for j in range(n):
                for i in range(n):
                    block = d[p, j * b:(j + 1) * b, i * b:(i + 1) * b]
                    assert pyr[l][p, j, i] == np.nanmin(block)
        assert pyr[l].dtype == np.float32


def test_bilinear_at_texel_centres_and_weights():
    N = 16
    for j in range(N):
        for i in range(N):
            u = -1 + (2 * i + 1) / N
            v = -1 + (2 * j + 1) / N
            idx, wt = oracle.bilinear_taps(u, v, N)
            assert idx[0] == j * N + i and wt[0] == 1.0 and np.all(wt[1:] == 0)
    rng = np.random.default_rng(4)
    for _ in range(500):
        idx, wt = oracle.bilinear_taps(*rng.uniform(-1, 1, 2), N)
        assert abs(wt.sum() - 1) < 1e-14 and np.all(wt >= 0) and np.all((idx >= 0) & (idx < N * N))


def _smooth(d):
    return 0.3 + 0.2 * d[..., 0] - 0.1 * d[..., 1] + 0.4 * d[..., 2] + 0.1 * d[..., 0] * d[..., 2]


def _baked_field(N):
    """A smooth function of direction sampled at texel centres."""
    c = -1 + (2 * np.arange(N) + 1) / N
    f = np.empty(N * N)
    for j in range(N):
        for i in range(N):
            f[j * N + i] = _smooth(oracle.oct_decode(np.array([c[i], c[j]])))
    return f


def _filtered(f, d, N):
    idx, wt = oracle.bilinear_taps(*oracle.oct_encode(d), N)
    return float(np.dot(f[idx], wt))


def test_bilinear_wrap_is_continuous_across_seams():
    # Sampling a smooth field just either side of every fold (the equator, the square's
    # edges and the -z pole) must agree: the octahedral border wrap mirrors taps across
    # the edge, which is where the neighbouring directions are stored.
    N = 32
    f = _baked_field(N)
    rng = np.random.default_rng(5)
    e = 1e-7
    for _ in range(300):
        # points on the equator z = 0 (fold between inner diamond and outer triangles)
        a = rng.uniform(0, 2 * np.pi)
        base = np.array([np.cos(a), np.sin(a), 0.0])
        up, dn = base + [0, 0, e], base - [0, 0, e]
        assert abs(_filtered(f, up, N) - _filtered(f, dn, N)) < 1e-3
        # points on the x = 0 and y = 0 meridians of the lower hemisphere (square edges)
        z = -rng.uniform(0.05, 1.0)
        for base in (np.array([0.0, np.sqrt(1 - z * z), z]), np.array([np.sqrt(1 - z * z), 0.0, z])):
            k = 0 if base[0] == 0 else 1
            p1, p2 = base.copy(), base.copy()
            p1[k] += e
            p2[k] -= e
            assert abs(_filtered(f, p1, N) - _filtered(f, p2, N)) < 1e-3
    # around the -z pole (the four corners of the square)
    vals = [_filtered(f, np.array([np.cos(a) * 1e-6, np.sin(a) * 1e-6, -1.0]), N) for a in np.linspace(0, 6, 13)]
    assert max(vals) - min(vals) < 1e-3


def test_filtered_field_converges_to_the_field():
    # bilinear of a smooth field sampled at texel centres converges to it: first order at
    # worst (the map's folds are only piecewise linear), second order in the RMS sense
    rng = np.random.default_rng(6)
    dirs = rng.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    mx, rms = [], []
    for N in (16, 32, 64):
        f = _baked_field(N)
        e = np.array([abs(_filtered(f, d, N) - _smooth(d)) for d in dirs])
        mx.append(e.max())
        rms.append(np.sqrt(np.mean(e ** 2)))
    assert mx[1] < mx[0] / 1.8 and mx[2] < mx[1] / 1.8
    assert rms[2] < rms[0] / 8
    assert mx[2] < 0.01


def test_half_decode_is_exact():
    for h, v in [(0x3C00, 1.0), (0xC000, -2.0), (0x0001, 2.0 ** -24), (0x7BFF, 65504.0), (0x3555, 0.333251953125)]:
        assert oracle.half_to_double(h) == v
    bits = np.arange(0, 0x7C00, 97, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = np.array([oracle.half_to_double(int(b)) for b in bits])
    assert np.array_equal(ref, got)

"""Pins of the oracle's ray march against what the geometry fixes.

* the projected ray of one probe splits into at most 4 straight pieces (Methodology,
  Ray Tracing Using One Probe), whose texel intervals tile the parameter range;
* the texel sequence found with boundary planes equals brute force: dense samples of
  the ray binned by the octahedral map;
* the hierarchical march over the min pyramid (appendix traceOneRaySegment and its
  low/high resolution helpers) finds the same first texel as the flat march
  (RayMarching) on every ray outside the float margin;
* rays cast from a probe centre return that probe's stored texel (Eye Aligned with a
  Probe);
* the reported hit point lies in the reported texel's cone at the stored distance.
"""
import numpy as np
import pytest

import oracle
from conftest import workload


def _brute_sequence(N, xp, w, ta, tb, n=400001):
    t = np.linspace(ta, tb, n)
    q = xp[None, :] + t[:, None] * w[None, :]
    l1 = np.abs(q).sum(1)
    p = q / l1[:, None]
    u = np.where(p[:, 2] >= 0, p[:, 0], (1 - np.abs(p[:, 1])) * np.where(p[:, 0] >= 0, 1.0, -1.0))
    v = np.where(p[:, 2] >= 0, p[:, 1], (1 - np.abs(p[:, 0])) * np.where(p[:, 1] >= 0, 1.0, -1.0))
    i = np.clip(np.floor((u + 1) * N / 2).astype(int), 0, N - 1)
    j = np.clip(np.floor((v + 1) * N / 2).astype(int), 0, N - 1)
    k = j * N + i
    change = np.nonzero(np.diff(k))[0]
    seq = [k[0]] + [k[c + 1] for c in change]
    tchange = [t[c] for c in change]
    return seq, tchange, (tb - ta) / (n - 1)


@pytest.mark.parametrize("N", [8, 16])
def test_texel_sequence_matches_brute_force(N):
    rng = np.random.default_rng(10 + N)
    checked = 0
    for _ in range(150):
        xp = rng.normal(size=3) * rng.uniform(0.2, 2.0)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        ta, tb = 0.0, rng.uniform(0.5, 6.0)
        ij, tio, piece = oracle.texel_sequence(N, xp, w, ta, tb)
        seq, tchange, dt = _brute_sequence(N, xp, w, ta, tb)
        # drop intervals too short for the sampling to see (corner passes)
        keep = (tio[:, 1] - tio[:, 0]) > 4 * dt
        ours = [int(j * N + i) for (i, j), k in zip(ij, keep) if k]
        ours = [k for n_, k in enumerate(ours) if n_ == 0 or k != ours[n_ - 1]]
        brute = [k for n_, k in enumerate(seq) if n_ == 0 or k != seq[n_ - 1]]
        # brute force also sees the short visits; remove texels it holds for < 4 samples
        tt = [ta] + list(tchange) + [tb]
        brute_long = [k for k, a, b in zip(seq, tt[:-1], tt[1:]) if b - a > 4 * dt]
        brute_long = [k for n_, k in enumerate(brute_long) if n_ == 0 or k != brute_long[n_ - 1]]
        assert ours == brute_long, (xp, w, tb)
        checked += 1
        # every boundary crossing of the march is one of the brute-force transitions
        bounds = tio[:-1, 1][np.diff(piece) == 0]
        for b in bounds:
            if len(tchange):
                assert np.min(np.abs(np.asarray(tchange) - b)) <= 2 * dt + 1e-12
    assert checked == 150


def test_pieces_tile_the_interval_and_are_at_most_four():
    rng = np.random.default_rng(11)
    for _ in range(500):
        N = int(rng.choice([8, 32, 128]))
        xp = rng.normal(size=3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        ta, tb = rng.uniform(0, 1), rng.uniform(1.5, 8)
        ij, tio, piece = oracle.texel_sequence(N, xp, w, ta, tb)
        assert piece.max() + 1 <= 4
        assert tio[0, 0] == ta and tio[-1, 1] == tb
        # texel intervals tile [ta, tb]: each starts where the previous one ended
        assert np.all(tio[1:, 0] == tio[:-1, 1])
        assert np.all(tio[:, 1] >= tio[:, 0])
        # consecutive texels inside a piece share an edge (or a corner at an exact tie)
        same = np.diff(piece) == 0
        d = np.abs(np.diff(ij, axis=0))[same]
        assert np.all(d.max(1) == 1)
        # each piece stays inside one quadrant of the map (one octant of directions)
        for pc in range(piece.max() + 1):
            sel = ij[piece == pc]
            assert len(set((sel[:, 0] >= N // 2).tolist())) == 1
            assert len(set((sel[:, 1] >= N // 2).tolist())) == 1


def test_pieces_count_matches_sign_changes():
    # pieces = 1 + number of coordinate sign changes of X' + t w inside (ta, tb)
    rng = np.random.default_rng(12)
    for _ in range(300):
        xp = rng.normal(size=3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        ta, tb = 0.0, 5.0
        _, _, piece = oracle.texel_sequence(32, xp, w, ta, tb)
        tz = -xp / w
        assert piece.max() + 1 == 1 + int(np.sum((tz > ta) & (tz < tb)))


def _non_margin(r):
    return r["margin"] == 0


def test_hierarchical_equals_flat(tiny, single_small):
    for scene, probes, views in (tiny, single_small):
        g = oracle.Grid.from_probes(probes)
        r = oracle.trace_view(g, views[0].as_tuple())
        hier = (r["margin"] & oracle.MG_HIER) != 0
        other = (r["margin"] & ~oracle.MG_HIER) != 0
        assert not np.any(hier & ~other)
        # starting lower in the pyramid (level 0 = flat) changes nothing
        for top in range(probes.levels):
            r2 = oracle.trace_view(g, views[0].as_tuple(), top_level=top)
            ok = _non_margin(r) & _non_margin(r2)
            assert np.array_equal(r["status"][ok], r2["status"][ok])
            assert np.array_equal(r["texel"][ok], r2["texel"][ok])
            assert np.array_equal(r["t"][ok], r2["t"][ok])


def test_hierarchy_saves_fetches(single_small):
    scene, probes, views = single_small
    g = oracle.Grid.from_probes(probes)
    r = oracle.trace_view(g, views[0].as_tuple())
    assert r["tests"].mean() < 0.5 * r["flat_tests"].mean()


def test_eye_at_probe_returns_stored_texel(tiny):
    scene, probes, views = tiny
    g = oracle.Grid.from_probes(probes)
    N = probes.N
    rng = np.random.default_rng(13)
    c = -1 + (2 * np.arange(N) + 1) / N
    for p in range(probes.n_probes):
        O = g.probe_position(p)
        ks = rng.choice(N * N, 200, replace=False)
        dirs = np.array([oracle.oct_decode(np.array([c[k % N], c[k // N]])) for k in ks])
        r = oracle.trace(g, np.broadcast_to(O, dirs.shape), dirs)
        # in the one-cell grid every ray from a probe centre is looked up in O(1)
        assert np.all(r["status"] == oracle.HIT)
        assert np.all(r["probe"] == p)
        assert np.array_equal(r["texel"], ks)
        assert np.array_equal(r["t"], probes.distance[p].ravel()[ks].astype(np.float64))
        rad = g.radiance[p].reshape(-1, 3)[ks]
        np.testing.assert_allclose(r["rgb"], rad, atol=1e-9)
        assert np.all(r["tests"] == 1)


def test_hit_point_lies_in_reported_texel(single_small):
    scene, probes, views = single_small
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    r = oracle.trace(g, o, d)
    N = probes.N
    tau = 8.0 / N
    hit = np.nonzero((r["status"] == oracle.HIT) & (r["margin"] == 0))[0]
    assert len(hit) > 0.8 * len(r["status"])
    for k in hit[::37]:
        p = r["probe"][k]
        q = o[k] - g.probe_position(p) + r["t"][k] * d[k]
        uv = oracle.oct_encode(q)
        x, y = (uv + 1) * N / 2
        i, j = r["texel"][k] % N, r["texel"][k] // N
        assert i - 1e-6 <= x <= i + 1 + 1e-6 and j - 1e-6 <= y <= j + 1 + 1e-6
        rk = float(probes.distance[p].ravel()[r["texel"][k]])
        rho = np.linalg.norm(q)
        # on the stored sphere, or entered behind it by less than the thickness
        assert abs(rho - rk) <= 1e-9 * rk or rk <= rho <= rk * (1 + tau) + 1e-12
        # the stored normal faces the ray
        nb = probes.normal[p].reshape(-1, 2)[r["texel"][k]]
        n = oracle.oct_decode(nb.view(np.float16).astype(np.float64))
        assert np.dot(n, d[k]) < 0


def test_hit_distance_is_the_larger_root(single_small):
    # where the ray enters the firing texel in front of the stored surface, the hit is the
    # exit point of the sphere rho = r (found here by bisection in double)
    scene, probes, views = single_small
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple(), pixels=np.arange(0, 240 * 135, 53))
    r = oracle.trace(g, o, d)
    n_checked = 0
    for k in np.nonzero(r["status"] == oracle.HIT)[0]:
        p = r["probe"][k]
        xp = o[k] - g.probe_position(p)
        rk = float(probes.distance[p].ravel()[r["texel"][k]])
        th = r["t"][k]
        rho = lambda t: np.linalg.norm(xp + t * d[k])
        if abs(rho(th) - rk) > 1e-9 * rk:
            continue  # entry-point hit
        lo, hi = th - 0.05 * rk, th + 0.05 * rk
        lo = max(lo, -np.dot(xp, d[k]))  # increasing branch of rho
        if rho(lo) > rk or rho(hi) < rk:
            continue
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if rho(mid) < rk else (lo, mid)
        assert abs(0.5 * (lo + hi) - th) <= 1e-9 * max(1.0, th)
        n_checked += 1
    assert n_checked > 50


def test_fall_through_to_next_probe(tiny):
    # a probe whose distance map is all zero answers UNKNOWN everywhere (every ray is
    # "below its surface"), so the next-closest probe must resolve the ray
    scene, probes, views = tiny
    g = oracle.Grid.from_probes(probes)
    v = views[0].as_tuple()
    r0 = oracle.trace_view(g, v)
    first = r0["rank"] % 8 == 0
    p0 = np.bincount(r0["probe"][first]).argmax()
    dist = probes.distance.copy()
    dist[p0] = 0.0
    g2 = oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                     probes.scene_max, dist, probes.normal, probes.radiance)
    r1 = oracle.trace_view(g2, v)
    assert not np.any(r1["probe"] == p0)
    moved = first & (r0["probe"] == p0) & (r1["status"] == oracle.HIT)
    assert moved.sum() > 100 and np.all(r1["rank"][moved] % 8 >= 1)
    # all probes empty of data (NaN never fires) -> MISS everywhere; all zero -> UNKNOWN
    for fill, expect in ((np.nan, oracle.MISS), (0.0, oracle.UNKNOWN)):
        g3 = oracle.Grid(probes.dims, probes.origin, probes.spacing, probes.N, probes.levels, probes.scene_min,
                         probes.scene_max, np.full_like(probes.distance, fill), probes.normal, probes.radiance)
        r3 = oracle.trace_view(g3, v, pixels=np.arange(0, 128 * 128, 7))
        assert np.all(r3["status"] == expect)
        assert np.all(np.isinf(r3["t"])) and np.all(r3["rgb"] == 0)


def test_two_probe_limit_is_a_subset(tiny):
    # with at most 2 probes per cell (the paper notes two usually suffice) every HIT found
    # is one the full search also finds at rank < 2
    scene, probes, views = tiny
    g = oracle.Grid.from_probes(probes)
    v = views[0].as_tuple()
    r8 = oracle.trace_view(g, v)
    r2 = oracle.trace_view(g, v, max_probes_per_cell=2)
    h2 = r2["status"] == oracle.HIT
    ok = h2 & (r8["margin"] == 0) & (r2["margin"] == 0)
    assert np.array_equal(r2["texel"][ok], r8["texel"][ok])
    assert np.all(r8["rank"][ok] % 8 < 2)
    assert (r8["status"] == oracle.HIT).sum() >= h2.sum()


def test_degenerate_rays_give_valid_hits(tiny, single_small):
    # axis-aligned rays, rays through probe centres and along cell planes: every HIT point
    # lies in its texel at a radial distance in [r, r (1 + tau)]
    from degenerate import degenerate_rays, hit_is_valid
    for scene, probes, views in (tiny, single_small):
        o, d, tag = degenerate_rays(scene, probes)
        r = oracle.trace(oracle.Grid.from_probes(probes), o.astype(np.float64), d.astype(np.float64))
        hit = np.stack([r["probe"], r["texel"]], 1)
        assert hit_is_valid(probes, o, d.astype(np.float64), r["status"], hit, r["t"], 8.0 / probes.N).all()
        assert (r["status"] == oracle.HIT).mean() > 0.95
        # planted mistakes are caught: a texel 7 columns away, another probe, a hit point 5%
        # in front of the stored surface (a few may still be valid at an exact tie)
        h = np.nonzero(r["status"] == oracle.HIT)[0][:200]
        N = probes.N
        for bad_hit, bad_t in ((np.stack([hit[h, 0], (hit[h, 1] // N) * N + (hit[h, 1] % N + 7) % N], 1), r["t"][h]),
                               (np.stack([(hit[h, 0] + 1) % probes.n_probes, hit[h, 1]], 1), r["t"][h]),
                               (hit[h], r["t"][h] * 0.95)):
            ok = hit_is_valid(probes, o[h], d[h].astype(np.float64), r["status"][h], bad_hit, bad_t, 8.0 / N)
            assert ok.mean() < 0.05, ok.mean()

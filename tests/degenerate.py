"""Degenerate camera rays for the parity tests: axis-aligned and plane-diagonal directions,
rays through probe centres (where the projected ray jumps across the map), rays starting
on cell planes and moving inside them, and rays starting at probe centres along the axes
(the eye-aligned lookup plus rays along lines of probes).  Several results can be correct
at such exact ties; the tests compare what is unique and check that the rest is valid."""
import numpy as np

import synth
from oracle.points import probe_origins


def degenerate_rays(scene, probes, seed=0, n_free=60):
    """(origins [n,3] f32, directions [n,3] f32, case tag [n]) in the room of ``probes``."""
    rng = np.random.default_rng(seed)
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    free = []
    while len(free) < n_free:
        p = rng.uniform(0.2 * probes.spacing[0], scene.room_max - 0.2 * probes.spacing[0])
        if synth.clearance(scene, p) > 0.05 * probes.spacing[0]:
            free.append(p)
    o, d, tag = [], [], []
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    for p in free:
        for a in axes:
            o.append(p); d.append(a); tag.append(0)
        for a in ([1, 1, 0], [1, 0, -1], [0, -1, 1], [1, 1, 1], [-1, 1, -1]):
            o.append(p); d.append(np.array(a, float) / np.linalg.norm(a)); tag.append(1)
    for p in free[:40]:
        for q in rng.choice(len(O), 6, replace=False):
            v = O[q] - p
            o.append(p); d.append(v / np.linalg.norm(v)); tag.append(2)
    s = probes.spacing[0]
    for p in free[:40]:
        for a in range(3):
            if probes.dims[a] < 3:
                continue
            q = p.copy()
            q[a] = probes.origin[a] + s * rng.integers(1, probes.dims[a] - 1)
            if synth.clearance(scene, q) > 0.05 * s:
                v = rng.normal(size=3)
                o.append(q); d.append(v / np.linalg.norm(v)); tag.append(3)
                v[a] = 0.0
                o.append(q); d.append(v / np.linalg.norm(v)); tag.append(4)
    for q in rng.choice(len(O), min(30, len(O)), replace=False):
        if synth.clearance(scene, O[q]) > 0.05 * s:
            for a in axes:
                o.append(O[q]); d.append(a); tag.append(5)
    return np.array(o, np.float32), np.array(d, np.float32), np.array(tag)


def _sideways(w, h):
    """The zero shift, then 16 shifts of length h perpendicular to w (evenly around it)."""
    a = np.zeros(3)
    a[int(np.argmin(np.abs(w)))] = 1.0
    e1 = a - np.dot(a, w) * w
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(w, e1)
    yield np.zeros(3)
    for m in range(16):
        ang = 2.0 * np.pi * m / 16.0
        yield h * (np.cos(ang) * e1 + np.sin(ang) * e2)


def _first_fire_ok(g, probes, D, p, k, X, w, ti, r, tau, max_probes):
    """Whether the ray (X, w) can report probe p, texel k at distance ti: the hit point in
    texel k, and some cell whose interval holds ti (for a ray moving inside a cell plane, a
    cell on either side) has p among its first max_probes cage probes, with k reached in
    p's flat texel sequence over that interval (double precision) with no earlier texel
    firing clearly, and k itself firing without a shadow entry."""
    import oracle
    N = probes.N
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    Xp = X - O[p]
    uv = oracle.oct_encode(Xp + ti * w)
    ui, vj = (uv + 1.0) * N / 2.0
    ki, kj = k % N, k // N
    if not (ki - 1e-3 <= ui <= ki + 1 + 1e-3 and kj - 1e-3 <= vj <= kj + 1 + 1e-3):
        return False
    walks = [oracle.cell_walk(g, X, w)]
    for a in range(3):
        q = (X[a] - probes.origin[a]) / probes.spacing[a]
        if abs(w[a]) < 1e-6 and abs(q - round(q)) < 1e-5:
            for sgn in (-1.0, 1.0):
                Xa = X.copy()
                Xa[a] += sgn * 1e-4 * probes.spacing[a]
                walks.append(oracle.cell_walk(g, Xa, w))
    for cells, tab in walks:
        for c, (ta, tb) in zip(cells, tab):
            if not (ta - 1e-5 * max(1.0, ti) <= ti <= tb + 1e-5 * max(1.0, ti)):
                continue
            if p not in oracle.cage_order(g, c, X)[:max_probes]:
                continue
            ij, tio, _ = oracle.texel_sequence(N, Xp, w, ta, tb)
            kk = ij[:, 1] * N + ij[:, 0]
            rin = np.linalg.norm(Xp[None, :] + tio[:, 0:1] * w[None, :], axis=1)
            rout = np.linalg.norm(Xp[None, :] + tio[:, 1:2] * w[None, :], axis=1)
            rmax = np.maximum(rin, rout)
            fires_clearly = D[p, kk] < rmax * (1 - 1e-5)
            may_fire = D[p, kk] < rmax * (1 + 1e-5)
            for m in np.nonzero(kk == k)[0]:
                if fires_clearly[:m].any():
                    break  # an earlier texel fires: the march stops before k
                if may_fire[m] and rin[m] <= r * (1 + tau) * (1 + 1e-5):
                    return True
    return False


def hit_is_valid(probes, o, d, status, hit, t, tau, max_probes=8):
    """Per ray: whether a reported HIT is one the method can give at an exact tie.

    A HIT of probe p, texel k at distance t is valid when (with FP32 slack: 1e-3 texel in
    the map, 1e-4 relative in distances, 1e-5 relative in the fire tests):
    * the hit point lies in texel k of probe p's map, at a radial distance rho between the
      stored r and r (1 + tau) (the root rho = r, or an entry point behind the surface);
    * the stored normal of the texel faces the ray (n . w < 0);
    * p is one of the first ``max_probes`` cage probes of a cell whose interval [ta, tb] of
      the ray holds t (for a ray moving inside a cell plane, a cell on either side), and
      in p's flat texel sequence over that interval (double precision) texel k is reached
      with no earlier texel firing (stored distance below the ray's largest radial distance
      in it), and k itself fires without a shadow entry (rho_in <= r (1 + tau)); at an
      exact tie of the texel sequence, for the ray itself or the ray moved sideways by
      1e-6 spacing in one of 16 directions around it;
    * for an eye at the probe (|X - O| <= 1e-6 spacing): t = r and k is the texel of oct(w).
    Non-HIT rays are valid with t = +inf."""
    import oracle
    N = probes.N
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    g = oracle.Grid.from_probes(probes)
    D = probes.distance.reshape(len(O), -1).astype(np.float64)
    nbits = probes.normal.reshape(len(O), N * N, 2)
    eye_eps = 1e-6 * float(np.min(probes.spacing))
    ok = np.ones(len(o), bool)

    def texel_of(uv):
        return (uv + 1.0) * N / 2.0

    def in_texel(uv, k, slack=1e-3):
        ti, tj = texel_of(uv)
        ki, kj = k % N, k // N
        return ki - slack <= ti <= ki + 1 + slack and kj - slack <= tj <= kj + 1 + slack

    for i in np.nonzero(status == oracle.HIT)[0]:
        p, k = int(hit[i, 0]), int(hit[i, 1])
        if not (0 <= p < len(O) and 0 <= k < N * N):
            ok[i] = False
            continue
        X = o[i].astype(np.float64)
        w = d[i].astype(np.float64)
        w /= np.linalg.norm(w)
        Xp = X - O[p]
        r = D[p, k]
        ti = float(t[i])
        nuv = np.array([oracle.half_to_double(int(b)) for b in nbits[p, k]])
        nrm = oracle.oct_decode(nuv)
        if not np.dot(nrm, w) < 1e-6:
            ok[i] = False
            continue
        if np.linalg.norm(Xp) <= eye_eps * (1 + 1e-3):
            ok[i] = abs(ti - r) <= 1e-4 * r and in_texel(oracle.oct_encode(w), k)
            continue
        # At an exact tie (a ray inside an axis plane through the probe projects onto a
        # texel boundary line, on the lower hemisphere onto the fold of the square's edge; a
        # ray through a texel corner) the texels on every side of the tie are valid: if the
        # ray itself does not validate the hit, the same ray moved sideways by 1e-6 spacing
        # in 16 directions around it is tried.
        if not (r * (1 - 1e-4) <= np.linalg.norm(Xp + ti * w) <= r * (1 + tau) * (1 + 1e-4)):
            ok[i] = False
            continue
        ok[i] = any(_first_fire_ok(g, probes, D, p, k, X + e, w, ti, r, tau, max_probes)
                    for e in _sideways(w, 1e-6 * float(np.min(probes.spacing))))
    ok[status != oracle.HIT] = ~np.isfinite(t[status != oracle.HIT])
    return ok

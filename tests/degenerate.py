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


def hit_is_valid(probes, o, d, status, hit, t, tau, texel_slack=1):
    """Per ray: a HIT is valid when its point lies in the reported probe's reported texel
    (within ``texel_slack`` texels) at a radial distance between the stored distance r and
    r (1 + tau) (the hit is the root rho = r or an entry point with r <= rho <= r (1 + tau)),
    with an FP32 slack of 1e-4 relative.  Non-HIT rays are valid with t = +inf."""
    import oracle
    N = probes.N
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    ok = np.ones(len(o), bool)
    for i in np.nonzero(status == oracle.HIT)[0]:
        p, k = int(hit[i, 0]), int(hit[i, 1])
        q = o[i].astype(np.float64) + float(t[i]) * d[i].astype(np.float64) - O[p]
        rho = np.linalg.norm(q)
        r = float(probes.distance[p].ravel()[k])
        if rho < 1e-9:
            ok[i] = False
            continue
        uv = oracle.oct_encode(q)
        ti, tj = (uv + 1) * N / 2
        ki, kj = k % N, k // N
        near = (ki - texel_slack - 1e-3 <= ti <= ki + 1 + texel_slack + 1e-3 and
                kj - texel_slack - 1e-3 <= tj <= kj + 1 + texel_slack + 1e-3)
        ok[i] = near and (r * (1 - 1e-4) <= rho <= r * (1 + tau) * (1 + 1e-4))
    ok[status != oracle.HIT] = ~np.isfinite(t[status != oracle.HIT])
    return ok

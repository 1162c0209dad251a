"""Degenerate rays on the GPU (tests/degenerate.py): axis-aligned and plane-diagonal
directions, rays through probe centres, rays on cell planes, rays from probe centres.
These are the exact ties the float margin exists for, so more of them may disagree than in
a random frame: every disagreeing ray must be in the oracle's margin, at most 1% may
disagree, and every HIT the GPU reports must be valid (tests/degenerate.py: the hit point
in the reported texel at a radial distance between r and r(1 + tau), the stored normal
facing the ray, and the texel the first to fire in the probe's traced interval)."""
import numpy as np
import pytest
import torch

import oracle
from conftest import workload
from degenerate import degenerate_rays, hit_is_valid
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,kw,seed", [("tiny", {}, 0), ("single", dict(size=(64, 64)), 0),
                                           ("single", dict(size=(64, 64)), 1)])
def test_degenerate_rays(name, kw, seed):
    import paper_2507_14624_amd as pt
    pt.load_library()
    scene, probes, views = workload(name, **kw)
    o, d, tag = degenerate_rays(scene, probes, seed=seed)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    res = pt.probe_trace_rays(grid, rad, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    res = {k: v.cpu().numpy() for k, v in res.items()}
    orc = oracle.trace(oracle.Grid.from_probes(probes), o.astype(np.float64), d.astype(np.float64))
    s = compare(res, orc)
    info = {k: v for k, v in s.items() if k != "disagree_idx"}
    print(f"[degenerate] {name} seed {seed}: {info}", flush=True)
    assert s["disagree_outside_margin"] == 0, info
    assert s["disagree"] <= 0.01 * s["n"], info
    valid = hit_is_valid(probes, o, d, res["status"], res["hit"], res["t"], 8.0 / probes.N)
    bad = np.nonzero(~valid)[0][:5]
    assert valid.all(), [dict(ray=int(i), tag=int(tag[i]), o=o[i].tolist(), d=d[i].tolist(),
                              gpu=(int(res["status"][i]), res["hit"][i].tolist(), float(res["t"][i])),
                              oracle=(int(orc["status"][i]), int(orc["probe"][i]), int(orc["texel"][i]),
                                      float(orc["t"][i]))) for i in bad]
    assert (res["status"] == orc["status"]).mean() >= 0.995

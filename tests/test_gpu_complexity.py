"""The trace over rooms of 3, 40 and 5,000 objects on one probe grid (8x8x4 probes): the
paper reports render times that do not grow with scene complexity (Results,
Reconstruction); the bench times the three rooms at 1080p.  Here, parity against the oracle
on each room, at reduced map and view size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import compare, assert_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [3, 40, 5000])
def test_trace_parity_over_scene_complexity(k):
    import paper_2507_14624_amd as pt
    pt.load_library()
    scene = synth.make_scene(1, (8, 8, 4), 1.0, (k, k))
    assert len(scene.obj_type) == k
    probes = synth.bake(scene, 64, 4)
    views = synth.make_views(scene, 101, 1, 240, 160)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    res = {kk: v.cpu().numpy() for kk, v in pt.probe_trace(grid, rad, views).items()}
    orc = oracle.trace_view(oracle.Grid.from_probes(probes), views[0].as_tuple())
    s = compare(res, orc)
    assert_parity(s, f"room of {k} objects")
    assert s["hit_frac"] > 0.8

"""Parity of the HIP trace on layouts of fewer than 8 probes (no grid iterator: every probe
per ray, closest to the eye first) against the oracle, forward and adjoint, through the
C ABI; and the layouts the library refuses."""
import numpy as np
import pytest
import torch

import oracle
from parity import compare, assert_parity
from test_gpu_backward import _check_grad
from test_oracle_few import LAYOUTS, few_room

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _setup(dims, **kw):
    pt = _pt()
    scene, probes, views = few_room(dims, **kw)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    return pt, scene, probes, views, grid, rad


# views of 320x200 (64,000 rays): the 1e-4 disagreement budget is a rate, which a test
# needs tens of thousands of rays to measure
PARITY_VIEW = (320, 200)


@pytest.mark.parametrize("dims", LAYOUTS)
def test_few_probe_layouts_match_oracle(dims):
    pt, scene, probes, views, grid, rad = _setup(dims, size=PARITY_VIEW)
    og = oracle.Grid.from_probes(probes)
    for label, opts in (("per-view", None), ("persistent", pt.trace_opts(flags=pt.PT_FLAG_PERSISTENT))):
        res = {k: v.cpu().numpy() for k, v in pt.probe_trace(grid, rad, views, opts).items()}
        orc = oracle.trace_view(og, views[0].as_tuple())
        s = compare(res, orc)
        assert_parity(s, f"{dims} {label}")
        assert s["hit_frac"] > 0.3


@pytest.mark.parametrize("dims", [(2, 1, 1), (3, 2, 1)])
def test_few_probe_arbitrary_rays_and_probe_limit(dims):
    # arbitrary rays (per-lane cage order) from the view's eye and from every probe centre;
    # and the one-probe limit (max_probes_per_cell = 1)
    pt, scene, probes, views, grid, rad = _setup(dims, size=PARITY_VIEW)
    og = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*views[0].as_tuple())
    rng = np.random.default_rng(4)
    pos = np.stack([og.probe_position(p) for p in range(probes.n_probes)])
    extra = rng.normal(size=(8000, 3))
    o = np.concatenate([o, pos[rng.integers(0, len(pos), 8000)]])
    d = np.concatenate([d, extra / np.linalg.norm(extra, axis=1, keepdims=True)])
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    for mp in (8, 1):
        opts = pt.trace_opts(max_probes_per_cell=mp)
        res = {k: v.cpu().numpy() for k, v in
               pt.probe_trace_rays(grid, rad, torch.from_numpy(o32).cuda(), torch.from_numpy(d32).cuda(),
                                   opts).items()}
        orc = oracle.trace(og, o32.astype(np.float64), d32.astype(np.float64), max_probes_per_cell=mp)
        assert_parity(compare(res, orc), f"{dims} rays max_probes={mp}")


@pytest.mark.parametrize("dims", [(2, 2, 1), (1, 1, 1)])
def test_few_probe_adjoint_matches_oracle(dims):
    pt, scene, probes, views, grid, rad = _setup(dims)
    _check_grad(pt, probes, grid, rad, views)
    _check_grad(pt, probes, grid, rad, views, flags=pt.PT_FLAG_PERSISTENT)


def test_layouts_the_library_refuses():
    pt = _pt()
    N = 16
    dist = torch.ones((8, N, N), device="cuda")
    nrm = torch.zeros((8, N, N, 2), dtype=torch.float16, device="cuda")
    with pytest.raises(pt.ProbeTraceError):
        pt.ProbeGrid((8, 1, 1), (0.5,) * 3, (1.0,) * 3, N, 2, (0, 0, 0), (8, 1, 1), dist, nrm)
    with pytest.raises(pt.ProbeTraceError):
        pt.ProbeGrid((4, 2, 1), (0.5,) * 3, (1.0,) * 3, N, 2, (0, 0, 0), (4, 2, 1), dist, nrm)
    # a hierarchy needs grids on both levels
    fine = pt.ProbeGrid((2, 2, 2), (0.5,) * 3, (1.0,) * 3, N, 2, (0, 0, 0), (2, 2, 2), dist, nrm)
    small = pt.ProbeGrid((2, 1, 1), (0.5,) * 3, (1.0,) * 3, N, 2, (0, 0, 0), (2, 2, 2), dist[:2], nrm[:2])
    with pytest.raises(pt.ProbeTraceError):
        fine.set_coarse(small, (0, 0, 0), (1, 1, 1))

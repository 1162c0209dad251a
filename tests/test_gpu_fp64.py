"""The trace in double precision (PT_FLAG_FP64) against the oracle, through the C ABI: the
same method, every decision taken in double, so disagreements with the oracle are left
only where a decision sits within double rounding of its threshold.  Workloads: the tiny
room, the 1080p room at reduced size, a few-probe layout, the two-level city block
(views and arbitrary rays), and the degenerate rays of the exact-tie tests."""
import numpy as np
import pytest
import torch

import oracle
from conftest import workload
from degenerate import degenerate_rays, hit_is_valid
from parity import compare, assert_parity

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _np(res):
    return {k: v.cpu().numpy() for k, v in res.items() if v is not None}


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("single", dict(size=(320, 180)))])
def test_fp64_views(name, kw):
    pt = _pt()
    scene, probes, views = workload(name, **kw)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    orc = oracle.trace_view(oracle.Grid.from_probes(probes), views[0].as_tuple())
    r64 = _np(pt.probe_trace(grid, rad, views[:1], pt.trace_opts(flags=pt.PT_FLAG_FP64)))
    s = compare(r64, orc)
    assert_parity(s, f"{name} FP64")
    assert s["disagree"] <= 1, s["disagree"]  # only decisions within double rounding may flip
    # and the FP32 trace of the same view agrees with it on all but a few rays
    r32 = _np(pt.probe_trace(grid, rad, views[:1]))
    same = (r32["status"] == r64["status"]) & (r32["hit"] == r64["hit"]).all(1)
    assert same.mean() >= 1 - 1e-3


def test_fp64_few_probes():
    from test_oracle_few import few_room
    pt = _pt()
    scene, probes, views = few_room((2, 2, 1), size=(320, 200))
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    orc = oracle.trace_view(oracle.Grid.from_probes(probes), views[0].as_tuple())
    r64 = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_FP64)))
    s = compare(r64, orc)
    assert_parity(s, "few (2,2,1) FP64")
    assert s["disagree"] <= 1


def test_fp64_two_level_views_and_rays():
    pt = _pt()
    scene, tl, views = workload("large_small")
    grid = pt.ProbeGrid.from_two_level(tl)
    rad = torch.from_numpy(tl.radiance().view(np.float16).copy()).cuda()
    og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
    o = np.concatenate([oracle.view_rays(*v.as_tuple())[0] for v in views])
    d = np.concatenate([oracle.view_rays(*v.as_tuple())[1] for v in views])
    orc = oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio))
    r64 = _np(pt.probe_trace(grid, rad, views, pt.trace_opts(flags=pt.PT_FLAG_FP64 | pt.PT_FLAG_PERSISTENT)))
    s = compare(r64, orc)
    assert_parity(s, "city views FP64")
    assert s["disagree"] <= 1
    # arbitrary rays, FP32 inputs widened to double on both sides
    import synth
    rng = np.random.default_rng(4)
    oo = []
    while len(oo) < 20000:  # free-space origins (clearance from every surface)
        p = rng.uniform([0.2, 0.2, 0.2], scene.room_max - 0.2)
        if synth.clearance(scene, p) > 0.05:
            oo.append(p)
    oo = np.array(oo, np.float32)
    dd = rng.normal(size=oo.shape).astype(np.float32)
    r64 = _np(pt.probe_trace_rays(grid, rad, torch.from_numpy(oo).cuda(), torch.from_numpy(dd).cuda(),
                                  pt.trace_opts(flags=pt.PT_FLAG_FP64)))
    orc = oracle.trace(og, oo.astype(np.float64), dd.astype(np.float64), coarse=(cg, tl.plane_off, tl.ratio))
    s = compare(r64, orc)
    assert_parity(s, "city rays FP64")
    assert s["disagree"] <= 2


def test_fp64_degenerate_rays():
    pt = _pt()
    scene, probes, views = workload("single", size=(64, 64))
    o, d, tag = degenerate_rays(scene, probes, seed=0)
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    res = _np(pt.probe_trace_rays(grid, rad, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(),
                                  pt.trace_opts(flags=pt.PT_FLAG_FP64)))
    orc = oracle.trace(oracle.Grid.from_probes(probes), o.astype(np.float64), d.astype(np.float64))
    s = compare(res, orc)
    print(f"[fp64 degenerate] {({k: v for k, v in s.items() if k != 'disagree_idx'})}", flush=True)
    assert s["disagree_outside_margin"] == 0
    valid = hit_is_valid(probes, o, d, res["status"], res["hit"], res["t"], 8.0 / probes.N)
    assert valid.all(), np.nonzero(~valid)[0][:10]
    # exact ties are still ties in double: fewer disagree than in FP32, none outside the margin
    assert s["disagree"] <= 0.01 * s["n"]


@pytest.mark.parametrize("kw", [dict(nearest=True), dict(thickness_rel=float("inf")), dict(max_probes_per_cell=2),
                                dict(thickness_rel=0.02, background=(0.25, 0.5, 1.0)),
                                dict(nearest=True, thickness_rel=float("inf"), max_probes_per_cell=2)],
                         ids=["nearest", "tau_inf", "two_probes", "tau_bg", "all_literal"])
def test_fp64_options(kw):
    # the trace options in double precision: nearest-texel radiance, the classification
    # without the shadow-entry rule, two cage probes per cell, a thin shell and a background
    pt = _pt()
    scene, probes, views = workload("single", size=(240, 135))
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    gkw = {k: v for k, v in kw.items() if k != "nearest"}
    gkw["flags"] = pt.PT_FLAG_FP64 | (pt.PT_FLAG_NEAREST if kw.get("nearest") else 0)
    r64 = _np(pt.probe_trace(grid, rad, views[:1], pt.trace_opts(**gkw)))
    orc = oracle.trace_view(oracle.Grid.from_probes(probes), views[0].as_tuple(), **kw)
    s = compare(r64, orc)
    assert_parity(s, f"FP64 {kw}")
    assert s["disagree"] <= 1
    if kw.get("nearest"):
        h = r64["status"] == oracle.HIT
        R = probes.radiance.view(np.float16).astype(np.float32).reshape(probes.n_probes, -1, 3)
        assert np.array_equal(r64["rgb"][h], R[r64["hit"][h, 0], r64["hit"][h, 1]])
    if "background" in kw:
        miss = r64["status"] != oracle.HIT
        assert miss.any() and np.all(r64["rgb"][miss] == np.float32(kw["background"]))

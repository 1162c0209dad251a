"""The paper's map configuration (Implementation Details: 2048 x 2048 maps and a 128 x 128
low-resolution map; Methodology, less than 8 probes): 4 probes of 2048^2 maps whose MIN
pyramid runs down to 128^2, the march starting at the 128^2 level.

Pins: the analytic scene at this resolution (the texel bound is 16 times tighter than at
128^2), and the flat march (no low-resolution map) against the two-map schedule and
every start level in between.
"""
import numpy as np

import oracle
from conftest import workload
from test_oracle_scene import _check


def test_paper_maps_against_analytic_scene():
    scene, probes, views = workload("paper", size=(160, 90))
    assert probes.N == 2048 and probes.levels == 5 and probes.n_probes == 4
    assert probes.N >> (probes.levels - 1) == 128
    s = _check(scene, probes, views[0])
    info = {k: v for k, v in s.items() if k != "r"}
    assert s["hit"] > 0.8 * s["n"], info
    assert s["checked"] > 0.6 * s["n"], info
    assert s["fails"] == 0, info


def test_low_resolution_map_changes_no_result():
    scene, probes, views = workload("paper", size=(120, 68))
    g = oracle.Grid.from_probes(probes)
    v = views[0].as_tuple()
    r = oracle.trace_view(g, v)  # starts at the 128^2 level, checked against the flat march
    hier = (r["margin"] & oracle.MG_HIER) != 0
    other = (r["margin"] & ~oracle.MG_HIER) != 0
    assert not np.any(hier & ~other)
    for top in (0, 2):
        r2 = oracle.trace_view(g, v, top_level=top)
        ok = (r["margin"] == 0) & (r2["margin"] == 0)
        assert ok.mean() > 0.3
        assert np.array_equal(r["status"][ok], r2["status"][ok])
        assert np.array_equal(r["texel"][ok], r2["texel"][ok])
        assert np.array_equal(r["t"][ok], r2["t"][ok])
    # the low-resolution map is what makes 2048^2 affordable: an order of magnitude fewer
    # texel tests than the flat march
    assert r["tests"].mean() < 0.15 * r["flat_tests"].mean()

"""The two-level city block at its full size (fine 64x64x16 + coarse 16x16x4 probes, 128^2
maps: ~17 GB of probe data, more than 4 GiB of pyramid, so the 64-bit addressing path),
traced in the launch form the benchmark times (8 views of 3840x2160, one graph-captured
persistent launch), checked against the oracle on sampled pixels.  Heavy: bakes the probes
on the host first (~1 minute) and holds ~40 GB of host memory while it runs."""
import gc

import numpy as np
import pytest
import torch

import oracle
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


def test_large_two_level_full_size_sampled_parity():
    import os
    import synth
    import paper_2507_14624_amd as pt
    pt.load_library()
    scene, tl, views = synth.workload("large", nthreads=min(16, os.cpu_count() or 1))
    assert tl.fine.n_probes == 64 * 64 * 16 and tl.coarse.n_probes == 16 * 16 * 4 and tl.fine.N == 128
    assert len(views) == 8 and views[0].width == 3840 and views[0].height == 2160
    grid = pt.ProbeGrid.from_two_level(tl)
    rad = torch.from_numpy(tl.radiance().view(np.float16)).cuda()
    opts = pt.trace_opts(flags=pt.PT_FLAG_GRAPH, tile=(4, 16), start_level=3)
    res = pt.probe_trace(grid, rad, views, opts)
    res = {k: v.cpu().numpy() for k, v in res.items()}
    del rad
    grid.close()
    torch.cuda.empty_cache()
    og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
    rng = np.random.default_rng(21)
    n = views[0].width * views[0].height
    o_all, d_all, sel = [], [], []
    for vi, v in enumerate(views):
        pix = np.sort(rng.choice(n, 1500, replace=False))
        o, d = oracle.view_rays(*v.as_tuple(), pixels=pix)
        o_all.append(o)
        d_all.append(d)
        sel.append(vi * n + pix)
    orc = oracle.trace(og, np.concatenate(o_all), np.concatenate(d_all), coarse=(cg, tl.plane_off, tl.ratio))
    s = compare(res, orc, sel=np.concatenate(sel))
    assert_parity(s, "large city, 8 x 3840x2160, 12k sampled rays")
    assert s["hit_frac"] > 0.9
    del og, cg, tl
    gc.collect()

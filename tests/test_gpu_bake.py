"""Probe baking from a point cloud on the GPU (probe_bake_points) against the oracle's
definition (oracle/points.py): the nearest point per texel is an integer decision taken in
FP32 with the same operations on both sides, so the maps must agree bit for bit; and the
GPU's maps are also held to a double-precision check that shares no part of that recipe
(a stored distance is never farther than a point binned to its texel in double)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import workload
from oracle.points import bake_points
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


def _pt():
    import paper_2507_14624_amd as pt
    pt.load_library()
    return pt


def _gpu_bake(probes, N, pts, col, nrm):
    pt = _pt()
    d, n, r = pt.probe_bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    return d.cpu().numpy(), n.cpu().numpy().view(np.uint16), r.cpu().numpy().view(np.uint16)


def _same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint32 if a.dtype == np.float32 else np.uint16),
                          np.ascontiguousarray(b).view(np.uint32 if b.dtype == np.float32 else np.uint16))


@pytest.mark.parametrize("normals", [True, False])
def test_bake_tiny_room_bit_exact(normals):
    scene, probes, views = workload("tiny")
    pts, col, nrm = synth.sample_points(scene, 300000, 21)
    nrm = nrm if normals else None
    gd, gn, gr = _gpu_bake(probes, 64, pts, col, nrm)
    od, on, orad, win = bake_points(probes.dims, probes.origin, probes.spacing, 64, pts, col, nrm)
    assert np.isnan(od).any() or np.isfinite(od).all()
    assert np.array_equal(np.isnan(gd), np.isnan(od))
    assert _same(gd, od) and _same(gn, on) and _same(gr, orad)
    assert np.isfinite(od).mean() > 0.9
    # and, independently of the FP32 recipe both sides share: bin a sample of the points
    # with the double-precision octahedral map and compare distances in double; the GPU's
    # stored distance of a texel is at most that of every point binned to it (points within
    # 1e-5 of a texel edge are left out: FP32 may bin them either way)
    from oracle.points import probe_origins
    O = probe_origins(probes.dims, probes.origin, probes.spacing).astype(np.float64)
    P64 = pts.astype(np.float64)[::11]
    N = 64
    for p in range(len(O)):
        d = P64 - O[p]
        r = np.linalg.norm(d, axis=1)
        uv = np.array([oracle.oct_encode(x) for x in d])
        x, y = (uv[:, 0] + 1) * N / 2, (uv[:, 1] + 1) * N / 2
        i, j = np.clip(np.floor(x), 0, N - 1).astype(int), np.clip(np.floor(y), 0, N - 1).astype(int)
        edge = (np.minimum(x - np.floor(x), np.ceil(x) - x) < 1e-5) | (np.minimum(y - np.floor(y), np.ceil(y) - y) < 1e-5)
        stored = gd[p][j, i].astype(np.float64)
        assert (edge | (stored <= r * (1 + 1e-6))).all(), p


def test_bake_room_sampled_probes_and_tiled_maps():
    # 256 probes at 128^2 (one LDS tile per map: every workgroup reads the whole cloud) and
    # 256^2 maps (four tiles per map: the points are binned per probe and tile first, and
    # 256 probes x 1.2M points take two batches of bins); the oracle bakes a sample of the
    # probes, from both batches
    scene, probes, views = workload("single", size=(64, 64))
    pts, col, nrm = synth.sample_points(scene, 1_200_000, 22)
    sel = np.array([0, 17, 100, 133, 200, 255])
    for N in (128, 256):
        gd, gn, gr = _gpu_bake(probes, N, pts, col, nrm)
        od, on, orad, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm, probes=sel)
        assert _same(gd[sel], od) and _same(gn[sel], on) and _same(gr[sel], orad), N


@pytest.mark.parametrize("name,N,n_points", [("tiny", 512, 300_000), ("paper", 2048, 2_000_000)])
def test_bake_binned_large_maps_bit_exact(name, N, n_points):
    # maps of 16 x 16 tiles (512^2 over 128^2 tiles) and the paper's 2048^2 maps (256 tiles
    # per map): the binned bake against the oracle's definition, every probe
    scene, probes, views = workload(name, size=(64, 64))
    pts, col, nrm = synth.sample_points(scene, n_points, 23)
    gd, gn, gr = _gpu_bake(probes, N, pts, col, nrm)
    od, on, orad, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    assert _same(gd, od) and _same(gn, on) and _same(gr, orad)
    assert np.isfinite(od).mean() > 0.2


def test_bake_empty_cloud_and_bad_arguments():
    pt = _pt()
    scene, probes, views = workload("tiny")
    z = np.zeros((0, 3), np.float32)
    d, n, r = pt.probe_bake_points(probes.dims, probes.origin, probes.spacing, 32, z, z)
    assert torch.isnan(d).all() and (n.view(torch.int16) == 0).all() and (r.view(torch.int16) == 0).all()
    pts = np.zeros((10, 3), np.float32)
    with pytest.raises(pt.ProbeTraceError):
        pt.probe_bake_points(probes.dims, probes.origin, probes.spacing, 48, pts, pts)  # not a power of 2
    with pytest.raises(pt.ProbeTraceError):
        pt.probe_bake_points(probes.dims, probes.origin, probes.spacing, 32, pts, pts[:5])  # size mismatch


def test_trace_of_a_point_cloud_bake():
    # bake on the GPU, build the grid from it, trace: parity with the oracle tracing the
    # oracle's own bake of the same cloud (the maps are identical, so this is the trace
    # parity on point-cloud data, with its empty texels)
    pt = _pt()
    scene, probes, views = workload("tiny")
    pts, col, nrm = synth.sample_points(scene, 300000, 23)
    N, L = 64, 4
    d, n, r = pt.probe_bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    grid = pt.ProbeGrid(probes.dims, probes.origin, probes.spacing, N, L, probes.scene_min, probes.scene_max, d, n)
    res = {k: v.cpu().numpy() for k, v in pt.probe_trace(grid, r, [views[0]]).items()}
    od, on, orad, win = bake_points(probes.dims, probes.origin, probes.spacing, N, pts, col, nrm)
    og = oracle.Grid(probes.dims, probes.origin, probes.spacing, N, L, probes.scene_min, probes.scene_max, od, on, orad)
    orc = oracle.trace_view(og, views[0].as_tuple())
    s = compare(res, orc)
    assert_parity(s, "tiny room 128x128 traced on a 300k-point cloud bake")
    assert s["hit_frac"] > 0.8

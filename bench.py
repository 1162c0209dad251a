"""Benchmark: probe-grid ray tracing on one MI355X.

One step = one full trace of the single-view workload: a seeded synthetic room of
20-40 boxes and spheres baked into an 8x8x4 grid of probes with 128x128 octahedral maps
(FP32 distance, FP16 normal and radiance, 5-level MIN pyramid), one 1920x1080 pinhole
view.  value = rays traced per second (Mrays/s), inputs resident in HBM.

Also reported: forward+backward Mrays/s on the same view (trace + radiance adjoint; the
soft-visibility trace and its adjoint),
the batched workload (64 views of uneven size in one persistent hipGraph launch) against
64 plain launches, the differentiable grid's training step kernel by kernel, the paper's
2048^2 maps (FP32 and FP64), the same grid over rooms of 3, 40 and 5,000 objects, the
two-level city block (8 views of 3840x2160), the HBM roofline of each workload's kernels
(algorithmic bytes from tests/golden/algorithmic_bytes.json over the measured launch
time, against 8 TB/s) and the CPU oracle timed on the host.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--autotune] [--legs LIST]

Launch options (tile shape, pyramid start level, launch form) come from the autotuner's
stored choice for each workload (paper_2507_14624_amd/tuned.json); --autotune re-tunes.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 78.6
BYTES_FILE = os.path.join(ROOT, "tests", "golden", "algorithmic_bytes.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trace_fwd_1080p_traffic.md")


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and spacing removed: a change of code, not
    of its comments, invalidates the committed counter summaries."""
    h = hashlib.sha256()
    for f in ("probetrace.hip", "trace_device.h", "bake_device.h"):
        with open(os.path.join(ROOT, "paper_2507_14624_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    s = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    if not m or not s or s.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


def measured_valu():
    """(VALU instructions per wavefront, wavefronts per launch) of the forward from the
    committed rocprofv3 counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    v = re.search(r"\| VALU instructions / wavefront \| ([0-9.]+) \|", text)
    w = re.search(r"\| wavefronts \| ([0-9]+) \|", text)
    s = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    if not v or not w or not s or s.group(1) != kernel_source_hash():
        return None
    return float(v.group(1)), int(w.group(1))


def hbm_roof(total_bytes, ms, kernel):
    """Algorithmic bytes of one launch over its measured duration, against HBM peak."""
    gbs = total_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "kernel": kernel, "algorithmic_bytes_per_launch": int(total_bytes),
            "ms": round(ms, 4)}


def algorithmic():
    with open(BYTES_FILE) as fh:
        return json.load(fh)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline(probes, view, large_kept=None):
    import numpy as np
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    g = oracle.Grid.from_probes(probes)
    o, d = oracle.view_rays(*view.as_tuple())
    t0 = time.perf_counter()
    r = oracle.trace(g, o, d, nthreads=threads)
    dt = time.perf_counter() - t0
    n = len(o)
    # one thread on every 8th ray of the frame
    t1 = time.perf_counter()
    oracle.trace(g, o[::8], d[::8], nthreads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=n / dt / 1e6, unit="Mrays/s", cores=threads, kind="oracle",
                sample=f"full {view.width}x{view.height} frame ({n} rays), double precision, {threads} threads, "
                       f"{dt:.1f} s", bytes_per_ray=float(oracle.algorithmic_bytes(r).mean()),
                one_thread={"value": len(o[::8]) / dt1 / 1e6, "unit": "Mrays/s",
                            "sample": f"every 8th ray of the frame ({len(o[::8])} rays), {dt1:.1f} s"},
                cpu_model=model, nproc=os.cpu_count(), other_workloads=cpu_other_workloads(threads, large_kept))


def cpu_other_workloads(threads, large_kept=None):
    """The oracle on the other workloads, on bounded samples: the tiny room in full, the
    batched walk on its first 4 views, the differentiable grid's forward and radiance
    VJP on 2 of its views, and (when the large leg ran and kept its host data) the two-level
    city on the central 256x256 pixels of its first view."""
    import numpy as np
    import oracle
    import synth
    out = {}

    def rays_of(views):
        parts = [oracle.view_rays(*v.as_tuple()) for v in views]
        return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])

    for name, nv, vjp in (("tiny", 1, False), ("batched", 4, False), ("diff", 2, True)):
        scene, probes, views = synth.workload(name, nthreads=threads)
        g = oracle.Grid.from_probes(probes)
        o, d = rays_of(views[:nv])
        t0 = time.perf_counter()
        r = oracle.trace(g, o, d, nthreads=threads)
        dt = time.perf_counter() - t0
        e = {"value": round(len(o) / dt / 1e6, 4), "unit": "Mrays/s", "rays": len(o), "s": round(dt, 2)}
        if vjp:
            t1 = time.perf_counter()
            oracle.vjp(g, r, np.ones((len(o), 3)))
            e["vjp_s"] = round(time.perf_counter() - t1, 2)
        out[name] = e
        del g
    if large_kept:
        tl, v = large_kept["tl"], large_kept["views"][0]
        og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
        o, d = oracle.view_rays(*v.as_tuple())
        x0, y0 = (v.width - 256) // 2, (v.height - 256) // 2
        pix = ((y0 + np.arange(256))[:, None] * v.width + x0 + np.arange(256)[None, :]).ravel()
        o = np.broadcast_to(o, d.shape)[pix] if o.ndim == 1 else o[pix]
        t0 = time.perf_counter()
        oracle.trace(og, np.ascontiguousarray(o), np.ascontiguousarray(d[pix]), coarse=(cg, tl.plane_off, tl.ratio),
                     nthreads=threads)
        dt = time.perf_counter() - t0
        out["large_crop"] = {"value": round(len(pix) / dt / 1e6, 4), "unit": "Mrays/s", "rays": len(pix),
                             "s": round(dt, 2), "sample": "central 256x256 pixels of the first 3840x2160 view"}
        del og, cg
    return out


def differentiable(pt, synth, torch, np, steps=5):
    """16x16x8 probes, 256^2 maps, 32 views of 512^2: Adam on FP32 master radiance against
    images of a second radiance field (same geometry, albedos redrawn)."""
    from paper_2507_14624_amd.differentiable import RadianceFit
    scene, probes, views = synth.workload("diff")
    target_probes = synth.bake(scene.with_albedos(synth.CONFIGS["diff"]["target_seed"]), probes.N, probes.levels)
    grid = pt.ProbeGrid.from_probes(probes)
    trad = torch.from_numpy(target_probes.radiance.view(np.float16).copy()).cuda()
    del target_probes
    target = pt.probe_trace(grid, trad, views, want_t=False, want_status=False, want_hit=False)["rgb"]
    del trad
    rays = pt.n_rays(views)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed_fit(keep_hits, optimizer="fused"):
        fit = RadianceFit(grid, views, target, keep_hits=keep_hits, optimizer=optimizer)
        for _ in range(3):  # warm-up on a throw-away fit
            fit.step()
        del fit
        fit = RadianceFit(grid, views, target, keep_hits=keep_hits, optimizer=optimizer)  # from the start
        losses = [fit.step().item()]
        torch.cuda.synchronize()
        e0.record()
        out = [fit.step() for _ in range(steps)]
        e1.record()
        torch.cuda.synchronize()
        return fit, e0.elapsed_time(e1) / steps, losses + [x.item() for x in out]

    # the default: adjoint from the forward's stored hits (no second trace) and the fused
    # Adam step writing the FP16 storage; then torch's Adam; then the recomputing adjoint
    fit, ms_sh, losses_sh = timed_fit(True)
    del fit
    fit, ms_ta, losses_ta = timed_fit(True, "torch")
    del fit
    fit, ms, losses = timed_fit(False)
    # the trace kernels alone in one step: forward and backward
    va = pt.make_views(views)
    g = torch.zeros((grid.P, grid.N, grid.N, 3), device="cuda")
    storage = fit.master.detach().to(torch.float16)
    gr = torch.randn((rays, 3), device="cuda")
    po = fit.opts  # the launch form the training step uses
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, storage, va, po, want_t=False, want_status=False, want_hit=False)
        pt.probe_trace_backward(grid, va, gr, g, po)
    e1.record()
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / steps
    hout = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"), None,
            torch.empty((rays, 2), dtype=torch.int32, device="cuda"))
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, storage, va, po, out=hout)
        pt.probe_trace_backward_hits(grid, va, hout[3], hout[1], gr, g, po)
    e1.record()
    torch.cuda.synchronize()
    ms_fh = e0.elapsed_time(e1) / steps

    def alone(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # each kernel of the step on its own, against its algorithmic bytes
    ab = algorithmic().get("diff_32x512")
    ms_k = {"forward": alone(lambda: pt.probe_trace(grid, storage, va, po, out=hout)),
            "adjoint_stored_hits": alone(lambda: pt.probe_trace_backward_hits(grid, va, hout[3], hout[1], gr, g, po)),
            "adjoint_recompute": alone(lambda: pt.probe_trace_backward(grid, va, gr, g, po))}
    m1, m2 = torch.zeros_like(fit.master), torch.zeros_like(fit.master)
    pm = fit.master.detach().clone()
    ms_k["adam"] = alone(lambda: pt.adam_step(pm, g.view(pm.shape), m1, m2, storage, 1, 1e-2))
    del m1, m2, pm
    kernels = {}
    if ab is not None:
        kernels = {"forward": hbm_roof(ab["total_bytes"], ms_k["forward"], "k_trace_persistent<false, 0>"),
                   "adjoint_stored_hits": hbm_roof(ab["adjoint_stored_hits_total_bytes"], ms_k["adjoint_stored_hits"],
                                                   "k_backward_hits<0>"),
                   "adjoint_recompute": hbm_roof(ab["adjoint_recompute_total_bytes"], ms_k["adjoint_recompute"],
                                                 "k_backward_persistent<false, 0, false>"),
                   "adam": hbm_roof(ab["adam_total_bytes"], ms_k["adam"], "k_adam_fp16")}
    del hout
    # gradient through the stored distances: forward (rgb and t) + distance adjoint
    del g
    gd = torch.zeros((grid.P, grid.N, grid.N), device="cuda")
    gt = torch.randn(rays, device="cuda")
    outs = pt._alloc_outputs(rays, gr.device, True, False, False)
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, storage, va, po, out=outs)
        pt.probe_trace_backward_distance(grid, storage, va, gr, gt, gd, po)
    e1.record()
    torch.cuda.synchronize()
    ms_geo = e0.elapsed_time(e1) / steps
    return {"workload": "16x16x8 probes, 256^2 maps (6 levels), 32 views of 512x512; FP32 master, FP16 storage; "
                        "Adam lr 1e-2 from 0.5",
            "rays_per_step": rays, "adam_step_ms": round(ms_sh, 3),
            "adam_step_mrays_s": round(rays / (ms_sh * 1e-3) / 1e6, 2),
            "fwd_bwd_kernels_ms": round(ms_fh, 3), "fwd_bwd_mrays_s": round(rays / (ms_fh * 1e-3) / 1e6, 2),
            "adjoint": "from the forward's hit and t outputs (12 B/ray kept: probe and texel as int32, t as FP32), no second trace",
            "optimizer": "pt_adam_step: Adam on the FP32 master writing the FP16 storage in one pass",
            "torch_adam": {"adam_step_ms": round(ms_ta, 3), "loss": [round(x, 6) for x in losses_ta],
                           "optimizer": "torch.optim.Adam (fused) + an FP16 rounding pass per forward"},
            "recompute": {"adam_step_ms": round(ms, 3), "adam_step_mrays_s": round(rays / (ms * 1e-3) / 1e6, 2),
                          "fwd_bwd_kernels_ms": round(ms_fb, 3),
                          "fwd_bwd_mrays_s": round(rays / (ms_fb * 1e-3) / 1e6, 2),
                          "loss": [round(x, 6) for x in losses],
                          "adjoint": "recomputes the trace"},
            "launch": "one persistent launch over the 32 views, forward and adjoint",
            "kernels_roofline": kernels,
            "geometry_fwd_bwd_kernels_ms": round(ms_geo, 3),
            "geometry_fwd_bwd_mrays_s": round(rays / (ms_geo * 1e-3) / 1e6, 2),
            "loss": [round(x, 6) for x in losses_sh]}


def bake(pt, synth, torch, np, n_points=4_000_000, steps=5):
    """Probe maps baked on the GPU from a 4M-point cloud sampled from the scene's surfaces
    (nearest point per texel): the 1080p room's 256 probes at 128^2 (one tile per map, every
    point against every probe), and the paper's 4 probes at 2048^2 (256 tiles per map, points
    binned per probe and tile first)."""
    res = {}
    for key, name in (("room", "single"), ("paper_maps", "paper")):
        scene, probes, views = synth.workload(name, size=(16, 16))
        pts, col, nrm = synth.sample_points(scene, n_points, 31)
        pts, col, nrm = (torch.from_numpy(a).cuda() for a in (pts, col, nrm))
        args = (probes.dims, probes.origin, probes.spacing, probes.N, pts, col, nrm)
        out = pt.probe_bake_points(*args)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            pt.probe_bake_points(*args)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        pairs = probes.n_probes * n_points
        res[key] = {"workload": f"{probes.n_probes} probes x {probes.N}^2 texels from {n_points} points",
                    "ms": round(ms, 3), "gpairs_s": round(pairs / (ms * 1e-3) / 1e9, 2),
                    "filled_texels": round(float(torch.isfinite(out[0]).float().mean()), 4)}
        del out, pts, col, nrm
    return res


def paper_maps(pt, synth, torch, np, steps=10):
    """The paper's map configuration: 4 probes (2x2x1, every probe per ray) of 2048^2 maps,
    the march starting at the 128^2 low-resolution level, one 1920x1080 frame; for
    comparison the flat march (no low-resolution map), and the trace in double precision."""
    scene, probes, views = synth.workload("paper")
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    va = pt.make_views(views)
    rays = pt.n_rays(views)
    out = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"),
           torch.empty(rays, dtype=torch.uint8, device="cuda"), None)
    res = {"workload": f"{probes.n_probes} probes (2x2x1) of {probes.N}^2 maps, pyramid to "
                       f"{probes.N >> (probes.levels - 1)}^2; room of {len(scene.obj_type)} objects; "
                       f"1 view of {views[0].width}x{views[0].height}", "rays": rays}
    # the FP32 trace from the low-resolution level and flat, and the double-precision trace
    # from the low-resolution level (the acceptance mode at these map sizes)
    for name, lvl, flags in (("low_res_128", probes.levels - 1, 0), ("flat", 0, 0),
                             ("low_res_128_fp64", probes.levels - 1, pt.PT_FLAG_FP64)):
        opts = pt.trace_opts(tile=(4, 16), start_level=lvl, flags=flags)
        ms, _ = time_steps(lambda: pt.probe_trace(grid, rad, va, opts, out=out), steps, 2, torch)
        res[name] = {"start_level": lvl, "value": round(rays / (ms * 1e-3) / 1e6, 2), "unit": "Mrays/s",
                     "ms_per_frame": round(ms, 4), "precision": "f64" if flags else "f32"}
    res["hit_frac"] = round(float((out[2] == 1).float().mean()), 4)
    return res


def large(pt, synth, torch, np, steps=3, keep=None):
    """Two-level city block: fine 64x64x16 + coarse 16x16x4 probes, 128^2 maps (~17 GB of
    probe data in HBM), 8 views of 3840x2160 in one graph-captured persistent launch;
    forward and forward + backward.  keep (a dict): receives the host-side hierarchy and
    views for the oracle's timing on a crop (the cpu leg)."""
    t0 = time.time()
    scene, tl, views = synth.workload("large", nthreads=min(16, os.cpu_count() or 1))
    bake_s = time.time() - t0
    grid = pt.ProbeGrid.from_two_level(tl)
    rad = torch.from_numpy(tl.radiance().view(np.float16)).cuda()
    P, N = tl.n_probes, tl.fine.N
    solid = [float((ps.distance.reshape(ps.n_probes, -1) <= 0).all(1).mean()) for ps in (tl.fine, tl.coarse)]
    n_boxes = len(scene.obj_type)
    if keep is not None:
        keep["tl"], keep["views"] = tl, views
    del tl
    va = pt.make_views(views)
    rays = pt.n_rays(views)
    opts = pt.trace_opts(flags=pt.PT_FLAG_GRAPH, tile=(4, 16), start_level=3)
    out = None
    res = pt.probe_trace(grid, rad, va, opts, want_t=False, want_status=True, want_hit=False)
    out = (res["rgb"], None, res["status"], None)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, rad, va, opts, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = out[2].cpu().numpy()
    hit_frac = float((st == 1).mean())
    gr = torch.ones((rays, 3), device="cuda")
    g = torch.zeros((P, N, N, 3), device="cuda")
    bopts = pt.trace_opts(tile=(4, 16), start_level=3)  # 8 views: one persistent adjoint launch
    pt.probe_trace_backward(grid, va, gr, g, bopts)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, rad, va, opts, out=out)
        pt.probe_trace_backward(grid, va, gr, g, bopts)
    e1.record()
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / steps
    hout = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"), None,
            torch.empty((rays, 2), dtype=torch.int32, device="cuda"))
    e0.record()
    for _ in range(steps):
        pt.probe_trace(grid, rad, va, opts, out=hout)
        pt.probe_trace_backward_hits(grid, va, hout[3], hout[1], gr, g, opts)
    e1.record()
    torch.cuda.synchronize()
    ms_fh = e0.elapsed_time(e1) / steps
    del hout
    ab = algorithmic().get("large_8x4k")
    roof = {}
    if ab is not None:
        roof = {"forward": hbm_roof(ab["total_bytes"], ms, "k_trace_persistent<true, 1>"),
                "bytes_per_ray": round(ab["bytes_per_ray"], 2), "sample": ab.get("sample")}
    return {"workload": f"city block of {n_boxes} boxes; fine 64x64x16 + coarse 16x16x4 probes (coarse planes = every "
                        f"4th fine plane), 128^2 maps, 5-level pyramids, {P} probes ({solid[0]:.0%} of the fine and "
                        f"{solid[1]:.0%} of the coarse inside buildings, D = 0); 8 views of 3840x2160", "rays": rays, "hbm_probe_bytes": int(P * N * N * (8 + 4 + 6)),
            "host_bake_s": round(bake_s, 1), "hit_frac": round(hit_frac, 4),
            "fwd": {"value": round(rays / (ms * 1e-3) / 1e6, 2), "unit": "Mrays/s", "ms": round(ms, 3),
                    "launch": "one graph-captured persistent launch over the 8 views"},
            "fwd_bwd": {"value": round(rays / (ms_fb * 1e-3) / 1e6, 2), "unit": "Mrays/s", "ms": round(ms_fb, 3)},
            "fwd_bwd_stored_hits": {"value": round(rays / (ms_fh * 1e-3) / 1e6, 2), "unit": "Mrays/s",
                                    "ms": round(ms_fh, 3)},
            "roofline": roof}


def complexity(pt, synth, torch, np, opts, steps=10):
    """The same probe grid (8x8x4 probes, 128^2 maps, 5 levels) over rooms of 3, 40 and
    5,000 objects (seed 1), one 1920x1080 view each (seed 101), the single-view options: the
    paper reports render times that do not grow with scene complexity."""
    out = {}
    for k in (3, 40, 5000):
        t0 = time.time()
        scene = synth.make_scene(1, (8, 8, 4), 1.0, (k, k))
        probes = synth.bake(scene, 128, 5, min(16, os.cpu_count() or 1))
        bake_s = time.time() - t0
        views = synth.make_views(scene, 101, 1, 1920, 1080)
        grid = pt.ProbeGrid.from_probes(probes)
        rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
        va = pt.make_views(views)
        rays = pt.n_rays(views)
        o = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"),
             torch.empty(rays, dtype=torch.uint8, device="cuda"), None)
        ms, _ = time_steps(lambda: pt.probe_trace(grid, rad, va, opts, out=o), steps, 3, torch)
        out[f"objects_{k}"] = {"value": round(rays / (ms * 1e-3) / 1e6, 2), "unit": "Mrays/s", "ms": round(ms, 4),
                               "hit_frac": round(float((o[2] == 1).float().mean()), 4),
                               "host_bake_s": round(bake_s, 1)}
        del grid, rad, o
    return out


LEGS = ("fwd_bwd", "batched", "diff", "bake", "paper", "complexity", "large", "cpu")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="workloads besides the single-view forward: " + ",".join(LEGS) + " (or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="leave out the leg 'cpu'")
    ap.add_argument("--no-large", action="store_true",
                    help="leave out the leg 'large' (it bakes ~20 GB of probes on the host first)")
    ap.add_argument("--no-autotune", action="store_true", help="library defaults instead of the tuned options")
    ap.add_argument("--autotune", action="store_true", help="re-run the autotuner and store its choice")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (scales HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (rays would shard by "
              "view, with the probe set replicated on every GPU).", file=sys.stderr)
        sys.exit(2)
    legs = set() if args.legs in ("", "none") else set(args.legs.split(","))
    unknown = legs - set(LEGS)
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if args.no_cpu_baseline:
        legs.discard("cpu")
    if args.no_large:
        legs.discard("large")

    import numpy as np
    import torch

    import paper_2507_14624_amd as pt
    import synth

    torch.cuda.set_device(0)
    print("[bench] building the single-view workload", file=sys.stderr, flush=True)
    scene, probes, views = synth.workload("single")
    view = views[0]
    grid = pt.ProbeGrid.from_probes(probes)
    rad = torch.from_numpy(probes.radiance.view(np.float16).copy()).cuda()
    rays = view.width * view.height
    va = pt.make_views([view])
    from paper_2507_14624_amd import tuning
    opts = pt.trace_opts() if args.no_autotune else tuning.options("single_1080p", grid, rad, va,
                                                                     retune=args.autotune)
    out = (torch.empty((rays, 3), device="cuda"), torch.empty(rays, device="cuda"),
           torch.empty(rays, dtype=torch.uint8, device="cuda"), torch.empty((rays, 2), dtype=torch.int32, device="cuda"))

    def fwd():
        pt.probe_trace(grid, rad, va, opts, out=out)

    print("[bench] timing forward", file=sys.stderr, flush=True)
    ms, wall = time_steps(fwd, args.steps, args.warmup, torch)
    value = rays / (ms * 1e-3) / 1e6

    allab = algorithmic()
    ab = allab["single_1080p"]
    achieved_tflops = ab["total_flops"] / (ms * 1e-3) / 1e12
    kernel = "k_trace_persistent<false, 0>" if opts.flags & pt.PT_FLAG_PERSISTENT else "k_trace_view<false, 0>"
    # The HBM roof: algorithmic bytes of one frame (the oracle's count on the reference
    # schedule) over the step's duration, which the HIP events around the steps measure on
    # the stream the library launches on (one k_cage_order and one trace launch per step).
    roof = hbm_roof(ab["total_bytes"], ms, kernel)
    roof["traffic"] = measured_traffic()
    roof["bytes_per_ray"] = round(ab["bytes_per_ray"], 2)
    roof["target_frac"] = 0.5
    roof["target_met"] = roof["frac"] >= 0.5
    # What bounds it in fact: vector-ALU issue (rocprofv3 SQ counters); the probe set is
    # cache resident.  FP32 peak without packed-FP32 instructions: 256 CUs x 64 lanes x 2
    # flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.
    roof["alu"] = {"achieved": round(achieved_tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(achieved_tflops / FP32_PEAK_TFLOPS, 5),
                   "algorithmic_flops_per_launch": ab["total_flops"], "flops_per_ray": round(ab["flops_per_ray"], 1)}
    result = {
        "metric": "Mrays/s probe trace (fwd, fwd+bwd) at 1080p; HBM GB/s vs peak; batched vs plain",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single view 1920x1080; seeded room (seed 1) of 26 boxes/spheres; 8x8x4 probes, "
                               "128x128 octahedral maps (FP32 distance, FP16 normal/radiance), 5-level min pyramid",
                   "rays_per_step": rays, "tile": [opts.tile_w, opts.tile_h], "start_level": opts.start_level,
                   "launch": "persistent" if opts.flags & pt.PT_FLAG_PERSISTENT else "per-view"},
        "roofline": roof,
    }
    valu = measured_valu()
    tiles = -(-view.width // opts.tile_w) * -(-view.height // opts.tile_h)  # one wavefront per tile
    if valu is not None and valu[1] == tiles:  # the profiled launch had this shape
        # issue time of the VALU instructions the counters saw (4 cycles per wave64
        # instruction on 1,024 SIMDs at 2.4 GHz) against this run's launch duration
        issue_ms = valu[0] * valu[1] * 4 / (1024 * 2.4e9) * 1e3
        result["roofline"]["valu_issue"] = {"instructions_per_launch": int(valu[0] * valu[1]),
                                            "issue_ms": round(issue_ms, 4), "frac": round(issue_ms / ms, 4),
                                            "source": "rocprofv3 SQ_INSTS_VALU (profiles/)"}
    if "fwd_bwd" in legs:
        gsz = (probes.n_probes, probes.N, probes.N, 3)
        grad = torch.zeros(gsz, device="cuda")
        gout = torch.randn((rays, 3), device="cuda")

        def fwd_bwd():
            pt.probe_trace(grid, rad, va, opts, out=out)
            grad.zero_()
            pt.probe_trace_backward(grid, va, gout, grad, opts)

        print("[bench] timing forward+backward", file=sys.stderr, flush=True)
        ms_fb, _ = time_steps(fwd_bwd, max(3, args.steps // 2), 1, torch)
        result["fwd_bwd"] = {"value": round(rays / (ms_fb * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                             "ms_per_step": round(ms_fb, 4), "adjoint": "recomputes the trace"}
        # the same step with the adjoint from the forward's stored hits (probe, texel, t)
        hout = (out[0], torch.empty(rays, device="cuda"), None, torch.empty((rays, 2), dtype=torch.int32, device="cuda"))

        def fwd_bwd_hits():
            pt.probe_trace(grid, rad, va, opts, out=hout)
            grad.zero_()
            pt.probe_trace_backward_hits(grid, va, hout[3], hout[1], gout, grad, opts)

        ms_fh, _ = time_steps(fwd_bwd_hits, max(3, args.steps // 2), 1, torch)
        result["fwd_bwd_stored_hits"] = {"value": round(rays / (ms_fh * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                                         "ms_per_step": round(ms_fh, 4),
                                         "adjoint": "from the forward's hit and t outputs (12 B/ray kept: probe and "
                                                    "texel as int32, t as FP32)"}
        ms_a, _ = time_steps(lambda: pt.probe_trace_backward_hits(grid, va, hout[3], hout[1], gout, grad, opts),
                             max(3, args.steps // 2), 1, torch)
        result["fwd_bwd_stored_hits"]["adjoint_roofline"] = hbm_roof(ab["adjoint_stored_hits_total_bytes"], ms_a,
                                                                     "k_backward_hits<0>")
        # soft visibility on the same view: the relaxed forward, and forward + its adjoint
        # into both the distances and the radiance
        sigma = 0.05
        srgb = torch.empty((rays, 3), device="cuda")
        gdist = torch.zeros((probes.n_probes, probes.N, probes.N), device="cuda")
        ms_sf, _ = time_steps(lambda: pt.probe_trace_soft(grid, rad, va, sigma, opts, out=srgb),
                              max(3, args.steps // 2), 1, torch)

        def soft_fwd_bwd():
            pt.probe_trace_soft(grid, rad, va, sigma, opts, out=srgb)
            pt.probe_trace_soft_backward(grid, rad, va, sigma, srgb, gout, gdist, grad, opts)

        ms_sb, _ = time_steps(soft_fwd_bwd, max(3, args.steps // 2), 1, torch)
        result["soft"] = {"sigma": sigma,
                          "fwd": {"value": round(rays / (ms_sf * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                                  "ms": round(ms_sf, 4)},
                          "fwd_bwd": {"value": round(rays / (ms_sb * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                                      "ms": round(ms_sb, 4), "adjoint": "distances and radiance"}}
    if "batched" in legs:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        _, _, bviews = synth.workload("batched")
        bva = pt.make_views(bviews)
        brays = pt.n_rays(bviews)
        bout = (torch.empty((brays, 3), device="cuda"), None, None, None)
        # the 64-view launch tuned on its own views, starting from the graph launch form
        gopts = pt.trace_opts() if args.no_autotune else tuning.options(
            "batched_64", grid, rad, bva, retune=args.autotune, flags=pt.PT_FLAG_GRAPH)
        gopts.flags |= pt.PT_FLAG_GRAPH
        popts = pt.trace_opts(tile=(gopts.tile_w, gopts.tile_h), start_level=gopts.start_level)  # per view
        ms_g, _ = time_steps(lambda: pt.probe_trace(grid, rad, bva, gopts, out=bout), 3, 1, torch)
        ms_p, _ = time_steps(lambda: pt.probe_trace(grid, rad, bva, popts, out=bout), 3, 1, torch)
        bab = allab.get("batched_64")
        result["batched"] = {"views": len(bviews), "rays": brays,
                             "options": {"tile": [gopts.tile_w, gopts.tile_h], "start_level": gopts.start_level,
                                         "flags": int(gopts.flags)},
                             "graph_persistent": {"value": round(brays / (ms_g * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                                                  "ms": round(ms_g, 3)},
                             "plain_launches": {"value": round(brays / (ms_p * 1e-3) / 1e6, 3), "unit": "Mrays/s",
                                                "ms": round(ms_p, 3)},
                             "roofline": hbm_roof(bab["total_bytes"], ms_g, "k_trace_persistent<false, 0>")
                             if bab else None}
    if "diff" in legs:
        print("[bench] differentiable workload", file=sys.stderr, flush=True)
        result["differentiable"] = differentiable(pt, synth, torch, np)
    if "bake" in legs:
        print("[bench] point-cloud bake", file=sys.stderr, flush=True)
        result["bake"] = bake(pt, synth, torch, np)
    if "paper" in legs:
        print("[bench] paper map configuration", file=sys.stderr, flush=True)
        result["paper_maps"] = paper_maps(pt, synth, torch, np)
    if "complexity" in legs:
        print("[bench] scene complexity", file=sys.stderr, flush=True)
        result["complexity"] = complexity(pt, synth, torch, np, opts)
    large_kept = {} if "cpu" in legs else None
    if "large" in legs:
        print("[bench] large two-level workload", file=sys.stderr, flush=True)
        result["large"] = large(pt, synth, torch, np, keep=large_kept)
    if "cpu" in legs:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cb = cpu_baseline(probes, view, large_kept)
        large_kept = None
        cb["one_thread"]["value"] = round(cb["one_thread"]["value"], 4)  # other_workloads are rounded already
        result["cpu_baseline"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in cb.items()}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Write algorithmic_bytes.json: per-ray algorithmic bytes and FP32 operations of each
benchmark workload, counted by the oracle running the reference hierarchical schedule
(start at the coarsest pyramid level, descend on fire, move up after a non-firing step
that leaves the parent, stop at the first level-0 fire):

    forward(ray)             = 4 * distance/mip fetches + 4 * normal fetches
                               + 24 * [HIT] + 17
    adjoint, recomputed      = forward - 17 + [HIT] * (12 + 96)
    adjoint, from stored hits = 8 + [HIT] * (4 + 12 + 96)

(4 B FP32 texel; 4 B packed FP16 normal; 4 bilinear taps x RGB FP16; rgb FP32 + t FP32 +
status u8 written; the adjoints read grad_rgb (12 B) of a HIT ray and add into 4 taps x 3
channels of the FP32 gradient, 8 B of read-modify-write each; the stored-hit adjoint reads
every ray's (probe, texel) and a HIT ray's t instead of tracing), and FP32 operations from
oracle.FLOPS times the oracle's counts of texel tests, pieces, probe traces, cells and
hits.  The Adam step of the radiance fit moves 30 B per texel (read master, gradient, two
moments; write master, moments, FP16 storage).

Calls only the oracle and the seeded input generator.

    python tests/golden/make_algorithmic_bytes.py [--workloads single,batched,diff,large]
                                                  [--stride K] [--threads T] [--out FILE]

large: the 8 views of 3840x2160 are sampled on every K-th pixel in x and y (default 8)
and the per-ray means scaled to the whole launch; it bakes ~20 GB of probes on the host.
Entries already in the output file for other workloads are kept.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

ADAM_BYTES_PER_TEXEL_CHANNEL = 30


def _adjoint_bytes(r):
    hit = (r["status"] == oracle.HIT).astype(np.int64)
    fwd = oracle.algorithmic_bytes(r)
    return fwd - 17 + hit * (12 + 96), 8 + hit * (4 + 12 + 96)


def _summary(r, rays_total=None):
    """Means per ray of the oracle's result r, and launch totals over rays_total rays (all
    of r's rays unless given: then r is a sample of the launch)."""
    b = oracle.algorithmic_bytes(r)
    f = oracle.algorithmic_flops(r)
    br, bh = _adjoint_bytes(r)
    n = len(b) if rays_total is None else int(rays_total)
    scale = n / len(b)
    return {
        "rays": n, "rays_counted": int(len(b)),
        "total_bytes": int(round(b.sum() * scale)), "bytes_per_ray": float(b.mean()),
        "total_flops": int(round(f.sum() * scale)), "flops_per_ray": float(f.mean()), "flops_model": oracle.FLOPS,
        "adjoint_recompute_total_bytes": int(round(br.sum() * scale)),
        "adjoint_recompute_bytes_per_ray": float(br.mean()),
        "adjoint_stored_hits_total_bytes": int(round(bh.sum() * scale)),
        "adjoint_stored_hits_bytes_per_ray": float(bh.mean()),
        "probe_traces_per_ray": float(r["work"][:, 0].mean()), "pieces_per_ray": float(r["work"][:, 1].mean()),
        "cells_per_ray": float(r["work"][:, 2].mean()),
        "distance_fetches_per_ray": float(r["tests"].mean()), "normal_fetches_per_ray": float(r["normals"].mean()),
        "hit_fraction": float((r["status"] == oracle.HIT).mean()),
        "flat_level0_fetches_per_ray": float(r["flat_tests"].mean()),
        "margin_fraction": float((r["margin"] != 0).mean()),
        "resolving_rank_histogram": np.bincount(r["rank"][r["rank"] >= 0] % 8, minlength=8).tolist(),
    }


def _concat(results):
    return {k: np.concatenate([r[k] for r in results]) for k in results[0]}


def single(threads):
    scene, probes, views = synth.workload("single", nthreads=threads)
    v = views[0]
    r = oracle.trace_view(oracle.Grid.from_probes(probes), v.as_tuple(), nthreads=threads)
    out = _summary(r)
    out.update(view=[v.width, v.height], scene_seed=scene.seed, N=probes.N, levels=probes.levels)
    return out


def batched(threads):
    scene, probes, views = synth.workload("batched", nthreads=threads)
    g = oracle.Grid.from_probes(probes)
    out = _summary(_concat([oracle.trace_view(g, v.as_tuple(), nthreads=threads) for v in views]))
    out.update(views=len(views), scene_seed=scene.seed, N=probes.N, levels=probes.levels)
    return out


def diff(threads):
    scene, probes, views = synth.workload("diff", nthreads=threads)
    g = oracle.Grid.from_probes(probes)
    out = _summary(_concat([oracle.trace_view(g, v.as_tuple(), nthreads=threads) for v in views]))
    texels = probes.n_probes * probes.N * probes.N * 3
    out.update(views=len(views), scene_seed=scene.seed, N=probes.N, levels=probes.levels,
               adam_texel_channels=texels, adam_total_bytes=ADAM_BYTES_PER_TEXEL_CHANNEL * texels,
               adam_bytes_per_texel_channel=ADAM_BYTES_PER_TEXEL_CHANNEL)
    return out


def large(threads, stride):
    print("[bytes] large: baking the two-level city block", file=sys.stderr, flush=True)
    scene, tl, views = synth.workload("large", nthreads=threads)
    og, cg = oracle.Grid.from_probes(tl.fine), oracle.Grid.from_probes(tl.coarse)
    parts = []
    rays = 0
    for k, v in enumerate(views):
        print(f"[bytes] large: view {k + 1} of {len(views)}", file=sys.stderr, flush=True)
        W, H = v.width, v.height
        rays += W * H
        yy, xx = np.meshgrid(np.arange(stride // 2, H, stride), np.arange(stride // 2, W, stride), indexing="ij")
        o, d = oracle.view_rays(*v.as_tuple(), pixels=(yy * W + xx).ravel())
        parts.append(oracle.trace(og, o, d, coarse=(cg, tl.plane_off, tl.ratio), nthreads=threads))
    out = _summary(_concat(parts), rays_total=rays)
    out.update(views=len(views), sample=f"every {stride}th pixel in x and y of each view", scene_seed=scene.seed,
               N=tl.fine.N, levels=tl.fine.levels, probes=tl.n_probes)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="single,batched,diff")
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(HERE, "algorithmic_bytes.json"))
    args = ap.parse_args()
    data = {}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            data = json.load(fh)
    names = {"single": "single_1080p", "batched": "batched_64", "diff": "diff_32x512", "large": "large_8x4k"}
    for w in args.workloads.split(","):
        t0 = time.time()
        print(f"[bytes] {w}", file=sys.stderr, flush=True)
        data[names[w]] = large(args.threads, args.stride) if w == "large" else globals()[w](args.threads)
        print(f"[bytes] {w}: {data[names[w]]['bytes_per_ray']:.2f} B/ray ({time.time() - t0:.0f} s)",
              file=sys.stderr, flush=True)
    tmp = args.out + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1)
    os.replace(tmp, args.out)


if __name__ == "__main__":
    main()

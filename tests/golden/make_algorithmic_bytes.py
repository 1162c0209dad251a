"""Write algorithmic_bytes.json: per-ray algorithmic bytes and FP32 operations of the
benchmark workload,
counted by the oracle running the reference hierarchical schedule (start at the coarsest
pyramid level, descend on fire, move up after a non-firing step that leaves the parent,
stop at the first level-0 fire):

    bytes(ray) = 4 * distance/mip fetches + 4 * normal fetches + 24 * [HIT] + 17

(4 B FP32 texel; 4 B packed FP16 normal; 4 bilinear taps x RGB FP16; rgb FP32 + t FP32 +
status u8 written), and FP32 operations from oracle.FLOPS times the oracle's counts of
texel tests, pieces, probe traces, cells and hits.  Calls only the oracle and the seeded
input generator.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    scene, probes, views = synth.workload("single")
    v = views[0]
    g = oracle.Grid.from_probes(probes)
    r = oracle.trace_view(g, v.as_tuple())
    b = oracle.algorithmic_bytes(r)
    f = oracle.algorithmic_flops(r)
    out = {"single_1080p": {
        "rays": int(len(b)), "total_bytes": int(b.sum()), "bytes_per_ray": float(b.mean()),
        "total_flops": int(f.sum()), "flops_per_ray": float(f.mean()), "flops_model": oracle.FLOPS,
        "probe_traces_per_ray": float(r["work"][:, 0].mean()), "pieces_per_ray": float(r["work"][:, 1].mean()),
        "cells_per_ray": float(r["work"][:, 2].mean()),
        "distance_fetches_per_ray": float(r["tests"].mean()), "normal_fetches_per_ray": float(r["normals"].mean()),
        "hit_fraction": float((r["status"] == oracle.HIT).mean()),
        "flat_level0_fetches_per_ray": float(r["flat_tests"].mean()),
        "margin_fraction": float((r["margin"] != 0).mean()),
        "resolving_rank_histogram": np.bincount(r["rank"][r["rank"] >= 0] % 8, minlength=8).tolist(),
        "view": [v.width, v.height], "scene_seed": scene.seed, "N": probes.N, "levels": probes.levels}}
    with open(os.path.join(HERE, "algorithmic_bytes.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

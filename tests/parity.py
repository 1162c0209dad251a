"""GPU-vs-oracle comparison used by the parity tests.

Acceptance (per ray, GPU FP32 against the double-precision oracle on the same seeded
inputs):
* "agree" = same status and, for HIT, same probe, same level-0 texel,
  |t_gpu - t_oracle| <= 1e-4 t_oracle and |rgb_gpu - rgb_oracle| <= 1e-3 (non-HIT rays:
  rgb equal to the background within 1e-3, t = +inf);
* at most 1e-4 of the rays may disagree (no floor: a test of fewer than 10^4 rays
  allows none), and every disagreeing ray must be flagged by the oracle as inside the
  float margin (a decision within its stated unit roundoff of flipping, or a hit distance
  FP32 cannot resolve to 1e-4 t);
* every disagreeing ray whose hit distance is well conditioned must have a decision
  within 1e-7 (relative to its error scale) of flipping: a gap FP32 cannot resolve.
"""
import numpy as np

import oracle

T_REL = 1e-4
RGB_ABS = 1e-3
MAX_DISAGREE = 1e-4
MAX_SCORE = 1e-7


def compare(gpu: dict, orc: dict, sel=None) -> dict:
    """gpu: numpy arrays status [n], t [n], rgb [n,3], hit [n,2]; orc: oracle.trace output.

    A ray agrees when status, probe and texel match and, for HIT, t and rgb are within
    tolerance; otherwise it counts against the disagreement budget and must lie inside
    the oracle's float margin."""
    pick = (lambda a: a[sel]) if sel is not None else (lambda a: a)
    st_g = pick(gpu["status"]).astype(np.int64)
    st_o = orc["status"].astype(np.int64)
    n = len(st_o)
    hit_g, t_g, rgb_g = pick(gpu["hit"]), pick(gpu["t"]), pick(gpu["rgb"])
    both_hit = (st_g == oracle.HIT) & (st_o == oracle.HIT)
    cls = (st_g == st_o) & (~both_hit | ((hit_g[:, 0] == orc["probe"]) & (hit_g[:, 1] == orc["texel"])))
    trel = np.zeros(n)
    rgb_err = np.zeros(n)
    h = cls & both_hit
    trel[h] = np.abs(t_g[h].astype(np.float64) - orc["t"][h]) / np.maximum(orc["t"][h], 1e-30)
    rgb_err[h] = np.abs(rgb_g[h].astype(np.float64) - orc["rgb"][h]).max(axis=1)
    nh = cls & ~both_hit
    rgb_err[nh] = np.abs(rgb_g[nh].astype(np.float64) - orc["rgb"][nh]).max(axis=1)
    t_bad = h & (trel > T_REL)
    rgb_bad = cls & (rgb_err > RGB_ABS)
    agree = cls & ~t_bad & ~rgb_bad
    dis = ~agree
    margin = orc["margin"] != 0
    thit = (orc["margin"] & oracle.MG_THIT) != 0
    return dict(
        n=n,
        disagree=int(dis.sum()),
        disagree_frac=float(dis.mean()) if n else 0.0,
        disagree_outside_margin=int((dis & ~margin).sum()),
        disagree_class=int((~cls).sum()),
        disagree_t=int(t_bad.sum()),
        disagree_rgb=int(rgb_bad.sum()),
        disagree_idx=np.nonzero(dis)[0],
        margin_frac=float(margin.mean()) if n else 0.0,
        hit_frac=float((st_o == oracle.HIT).mean()) if n else 0.0,
        t_rel_max_agreeing=float(trel[agree & both_hit].max()) if (agree & both_hit).any() else 0.0,
        rgb_abs_max_agreeing=float(rgb_err[agree].max()) if agree.any() else 0.0,
        t_nonhit_finite=int(np.isfinite(t_g[st_g != oracle.HIT]).sum()),
        # the closest call among the disagreeing rays: the smallest relative gap of a decision
        # to its threshold (FP32 resolves about 1e-7)
        score_max_disagreeing=float(orc["score"][dis].max()) if ("score" in orc and dis.any()) else 0.0,
        # the same over the disagreeing rays whose hit distance is well conditioned
        score_max_disagreeing_nonthit=float(orc["score"][dis & ~thit].max()) if (dis & ~thit).any() else 0.0,
        disagree_thit=int((dis & thit).sum()),
    )


def assert_parity(s: dict, label: str = "", max_frac: float = MAX_DISAGREE, max_score: float = MAX_SCORE):
    """The acceptance above: every disagreeing ray in the margin, at most `max_frac` of the
    rays disagreeing, and every disagreeing ray with a well-conditioned hit distance within
    `max_score` of flipping a decision."""
    info = {k: v for k, v in s.items() if k != "disagree_idx"}
    print(f"[parity] {label} {info}", flush=True)
    assert s["disagree_outside_margin"] == 0, (label, info)
    assert s["disagree"] <= max_frac * s["n"], (label, info)
    assert s["t_nonhit_finite"] == 0, (label, info)
    assert s["score_max_disagreeing_nonthit"] <= max_score, (label, info)

"""Cache of autotuned launch options per workload.

probe_autotune (native, in the library) times tile shapes, pyramid start levels and the
launch form on the caller's views.  Tuning once and reusing the choice keeps every later
run launching exactly the same kernels; this module stores the choices in tuned.json
beside the package, keyed by a workload name.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")

_FIELDS = ("tile_w", "tile_h", "start_level", "flags")


def load(key: str):
    """Stored options for `key` as a dict, or None."""
    if not os.path.exists(TUNED):
        return None
    with open(TUNED) as fh:
        return json.load(fh).get(key)


def save(key: str, opts, note: str = "") -> dict:
    data = {}
    if os.path.exists(TUNED):
        with open(TUNED) as fh:
            data = json.load(fh)
    entry = {f: int(getattr(opts, f)) for f in _FIELDS}
    if note:
        entry["note"] = note
    data[key] = entry
    tmp = TUNED + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, TUNED)
    return entry


def apply(opts, entry: dict):
    """Copy a stored choice into a PtTraceOpts."""
    for f in _FIELDS:
        setattr(opts, f, int(entry[f]))
    return opts


def options(key: str, grid, radiance_half, views, retune: bool = False, flags: int = 0):
    """Stored options for `key`, tuning (and storing) them first if absent or asked.
    `flags` is the launch form the tuner starts from (PT_FLAG_GRAPH is kept)."""
    from . import probe_autotune, trace_opts
    entry = None if retune else load(key)
    if entry is not None:
        return apply(trace_opts(), entry)
    opts = probe_autotune(grid, radiance_half, views, trace_opts(flags=flags))
    save(key, opts, note=f"probe_autotune on MI355X over {len(views)} view(s)")
    return opts

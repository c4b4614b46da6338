"""Column-tile autotuner for FCN plans.

The column pass has two tile parameters: W, the adjacent frequencies per workgroup, and L,
the rows each thread eliminates (include/fcn.h, fcn_options.col_tile / col_rows).  The best
pair depends on the grid shapes of the batch and on the precision.  `tune` times every
built pair on the GPU with the kernels' own start/end events (fcn_step_timed) and picks the
fastest column pass; results can be cached in a JSON file keyed by precision and the
multiset of grid shapes, so a later plan of the same shapes reuses the choice.
"""
from __future__ import annotations

import json
import os
import tempfile

import numpy as np

# (W, L) pairs built into the library; FP64 arithmetic (also the column solve of fp32_cn64)
# keeps L = 8 (L = 16 needs twice the registers of the FP32 solve and spills)
CANDIDATES = {
    "fp32": [(4, 8), (4, 16), (8, 8), (8, 16), (16, 8), (16, 16), (32, 8), (2, 16), (1, 16)],
    "fp64": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8)],
    "fp32_storage": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8)],
    "fp32_cn64": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8)],
}
MAX_THREADS = 512


def shape_key(instances, precision: str) -> str:
    shapes = sorted((int(i["nr"]), int(i["nt"])) for i in instances)
    return precision + "|" + ",".join(f"{nr}x{nt}" for nr, nt in shapes)


def fits(w: int, l: int, nr_max: int) -> bool:
    """A workgroup holds W * ceil(nr / L) threads, at most 512."""
    return w * ((nr_max + l - 1) // l) <= MAX_THREADS


def select(candidates, measure):
    """measure(w, l) -> mean column-pass milliseconds, or None if the pair cannot run.
    Returns (best (w, l), {"WxL": ms}).  Ties keep the earlier candidate."""
    table = {}
    best, best_ms = None, float("inf")
    for w, l in candidates:
        ms = measure(w, l)
        if ms is None:
            continue
        table[f"{w}x{l}"] = ms
        if ms < best_ms:
            best, best_ms = (w, l), ms
    if best is None:
        raise RuntimeError("no column tile could be measured")
    return best, table


def load_cache(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def store_cache(path, cache):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(instances, precision: str = "fp32", steps: int = 20, repeats: int = 3, cache_path=None, log=None):
    """Times every candidate column tile for `instances` and returns
    {"col_tile": W, "col_rows": L, "col_ms": ms, "table": {...}, "cached": bool}."""
    from . import fcn
    from . import workloads as wl

    if isinstance(instances, dict):
        instances = [instances]
    key = shape_key(instances, precision)
    cache = load_cache(cache_path)
    if key in cache:
        r = dict(cache[key])
        r["cached"] = True
        return r
    nr_max = max(int(i["nr"]) for i in instances)
    dt = np.complex128 if precision == "fp64" else np.complex64
    fields = [wl.gaussian_field(i, dt) if "I0" in i else wl.random_field(int(i["nr"]), int(i["nt"]), 0, dtype=dt)
              for i in instances]
    seen = {}

    def measure(w, l):
        if not fits(w, l, nr_max):
            return None
        try:
            plan = fcn.Plan(instances, precision=precision, col_tile=w, col_rows=l)
        except fcn.FcnError:
            return None
        actual = plan.tiles()[:2]
        if actual in seen:  # the runtime adjusted the request to a pair already timed
            return None
        f = plan.pack(fields)
        plan.step(f, 2)
        ms = float(np.median([plan.step_timed(f, steps)[1] for _ in range(repeats)]))
        plan.sync()
        seen[actual] = ms
        if log:
            log(f"col tile {w}x{l}: {ms * 1e3:.2f} us")
        return ms

    (w, l), table = select(CANDIDATES[precision], measure)
    r = {"col_tile": w, "col_rows": l, "col_ms": table[f"{w}x{l}"], "table": table}
    if cache_path:
        cache[key] = r
        store_cache(cache_path, cache)
    r["cached"] = False
    return r


def tuned_plan(instances, precision: str = "fp32", cache_path=None, **kw):
    """An fcn.Plan with the column tile chosen by `tune`."""
    from . import fcn

    t = tune(instances, precision, cache_path=cache_path)
    return fcn.Plan(instances, precision=precision, col_tile=t["col_tile"], col_rows=t["col_rows"], **kw)

"""Column-tile autotuner for FCN plans, per radial bucket.

The column pass has two tile parameters: W, the frequency pairs (p, nt - p) per workgroup, and
L, the rows each thread eliminates (include/fcn.h, fcn_options.col_tile / col_rows).  A ragged
plan launches the column pass once per distinct nr, and the best pair depends on nr and on the
precision.  `tune` runs every built pair on the GPU, times every launch of the step with the
kernels' own start/end events (fcn_step_timed_launches), and picks the fastest pair for each nr
separately.  The choice is kept in a tune cache, a text file the library itself reads
(fcn_options.tune_cache): one line per (precision, nr), "<precision> col <nr> <W> <L> <us>", so a
later plan of the same precision and radial sizes takes its tiles from the file with no tuning.

The row kernel's configuration (elements per thread, rows per workgroup) follows a fixed rule
in the library: 16 elements per thread from nt = 4096 (and nt = 2048 with FP64 arithmetic), 8
below; 16 at nt = 1024 and 2048 with FP32 arithmetic measured no faster on the batched sweep
(88 and 174 against 88 and 155 us), so it is not a tuned parameter.
"""
from __future__ import annotations

import os
import tempfile

import numpy as np

# (W, L) pairs built into the library; FP64 arithmetic (also the column solve of fp32_cn64)
# takes L = 8, 6 or 4 (L = 16 needs twice the registers of the FP32 solve and spills; L = 6 keeps
# three wavefronts per SIMD, L = 4 four)
CANDIDATES = {
    "fp32": [(4, 8), (4, 16), (8, 8), (8, 16), (16, 8), (16, 16), (32, 8), (2, 16), (1, 16), (2, 8), (1, 8),
             (8, 4), (4, 4), (2, 4)],
    "fp64": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8), (8, 6), (4, 6), (2, 6), (1, 6),
             (8, 4), (4, 4), (2, 4), (1, 4)],
    "fp32_storage": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8), (8, 6), (4, 6), (2, 6), (1, 6),
                     (8, 4), (4, 4), (2, 4), (1, 4)],
    "fp32_cn64": [(4, 8), (8, 8), (16, 8), (32, 8), (2, 8), (1, 8), (8, 6), (4, 6), (2, 6), (1, 6),
                  (8, 4), (4, 4), (2, 4), (1, 4)],
}
MAX_THREADS = 512


def system_lengths(instances) -> set:
    """Lengths of the column pass's tridiagonal systems: nr of a radial instance, nx and ny of
    a Cartesian one (its x and y solves)."""
    out = set()
    for i in instances:
        if i.get("geometry") == "cartesian":
            out.update((int(i["nx"]), int(i["ny"])))
        else:
            out.add(int(i["nr"]))
    return out


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


def load_cache(path) -> dict:
    """Tune cache text file -> {(precision, nr): (W, L, us)}; {} if absent."""
    out = {}
    if not path or not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            tok = line.split("#", 1)[0].split()
            if len(tok) >= 5 and tok[1] == "col":
                us = float(tok[5]) if len(tok) > 5 else float("nan")
                out[(tok[0], int(tok[2]))] = (int(tok[3]), int(tok[4]), us)
    return out


def store_cache(path, cache: dict):
    """Writes {(precision, nr): (W, L, us)} as the text file the library reads."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        fh.write("# FCN column tiles: precision col nr W L microseconds\n")
        for (prec, nr), (w, l, us) in sorted(cache.items()):
            fh.write(f"{prec} col {nr} {w} {l} {us:.2f}\n")
    os.replace(tmp, path)


def tune(instances, precision: str = "fp32", steps: int = 20, repeats: int = 3, cache_path=None, log=None):
    """Times every candidate column tile on `instances` and picks the fastest for each nr.

    Returns {"per_nr": {nr: {"col_tile", "col_rows", "us", "table": {"WxL": us}}}, "col_tile",
    "col_rows" (the single pair with the least total column-pass time, for plans that take one
    tile), "col_ms", "table" ({"WxL": total ms}), "cached"}.  With cache_path, entries for every
    nr of the plan are read from and written to that tune cache."""
    from . import fcn
    from . import workloads as wl

    if isinstance(instances, dict):
        instances = [instances]
    nrs = sorted(system_lengths(instances))
    cache = load_cache(cache_path)
    if all((precision, nr) in cache for nr in nrs):
        per = {nr: {"col_tile": cache[(precision, nr)][0], "col_rows": cache[(precision, nr)][1],
                    "us": cache[(precision, nr)][2]} for nr in nrs}
        w0, l0 = per[nrs[-1]]["col_tile"], per[nrs[-1]]["col_rows"]
        return {"per_nr": per, "col_tile": w0, "col_rows": l0, "col_ms": None, "table": {}, "cached": True}
    dt = np.complex128 if precision == "fp64" else np.complex64
    fields = [wl.cartesian_field(i, dt) if fcn.is_cartesian(i) else
              wl.gaussian_field(i, dt) if "I0" in i else wl.random_field(int(i["nr"]), int(i["nt"]), 0, dtype=dt)
              for i in instances]
    per_nr = {nr: {} for nr in nrs}      # nr -> {"WxL": us} where that bucket ran exactly W x L

    def measure(w, l):
        try:
            plan = fcn.Plan(instances, precision=precision, col_tile=w, col_rows=l)
        except fcn.FcnError:
            return None
        f = plan.pack(fields)
        plan.step(f, 2)
        runs = [plan.step_timed_launches(f, steps) for _ in range(repeats)]
        plan.sync()
        total = 0.0
        exact = True
        for j, launch in enumerate(runs[0]):
            if not launch["pass"].startswith("col"):
                continue
            ms = float(np.median([r[j]["ms"] for r in runs]))
            total += ms
            if tuple(launch["tile"]) == (w, l):
                per_nr[launch["size"]][f"{w}x{l}"] = ms * 1e3
            else:
                exact = False  # the runtime fitted a smaller tile for this nr
        if log:
            log(f"col tile {w}x{l}: {total * 1e3:.2f} us")
        return total if exact else None

    (w, l), table = select(CANDIDATES[precision], measure)
    per = {}
    for nr in nrs:
        if not per_nr[nr]:
            raise RuntimeError(f"no column tile could be measured for nr={nr}")
        key = min(per_nr[nr], key=per_nr[nr].get)
        bw, bl = (int(x) for x in key.split("x"))
        per[nr] = {"col_tile": bw, "col_rows": bl, "us": per_nr[nr][key], "table": per_nr[nr]}
        cache[(precision, nr)] = (bw, bl, per_nr[nr][key])
    if cache_path:
        store_cache(cache_path, cache)
    return {"per_nr": per, "col_tile": w, "col_rows": l, "col_ms": table[f"{w}x{l}"], "table": table,
            "cached": False}


def tuned_plan(instances, precision: str = "fp32", cache_path=None, **kw):
    """An fcn.Plan whose column tiles come from the tune cache (tuned first where missing)."""
    from . import fcn

    if cache_path is None:
        fd, cache_path = tempfile.mkstemp(suffix=".tiles")
        os.close(fd)
        os.unlink(cache_path)
    tune(instances, precision, cache_path=cache_path)
    return fcn.Plan(instances, precision=precision, tune_cache=cache_path, **kw)


def main(argv=None):
    """Tunes the column tiles of the benchmark's workloads (the batched sweep, the full-model
    pulse, the long pulse and the paper's two grids) in every precision into one tune cache."""
    import argparse

    from . import workloads as wl

    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--out", required=True, help="tune cache file to write (entries are added or replaced)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args(argv)
    # the headline workload last: where two workloads share an nr, its choice is the one kept
    work = {"full": [wl.config_full()], "long": [wl.config_long()], "application": [wl.config_paper_application()],
            "timing": [wl.config_paper_timing()], "cartesian": [wl.config_cartesian()], "sweep": wl.config_batch()}
    cache = load_cache(args.out)
    for prec in ("fp32_cn64", "fp32", "fp32_storage", "fp64"):
        for name, insts in work.items():
            for nr in system_lengths(insts):
                cache.pop((prec, nr), None)
            store_cache(args.out, cache)
            r = tune(insts, prec, steps=args.steps, repeats=args.repeats, cache_path=args.out)
            cache = load_cache(args.out)
            print(f"{prec} {name}: " + ", ".join(f"nr={nr} {v['col_tile']}x{v['col_rows']} {v['us']:.1f} us"
                                                for nr, v in sorted(r["per_nr"].items())), flush=True)


if __name__ == "__main__":
    main()

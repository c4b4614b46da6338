#!/usr/bin/env python3
"""Throughput of the FCN z-step on one MI355X, in grid-point z-steps per second.

Headline workload: the batched sweep -- 64 Kerr pulses of uneven grids in one plan (Nr in
{256, 512, 1024}, Nt in {512, 1024, 2048, 4096}, P in [1, 10] Pcr, tau in [30, 200] fs, w0 in
[0.5, 3] mm, seeded; 7.56e7 grid points, 605 MB as FP32 complex), advanced together one whole
Strang z-step at a time (one row-kernel launch per distinct Nt: inverse FFT, two nonlinear half
steps, diagnostics partials, FFT; one column-kernel launch per distinct Nr: the Crank-Nicholson
solve) in the FP32-CN64 mode (FP32 field, FP32 FFTs with twiddle pairs and FP32 nonlinear step,
FP64 column solve, FP64 diagnostics), replayed from captured HIP graphs of 16 steps, with the
field resident in HBM.  Each instance steps with its own dz (1 cm or z_c/200); a run is 100
steps, and longer timed runs restart from the resident initial pulses every 100 steps.
The line also carries, on the same sweep, the FP64 plain method and plain FP32 with per-instance
errors against FP64; per-launch kernel times with the roofline of the dominant kernel (HBM bytes
and vector-ALU issue from the committed rocprofv3 counters); the full-model pulse (Nr=512,
Nt=2048, plasma, MPA and collisions) in four precisions with errors at checkpoints; the paper's
own grids; the long-distance pulse at checkpoints against the CPU oracle's stored values;
parareal along z with the classical and the learned coarse propagator; the learned network's
rates; and the CPU oracle's rate on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

METRIC = "grid-pt z-steps/s, FP32/parareal vs FP64 plain at 1e-5 rel err; HBM GB/s"
HBM_PEAK_GBS = 8000.0
# Vector-ALU issue peak of one MI355X in lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  A
# wave64 VALU instruction occupies a SIMD for 4 cycles (the build disables packed FP32, whose
# dual issue is what the 157.3 TFLOP/s FP32 vector figure counts).
VALU_PEAK_TLANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12


def weighted_rel_err(a, ref):
    nr = ref.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    return math.sqrt(np.sum(w[:, None] * np.abs(a - ref) ** 2) / np.sum(w[:, None] * np.abs(ref) ** 2))


CHUNK = 500          # full-model pulse: timed chunks restart from z = 0 (before the collapse)
ROOT = os.path.dirname(os.path.abspath(__file__))
COUNTER_FILE = os.path.join(ROOT, "profiles", "fcn_step_batched64_counters.json")
# Column tiles per nr chosen by the autotuner on an MI355X (autotune.tune; regenerate with --retune)
SHIPPED_TILES = os.path.join(ROOT, "paper_1507_05988_amd", "tuning", "mi355x_tiles.txt")


def _sources_hash(paths):
    import hashlib

    h = hashlib.sha256()
    for src in paths:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(precision, kernel_name):
    """The committed rocprofv3 counters (HBM bytes per launch, copy-calibrated; VALU instructions
    per launch) of one kernel of the batched sweep, or None when no run covers it or its sources
    changed since."""
    try:
        with open(COUNTER_FILE) as fh:
            entries = json.load(fh)["kernels"]
        for t in entries:
            if t["precision"] == precision and t["kernel"] == kernel_name:
                return t if _sources_hash(t["sources"]) == t["sources_sha256"] else None
    except (OSError, KeyError, ValueError):
        pass
    return None


def timed_steps(plan, field, init, steps, torch, chunk=CHUNK):
    """`steps` steps in chunks of `chunk`, each chunk restarting from the resident initial field
    `init`; every chunk is bracketed by device synchronisation and timed with events on the
    plan's stream (the restart copies are outside the timed intervals).  Seconds."""
    total = 0.0
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        with torch.cuda.stream(plan.stream):
            field.copy_(init)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(plan.stream)
        plan.step(field, n)
        end.record(plan.stream)
        torch.cuda.synchronize()
        total += start.elapsed_time(end) * 1e-3
        done += n
    return total


def copy_bandwidth(torch):
    """Practical HBM bandwidth of the box: a 1 GiB device-to-device copy (read + write bytes),
    best of 10, timed with events -- the attainable ceiling beside the 8 TB/s vendor peak."""
    src = torch.ones(2 ** 27, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    nbytes = 2 * src.numel() * src.element_size()
    del src, dst
    return round(nbytes / best / 1e9, 1)


def cpu_baseline(insts, seconds: float):
    """The FP64 oracle on the host cores over a bounded sample of the headline workload: whole
    sweep steps (every instance one step from its initial pulse, then the next step ...), as many
    as fit in about `seconds`; plus the oracle on the paper's timing grid (Sec. 5.1, Table 2) on
    one thread and on all threads, as CPU context."""
    import oracle
    from paper_1507_05988_amd import workloads as wl

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fields = [wl.gaussian_field(i) for i in insts]
    pts = wl.points(insts)
    t0 = time.perf_counter()
    fields = [oracle.propagate(i, a, 1, threads=threads) for i, a in zip(insts, fields)]
    t1 = time.perf_counter() - t0
    n = max(1, min(100, int(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(n):
        fields = [oracle.propagate(i, a, 1, threads=threads) for i, a in zip(insts, fields)]
    dt = time.perf_counter() - t0
    out = {"value": pts * n / dt, "unit": "grid-pt z-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} FP64 oracle z-steps of all {len(insts)} pulses of the batched sweep "
                     f"({pts} points; after 1 warm step), {dt:.1f} s"}
    pg = wl.config_paper_timing()
    ag = wl.gaussian_field(pg)
    rec = {"grid": f"{pg['nr']}x{pg['nt']}"}
    for label, th, steps in (("all_threads", threads, 3), ("one_thread", 1, 1)):
        t0 = time.perf_counter()
        oracle.propagate(pg, ag, steps, threads=th)
        d = time.perf_counter() - t0
        rec[label] = {"threads": th, "seconds_per_step": round(d / steps, 3)}
    out["paper_timing_grid"] = rec
    return out


def kernel_name(precision, launch):
    """Template name of one launch of the sweep's step, as rocprofv3 reports it."""
    if launch["pass"] == "row":
        nt = launch["size"]
        e = 16 if nt >= 4096 or (precision in ("fp64", "fp32_storage") and nt >= 2048) else 8
        r = "double" if precision in ("fp64", "fp32_storage") else "float"
        st = "double" if precision == "fp64" else "float"
        # iFFT, NL, diagnostics, NL, FFT, store (63); twiddle pairs (256); the sweep is Kerr only:
        # no density or absorption term, the phase-only nonlinear step (512)
        flags = 63 + (256 if precision == "fp32_cn64" else 0) + 512
        return f"row_kernel<{r}, {st}, {nt}, {e}, {flags}>"
    r = "float" if precision == "fp32" else "double"
    st = "double" if precision == "fp64" else "float"
    cart = "true" if launch["pass"] in ("col_x", "col_y") else "false"
    # the step's spectrum is in pair order (last template argument)
    return f"col_kernel<{r}, {st}, {launch['tile'][0]}, {launch['tile'][1]}, {cart}, true>"


def sweep_run(torch, insts, precision, steps, warmup, tune_cache, lanes, graph=True):
    """One plan over the whole sweep on its own stream, column tiles per nr from the tune cache,
    the instances in `lanes` concurrent groups: `steps` timed steps (graph replay), then per-launch
    kernel times (the launches one after another), then the field after one 100-step run.
    Returns (seconds, launches, fields, diagnostics)."""
    from paper_1507_05988_amd import fcn
    from paper_1507_05988_amd import workloads as wl

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = fcn.Plan(insts, precision=precision, use_graph=graph, stream=stream, tune_cache=tune_cache,
                        lanes=lanes)
        dt = np.complex128 if precision == "fp64" else np.complex64
        init = plan.pack([wl.gaussian_field(i, dt) for i in insts])
        f = init.clone()
        if warmup > 0:
            plan.step(f, min(warmup, wl.BATCH_STEPS))
        sec = timed_steps(plan, f, init, steps, torch, chunk=wl.BATCH_STEPS)
        f.copy_(init)
        launches = plan.step_timed_launches(f, 20)
        f.copy_(init)
        plan.step(f, wl.BATCH_STEPS)
        plan.sync()
        fields = plan.unpack(f)
        diags = plan.split_diag(plan.diagnostics(f))
        plan.close()
        del f, init
    return sec, launches, fields, diags


def sweep_measurement(torch, args):
    """The headline: the 64-pulse sweep in `args.headline_precision`, graph-replayed; FP64 plain
    and the other FP32 mode beside it; per-instance errors against FP64 after one 100-step run."""
    from paper_1507_05988_amd import autotune
    from paper_1507_05988_amd import workloads as wl

    insts = wl.config_batch()
    pts = wl.points(insts)
    hp = args.headline_precision
    modes = [hp] if args.only_headline else [hp, "fp64", "fp32" if hp == "fp32_cn64" else "fp32_cn64"]
    res = {}
    cache = args.tune_cache
    if args.retune:  # tune anew into the given file (a fresh one when it is the shipped table)
        if os.path.abspath(cache) == os.path.abspath(SHIPPED_TILES):
            cache = os.path.join(tempfile.mkdtemp(prefix="fcn_tiles_"), "tiles.txt")
        elif os.path.exists(cache):
            os.unlink(cache)
    for prec in modes:
        t = autotune.tune(insts, prec, steps=10, repeats=2, cache_path=cache)
        steps = args.steps if prec == hp else wl.BATCH_STEPS
        sec, launches, fields, diags = sweep_run(torch, insts, prec, steps, args.warmup, cache, args.lanes)
        tiles = {nr: [v["col_tile"], v["col_rows"]] for nr, v in t["per_nr"].items()}
        res[prec] = dict(sec=sec, steps=steps, launches=launches, fields=fields, diags=diags, tiles=tiles,
                         tune=({nr: {k: round(x, 2) for k, x in v["table"].items()} for nr, v in t["per_nr"].items()}
                               if not t["cached"] else f"from {os.path.relpath(cache, ROOT)}"))
        print(f"[bench] sweep {prec}: {steps} steps in {sec:.4f} s ({sec / steps * 1e3:.3f} ms/step), "
              f"column tiles per nr {tiles}", file=sys.stderr, flush=True)
    return insts, pts, res


def sweep_errors(insts, got, ref, dgot, dref):
    """Per-instance errors of a sweep run against the FP64 one: r-weighted field error, largest
    element error relative to the largest element, fluence and energy."""
    rows = []
    for i, (g, r, dg, dr) in enumerate(zip(got, ref, dgot, dref)):
        g = g.astype(np.complex128)
        rows.append({"field": weighted_rel_err(g, r),
                     "elementwise": float(np.max(np.abs(g - r)) / np.max(np.abs(r))),
                     "fluence": float(np.max(np.abs(dg["fluence"] - dr["fluence"])) / np.max(dr["fluence"])),
                     "energy": abs(dg["energy"] / dr["energy"] - 1)})
    out = {}
    for k in ("field", "elementwise", "fluence", "energy"):
        v = [r[k] for r in rows]
        out[k + "_max"] = max(v)
        out[k + "_median"] = float(np.median(v))
    worst = int(np.argmax([r["field"] for r in rows]))
    out["worst_instance"] = {"index": worst, "grid": f"{insts[worst]['nr']}x{insts[worst]['nt']}"}
    return out


def paper_shapes_measurement(torch, tune_cache):
    """The paper's own grids, as context beside its CPU numbers (Sec. 5.1 Table 2 and Sec. 5.2;
    the values come from tests/golden/paper_printed_values.json).  The paper's runs are FP64 on
    an Intel Xeon with Pthreads and state no physics for the timing example; the comparison is
    of wall time for the same grid and step count, not of a like-for-like machine."""
    from paper_1507_05988_amd import autotune, fcn
    from paper_1507_05988_amd import workloads as wl

    with open(os.path.join(ROOT, "tests", "golden", "paper_printed_values.json")) as fh:
        paper = json.load(fh)
    out = {}
    t2 = paper["timing_table"]
    cases = (("timing_example", wl.config_paper_timing(), t2["grid"]["Nz"], 1000,
              {"paper_seconds_1_thread": t2["seconds"][0], "paper_seconds_20_threads": t2["seconds"][-1]}),
             ("application_1p1km", wl.config_paper_application(), int(paper["application_run"]["Nz"]), 1000,
              {"paper_statement": "under 3 days with 20 threads, about two months serially (Sec. 5.2)"}))
    for name, inst, nz, timed, ctx in cases:
        pts = int(inst["nr"]) * int(inst["nt"])
        rec = {"grid": f"{inst['nr']}x{inst['nt']}", "steps_in_paper": nz, "timed_steps": timed, **ctx}
        for prec in ("fp64", "fp32"):
            t = autotune.tune(inst, prec, steps=10, repeats=2, cache_path=tune_cache)
            plan = fcn.Plan(inst, precision=prec, col_tile=t["col_tile"], col_rows=t["col_rows"])
            a0 = wl.gaussian_field(inst)
            init = plan.pack(a0 if prec == "fp64" else a0.astype(np.complex64))
            f = init.clone()
            plan.step(f, 5)
            sec = timed_steps(plan, f, init, timed, torch)
            plan.sync()
            rec[prec] = {"seconds_per_step": sec / timed, "seconds_for_paper_steps": sec / timed * nz,
                         "value": round(pts * timed / sec, 1), "col_tile": [t["col_tile"], t["col_rows"]]}
        out[name] = rec
    return out


def cartesian_measurement(torch, tune_cache, steps=100):
    """The Cartesian 3D+1 multi-filament pulse (255 x 255 x 256 = 1.66e7 points, full model,
    Delta_perp = d2/dx2 + d2/dy2): step rate of each precision over `steps` steps of 1 cm from the
    noisy beam, mean per-launch kernel times (row pass, x solves, y solves; each pass reads and
    writes the field once, 48 B per point-step in FP32), and the field error of the FP32-field
    modes against the FP64 run after those steps (relative L2)."""
    from paper_1507_05988_amd import fcn
    from paper_1507_05988_amd import workloads as wl

    inst = wl.config_cartesian()
    pts = wl.points(inst)
    a0 = wl.cartesian_field(inst)
    out = {"grid": f"{inst['nx']}x{inst['ny']}x{inst['nt']}", "points": pts, "steps": steps,
           "z_m": steps * inst["dz"], "bytes_per_point_step": {"fp32_field": 48, "fp64_field": 96}}
    fields = {}
    for prec in ("fp32_cn64", "fp64", "fp32", "fp32_storage"):
        plan = fcn.Plan(inst, precision=prec, tune_cache=tune_cache)
        init = plan.pack(a0 if prec == "fp64" else a0.astype(np.complex64))
        f = init.clone()
        plan.step(f, 3)
        launches = plan.step_timed_launches(f, 10)
        sec = timed_steps(plan, f, init, steps, torch, chunk=steps)
        plan.sync()
        fields[prec] = plan.unpack(f)[0]
        v = pts * steps / sec
        bpp = 96 if prec == "fp64" else 48
        out[prec] = {"value": round(v, 1), "ms_per_step": round(sec * 1e3 / steps, 4),
                     "gbs_algorithmic": round(v * bpp / 1e9, 1),
                     "launches": [{"pass": L["pass"], "size": L["size"], "tile": L["tile"], "ms": round(L["ms"], 6),
                                   "gbs": round(L["points"] * bpp / 3 / (L["ms"] * 1e-3) / 1e9, 1)}
                                  for L in launches]}
        del plan, init, f
    ref = fields["fp64"]
    nref = np.linalg.norm(ref.ravel())
    for prec in ("fp32_cn64", "fp32", "fp32_storage"):
        out[prec]["field_err_vs_fp64"] = float(np.linalg.norm((fields[prec].astype(np.complex128) - ref).ravel()) / nref)
    out["fp32_cn64"]["vs_fp64"] = round(out["fp32_cn64"]["value"] / out["fp64"]["value"], 3)
    return out


def long_pulse_measurement(torch, checkpoints):
    """Long-distance pulse 1024 x 8192, full model, adaptive dz (0.05 rad): FP64 adaptive run;
    FP32, FP32 storage and an FP64 run from the FP32-rounded input (the floor: what the
    trajectory itself makes of FP32 input rounding) replay its dz log.  Errors against the
    FP64 GPU run at every checkpoint; the FP64 run against the CPU oracle's stored values
    (tests/golden/long_pulse_reference.json, written by a script that calls only the oracle)
    at the checkpoints the oracle covers."""
    from paper_1507_05988_amd import fcn
    from paper_1507_05988_amd import workloads as wl

    with open(os.path.join(ROOT, "tests", "golden", "long_pulse_reference.json")) as fh:
        oracle_ref = {c["steps"]: c for c in json.load(fh)["checkpoints"]}
    inst = wl.config_long()
    pts = int(inst["nr"]) * int(inst["nt"])
    a0 = wl.gaussian_field(inst)
    a32 = a0.astype(np.complex64)
    kw = dict(adaptive=True, max_phase=wl.LONG_MAX_PHASE, dz_min=wl.LONG_DZ_MIN, dz_max=wl.LONG_DZ_MAX)
    p64 = fcn.Plan(inst, precision="fp64", **kw)
    runs = {"floor": fcn.Plan(inst, precision="fp64"), "fp32": fcn.Plan(inst, precision="fp32"),
            "fp32_storage": fcn.Plan(inst, precision="fp32_storage"),
            "fp32_cn64": fcn.Plan(inst, precision="fp32_cn64")}
    g64 = p64.pack(a0)
    g = {"floor": runs["floor"].pack(a32.astype(np.complex128)), "fp32": runs["fp32"].pack(a32),
         "fp32_storage": runs["fp32_storage"].pack(a32), "fp32_cn64": runs["fp32_cn64"].pack(a32)}
    log = torch.zeros(checkpoints[-1], dtype=torch.float64, device=p64.device)
    ms = {"fp64": 0.0, "floor": 0.0, "fp32": 0.0, "fp32_storage": 0.0, "fp32_cn64": 0.0}
    alive = {k: True for k in runs}
    rows = []
    done = 0

    def timed(key, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ms[key] += e0.elapsed_time(e1)

    for cp in checkpoints:
        n = cp - done
        timed("fp64", lambda: p64.propagate(g64, n, dz_log=log[done:cp]))
        p64.sync()
        for name, p in runs.items():
            if not alive[name]:
                continue
            timed(name, lambda: p.propagate(g[name], n, dz_log=log[done:cp], replay=True))
            try:
                p.sync()
            except fcn.FcnError:
                alive[name] = False
        done = cp
        lg = log[:cp].cpu().numpy()
        x64 = p64.unpack(g64)[0]
        d64 = p64.split_diag(p64.diagnostics(g64))[0]
        row = {"steps": cp, "z_m": round(float(lg.sum()), 4), "dz_last": float(lg[-1]), "dz_min": float(lg.min()),
               "i_max_fp64": d64["i_max"], "rho_max_fp64": d64["rho_max"]}
        row["floor_fp64_from_fp32_input"] = (weighted_rel_err(runs["floor"].unpack(g["floor"])[0], x64)
                                             if alive["floor"] else None)
        for name in ("fp32", "fp32_storage", "fp32_cn64"):
            if not alive[name]:
                row[name] = None
                continue
            p = runs[name]
            d = p.split_diag(p.diagnostics(g[name]))[0]
            row[name] = {"field": weighted_rel_err(p.unpack(g[name])[0].astype(np.complex128), x64),
                         "fluence": float(np.max(np.abs(d["fluence"] - d64["fluence"])) / np.max(d64["fluence"])),
                         "rho_max": abs(d["rho_max"] - d64["rho_max"]) / max(d64["rho_max"], 1e-300),
                         "energy": abs(d["energy"] / d64["energy"] - 1)}
        c = oracle_ref.get(cp)
        if c is not None:
            smp = np.array([x64[m, t] for m, t, _, _ in c["field_samples"]])
            want = np.array([complex(re, im) for _, _, re, im in c["field_samples"]])
            flu = np.asarray(d64["fluence"][::c["fluence_stride"]])
            row["fp64_vs_oracle"] = {
                "z": abs(float(lg.sum()) / c["z"] - 1),
                "field_samples": float(np.max(np.abs(smp - want)) / c["abs_max"]),
                "fluence": float(np.max(np.abs(flu - np.asarray(c["fluence"]))) / max(c["fluence"])),
                "rho_max": abs(d64["rho_max"] / c["rho_max"] - 1), "energy": abs(d64["energy"] / c["energy"] - 1)}
        rows.append(row)
        print(f"long pulse {cp} steps: z = {row['z_m']} m", file=sys.stderr, flush=True)
    rates = {k: round(pts * checkpoints[-1] / (v / 1e3), 1) for k, v in ms.items() if alive.get(k, True)}
    return {"grid": f"{inst['nr']}x{inst['nt']}", "checkpoints": rows,
            "seconds": {k: round(v / 1e3, 3) for k, v in ms.items()},
            "pt_steps_per_s": {"fp64_adaptive": rates.get("fp64"), "fp32_replay": rates.get("fp32"),
                               "fp32_storage_replay": rates.get("fp32_storage"),
                               "fp32_cn64_replay": rates.get("fp32_cn64")}}


def coarse_net_measurement(torch):
    """The learned coarse network (C = 32): full-grid forward on one 512 x 2048 window (the
    inference of one coarse step; 4.4e11 flop counting a complex multiply-add as 4 real ones)
    and training steps (forward, loss, backward, Adam) on 64 crops of 128 x 128, for BF16 and
    FP32 activations (BF16 with the hidden layers on BF16 matrix cores, and on FP32 vector
    FMAs); device time by events on the network's stream.  Flop rates are against the FP32
    vector peak (157.3 TFLOP/s) and, for the matrix-core form, the dense BF16 peak
    (2.5 PFLOP/s)."""
    from paper_1507_05988_amd import coarse
    from paper_1507_05988_amd import workloads as wl

    inst = wl.config_parareal_trajectory(2000)
    nr, nt = int(inst["nr"]), int(inst["nt"])
    field = torch.from_numpy(wl.gaussian_field(inst, np.complex64).reshape(-1)).cuda()
    flops = 2.0 * 25 * 2 * 64 * (nr + 12) * (nt + 12) + 2.0 * 25 * 64 * 64 * ((nr + 8) * (nt + 8) + (nr + 4) * (nt + 4)) \
        + 2.0 * 25 * 64 * 2 * nr * nt
    out = {"flop_per_forward": flops}

    def timed(fn, reps, stream):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    for key, bf16, mfma in (("bf16_mfma", True, True), ("bf16", True, False), ("fp32", False, False)):
        net = coarse.CoarseNet(channels=32, bf16=bf16, max_batch=1, max_h=nr, max_w=nt, mfma=mfma)
        smp = coarse.samples_tensor(torch, net.device, [(0, 0, 0, 0, 1.0 / coarse.S_REF, 1.0)])
        net.input(field, smp, 1, nr, nt, nr, nt)
        ms = timed(lambda: net.forward(1, nr, nt), 5, net.stream)
        net.close()
        tr = coarse.CoarseNet(channels=32, bf16=bf16, max_batch=64, max_h=128, max_w=128, training=True, mfma=mfma)
        smp = coarse.samples_tensor(torch, tr.device, [(0, 0, (7 * i) % 256, nt // 2 - 64 + i, 1.0 / coarse.S_REF, 1.0)
                                                       for i in range(64)])
        tgt = torch.ones((64, 2, 128, 128), dtype=torch.float32, device=tr.device)
        tr.input(field, smp, 64, nr, nt, 128, 128)
        row0 = [(7 * i) % 256 for i in range(64)]

        def step():
            tr.forward(64, 128, 128)
            tr.loss(tgt, row0, 64, 128, 128)
            tr.backward(64, 128, 128)
            tr.adam(1e-4)

        ms_tr = timed(step, 3, tr.stream)
        tr.close()
        peak = 2500.0 if mfma else 157.3
        out[key] = {"forward_ms": round(ms, 4), "inferences_per_s": round(1e3 / ms, 2),
                    "roofline": {"bound": "mfma" if mfma else "alu", "achieved": round(flops / ms * 1e-9, 2),
                                 "peak": peak, "unit": "TFLOP/s", "frac": round(flops / ms * 1e-9 / peak, 4)},
                    "train_step_ms": round(ms_tr, 3), "train_samples_per_s": round(64 * 1e3 / ms_tr, 1)}
    return out


def parareal_measurement(torch, precision="fp32_cn64"):
    """Parareal along z for held-out learned-coarse trajectory 2000 (Nr=512, Nt=2048, Kerr only,
    never used in training), fine and coarse FCN steps in `precision`, against the serial
    FP64 plain method and the serial fine solver in `precision` over the same steps (device time;
    on one GPU a parareal iteration redoes the whole serial fine work, batched over the windows):
      * the parareal workload as specified, 32 windows x 50 steps of 0.2 mm, classical coarse
        step (one FCN step per window);
      * the learned-coarse variant, 8 windows x 250 steps, classical and learned coarse step
        (the shipped network is trained for these 5 cm windows).
    Errors: r-weighted relative field error against the FP64 solution, max over windows, per
    iteration (k = 0 is the coarse sweep alone; from the Python driver, which can evaluate
    every iterate); stopping rule: change < 1e-4, or the corrections grow.  Wall time is that of
    the library's driver call (fcn_parareal, one host synchronisation per iteration), with the
    plans and the workspace already set up."""
    from paper_1507_05988_amd import coarse, fcn
    from paper_1507_05988_amd import workloads as wl

    inst = wl.config_parareal_trajectory(2000)
    pts = int(inst["nr"]) * int(inst["nt"])
    wfile = os.path.join(ROOT, "paper_1507_05988_amd", "weights", "coarse_c32_bf16.npz")
    net = coarse.CoarseNet.load(wfile) if os.path.exists(wfile) else None
    res = {"trajectory": 2000, "grid": "512x2048", "fine_precision": precision, "tol": 1e-4}
    for label, nwin, spw, learned in (("windows_32x50", wl.PARAREAL_WINDOWS, wl.PARAREAL_STEPS_PER_WINDOW, False),
                                      ("windows_8x250", wl.LEARNED_WINDOWS, wl.LEARNED_STEPS_PER_WINDOW, True)):
        work = pts * nwin * spw
        p64 = fcn.Plan(inst, precision="fp64")
        a0 = wl.gaussian_field(inst)
        f = p64.pack(a0)
        ref = []
        for _ in range(nwin):
            p64.step(f, spw)
            ref.append(f.clone())
        f = p64.pack(a0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(p64.stream)
        p64.step(f, nwin * spw)
        e1.record(p64.stream)
        torch.cuda.synchronize()
        t64 = e0.elapsed_time(e1) * 1e-3
        # the serial fine solver in the fine precision of parareal: the same-precision comparison
        ps = fcn.Plan(inst, precision=precision)
        fs = ps.pack(a0.astype(np.complex64))
        ps.step(fs, 2)
        fs = ps.pack(a0.astype(np.complex64))
        torch.cuda.synchronize()
        e0.record(ps.stream)
        ps.step(fs, nwin * spw)
        e1.record(ps.stream)
        torch.cuda.synchronize()
        tfine = e0.elapsed_time(e1) * 1e-3
        efine = weighted_rel_err(ps.unpack(fs)[0].astype(np.complex128), p64.unpack(ref[-1])[0])
        del ps, fs
        out = {"fp64_plain_serial": {"seconds": round(t64, 6), "value": round(work / t64, 1)},
               "serial_fine_same_precision": {"seconds": round(tfine, 6), "value": round(work / tfine, 1),
                                              "error_vs_fp64": efine}}
        variants = [("classical", None)]
        if learned and net is not None:
            variants.append(("learned", net))
        for name, m in variants:
            kw = dict(windows=nwin, steps_per_window=spw, kmax=nwin, tol=1e-4, precision=precision,
                      fallback=True)
            if m is not None:
                kw.update(channels=m["channels"], bf16=m["bf16"], kappa=m["kappa"], s_ref=m["s_ref"])
            params = m["params"] if m is not None else None
            _, hist = coarse.parareal(inst, params, reference=ref, **kw)
            coarse.parareal_native(inst, params, **kw)  # warm-up
            _, nat = coarse.parareal_native(inst, params, **kw)
            tp = nat["seconds"]
            out[name] = {"seconds": round(tp, 6), "value": round(work / tp, 1), "vs_fp64_plain": round(t64 / tp, 3),
                         "vs_serial_fine_same_precision": round(tfine / tp, 3),
                         "iterations": [{"k": h["iter"], "error": h["error"],
                                         "change": h["change"] if h["iter"] else None} for h in hist],
                         "status": hist[-1].get("status"), "final_error": hist[-1]["error"],
                         "native_driver": {"status": nat["status"], "iterations": nat["iterations"]}}
            if m is not None:
                out[name]["weights"] = os.path.relpath(wfile, ROOT)
        res[label] = out
    return res


def full_model_measurement(torch, args):
    """The full-model pulse (Nr=512, Nt=2048, Kerr n2+n4, plasma, MPA and collisions, dz = 5 mm)
    in FP32-CN64, plain FP32, FP32 storage and FP64, timed in chunks of 500 steps from z = 0
    (before the collapse near 4.2 m; past it the explicit RK4 density step can leave its
    stability region, which the library reports as FCN_E_UNSTABLE); per-kernel times; errors of
    the FP32-field modes against FP64 at checkpoints, with the FP64 run's own sensitivity to FP32
    input rounding as the conditioning floor."""
    from paper_1507_05988_amd import autotune, fcn
    from paper_1507_05988_amd import workloads as wl

    inst = wl.config_full()
    pts = int(inst["nr"]) * int(inst["nt"])
    a0 = wl.gaussian_field(inst)
    n = min(max(args.steps, 100), 1000)
    out = {"grid": "512x2048", "steps": n, "unit": "grid-pt z-steps/s"}
    for prec in ("fp32_cn64", "fp32", "fp32_storage", "fp64"):
        t = autotune.tune(inst, prec, steps=50, repeats=3, cache_path=args.tune_cache)
        plan = fcn.Plan(inst, precision=prec, col_tile=t["col_tile"], col_rows=t["col_rows"])
        init = plan.pack(a0 if prec == "fp64" else a0.astype(np.complex64))
        f = init.clone()
        plan.step(f, 20)
        sec = timed_steps(plan, f, init, n, torch)
        plan.sync()
        f.copy_(init)
        krow, kcol, _ = plan.step_timed(f, min(n, CHUNK))
        plan.sync()
        byt = 64 if prec == "fp64" else 32
        out[prec] = {"value": round(pts * n / sec, 1), "ms_per_step": round(sec * 1e3 / n, 6),
                     "row_ms": round(krow, 6), "col_ms": round(kcol, 6),
                     "hbm_gbs_algorithmic": round(pts * n / sec * byt / 1e9, 1),
                     "col_tile": [t["col_tile"], t["col_rows"]]}
        del plan, f, init
    for prec in ("fp32_cn64", "fp32", "fp32_storage"):
        out[prec]["vs_fp64_plain"] = round(out[prec]["value"] / out["fp64"]["value"], 3)
    if args.no_accuracy:
        return out
    checkpoints = (250, 500, 750, 1000, wl.FULL_STEPS)
    runs = {"fp64": fcn.Plan(inst, precision="fp64"), "floor": fcn.Plan(inst, precision="fp64"),
            "fp32": fcn.Plan(inst, precision="fp32"), "fp32_storage": fcn.Plan(inst, precision="fp32_storage"),
            "fp32_cn64": fcn.Plan(inst, precision="fp32_cn64")}
    a32 = a0.astype(np.complex64)
    g = {k: p.pack(a0 if k == "fp64" else (a32.astype(np.complex128) if k == "floor" else a32))
         for k, p in runs.items()}
    alive = {k: True for k in runs}
    acc = []
    done = 0
    for cp in checkpoints:
        for k, p in runs.items():
            if not alive[k]:
                continue
            p.step(g[k], cp - done)
            try:
                p.sync()
            except fcn.FcnError as e:
                alive[k] = f"stopped before step {cp}: {e}"
        done = cp
        x64 = runs["fp64"].unpack(g["fp64"])[0]
        d64 = runs["fp64"].split_diag(runs["fp64"].diagnostics(g["fp64"]))[0]
        row = {"steps": cp, "z_m": round(cp * inst["dz"], 4), "i_max_fp64": d64["i_max"],
               "rho_max_fp64": d64["rho_max"],
               "floor_fp64_from_fp32_input": weighted_rel_err(runs["floor"].unpack(g["floor"])[0], x64)}
        for k in ("fp32", "fp32_storage", "fp32_cn64"):
            if alive[k] is not True:
                row[k] = alive[k]
                continue
            p = runs[k]
            x = p.unpack(g[k])[0].astype(np.complex128)
            d = p.split_diag(p.diagnostics(g[k]))[0]
            row[k] = {"field": weighted_rel_err(x, x64),
                      "elementwise": float(np.max(np.abs(x - x64)) / np.max(np.abs(x64))),
                      "fluence": float(np.max(np.abs(d["fluence"] - d64["fluence"])) / np.max(d64["fluence"])),
                      "rho_max": abs(d["rho_max"] - d64["rho_max"]) / max(d64["rho_max"], 1e-300),
                      "energy": abs(d["energy"] / d64["energy"] - 1)}
        acc.append(row)
    out["accuracy_vs_fp64"] = acc
    return out


def dominant_roofline(hp, launches):
    """Roofline of the dominant kernel: the kernel template with the longest total time per step
    (with several lanes a template serves several launches of a step): its average bytes per
    launch over its average launch duration.  The launch durations come from the per-launch timed
    steps, which run the launches one after another (each kernel alone on the GPU); rocprofv3's
    per-kernel average over a run of such steps (`--launch-timing-only`) measures the same.
    Annotates `launches` with kernel names, bytes and GB/s."""
    by_kernel = {}
    for L in launches:
        L["kernel"] = kernel_name(hp, L)
        L["bytes"] = L["points"] * 16  # FP32 field: each launch reads and writes its points once
        L["gbs"] = round(L["bytes"] / (L["ms"] * 1e-3) / 1e9, 1)
        k = by_kernel.setdefault(L["kernel"], {"ms": 0.0, "bytes": 0, "launches": 0})
        k["ms"] += L["ms"]
        k["bytes"] += L["bytes"]
        k["launches"] += 1
    dom_name, dom = max(by_kernel.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    avg_bytes = dom["bytes"] / dom["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    cnt = measured_counters(hp, dom_name)
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": int(cnt["bytes_per_launch"]) if cnt else None}
    roofline = dict(hbm)
    if cnt and cnt.get("valu_insts_per_launch"):
        lane_ops = cnt["valu_insts_per_launch"] * 64 / (avg_ms * 1e-3) / 1e12
        valu = {"bound": "alu", "achieved": round(lane_ops, 3), "peak": round(VALU_PEAK_TLANE_OPS, 3),
                "unit": "T VALU lane-ops/s", "frac": round(lane_ops / VALU_PEAK_TLANE_OPS, 4),
                "valu_insts_per_launch": cnt["valu_insts_per_launch"]}
        if valu["frac"] > hbm["frac"]:
            roofline = dict(valu, traffic=hbm["traffic"], hbm=hbm)
        else:
            roofline["valu"] = valu
    # target_frac: the 60% of the HBM roofline the step aims at; the dominant kernels are bound by
    # vector-ALU issue (row passes) and by the latency of the FP64 solve chain (column passes)
    # before HBM, which the "valu" object beside the HBM figure shows
    roofline.update(kernel=dom_name, kernel_ms=round(avg_ms, 6), launches_per_step=dom["launches"],
                    bytes_per_launch=round(avg_bytes), kernel_ms_per_step=round(dom["ms"], 6), target_frac=0.6)
    return roofline


def launch_timing_only(torch, args):
    """Only the per-launch timing of the headline plan: two timed steps to warm up, then the timed
    steps whose launch durations the roofline uses, every dispatch eager and one after another,
    so a rocprofv3 kernel trace of this run averages the same dispatches the events time."""
    from paper_1507_05988_amd import fcn
    from paper_1507_05988_amd import workloads as wl

    hp = args.headline_precision
    insts = wl.config_batch()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = fcn.Plan(insts, precision=hp, use_graph=True, stream=stream, tune_cache=args.tune_cache,
                        lanes=args.lanes)
        f = plan.pack([wl.gaussian_field(i, np.complex64) for i in insts])
        plan.step_timed_launches(f, 2)
        launches = plan.step_timed_launches(f, 20)
        plan.sync()
    return {"launches": launches, "roofline": dominant_roofline(hp, launches)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--headline-precision", default="fp32_cn64", choices=["fp32_cn64", "fp32"],
                    help="mode of the headline line: fp32_cn64 (within 1e-5 of FP64 on every pulse of the "
                         "sweep) or fp32 (faster; its largest pulse misses 1e-5)")
    ap.add_argument("--tune-cache", default=SHIPPED_TILES,
                    help="tune cache of column tiles per nr (tuned where it lacks an entry)")
    ap.add_argument("--retune", action="store_true", help="tune every column tile anew")
    ap.add_argument("--lanes", type=int, default=6,
                    help="concurrent instance groups of the sweep plans (fcn_options.lanes)")
    ap.add_argument("--only-headline", action="store_true",
                    help="only the headline sweep in the headline mode (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-full-model", action="store_true")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--no-net", action="store_true")
    ap.add_argument("--no-paper-shapes", action="store_true")
    ap.add_argument("--no-long-pulse", action="store_true")
    ap.add_argument("--no-cartesian", action="store_true")
    ap.add_argument("--long-pulse-checkpoints", default="100,1000,10000",
                    help="comma-separated step counts of the long-distance pulse checkpoints")
    ap.add_argument("--launch-timing-only", action="store_true",
                    help="only the headline plan's per-launch timing and the roofline of its dominant kernel "
                         "(the run to profile for the kernel trace that the roofline's durations match)")
    ap.add_argument("--only-net", action="store_true",
                    help="only the learned coarse network's inference and training rates (one JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy 10 times (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: this build runs the "
              "z-step on a single MI355X (multi-GPU sharding is a design note, not implemented).",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 2:
        print("--steps must be >= 2", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.only_net:
        print(json.dumps({"coarse_net": coarse_net_measurement(torch)}), flush=True)
        return
    if args.launch_timing_only:
        print(json.dumps(launch_timing_only(torch, args)), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "reps": 10}))
        return

    insts, pts, sw = sweep_measurement(torch, args)
    hp = args.headline_precision
    h = sw[hp]
    value = pts * h["steps"] / h["sec"]
    ms_per_step = h["sec"] * 1e3 / h["steps"]

    launches = h["launches"]
    roofline = dominant_roofline(hp, launches)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "grid-pt z-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if hp == "fp32_cn64" else "f32",
        "data": "synthetic",
        "config": {"workload": ("batched sweep: 64 Kerr pulses of uneven grids (Nr 256-1024, Nt 512-4096, "
                                "7.56e7 points) advanced together, one Strang z-step per step, "
                                + ("FP32 field, FP32 FFTs (twiddle pairs) and nonlinear step, FP64 CN column "
                                   "solve and diagnostics" if hp == "fp32_cn64" else "FP32 field and arithmetic, "
                                   "FP64 diagnostics")
                                + f", {args.lanes} concurrent instance groups, HIP-graph replay, timed in runs of "
                                  f"{wl_batch_steps()} steps from the initial pulses"),
                   "precision": hp, "instances": len(insts), "points": pts, "lanes": args.lanes,
                   "column_tiles_per_nr": h["tiles"], "terms": "diffraction+GVD+Kerr(n2)"},
        "column_tile_tuning_us": h["tune"],
        "hbm_gbs_algorithmic": round(value * 32 / 1e9, 1),
        "roofline": roofline,
        "launches": [{k: (round(v, 6) if k == "ms" else v) for k, v in L.items()} for L in launches],
        "hbm_copy_gbs": copy_bandwidth(torch),
    }
    if "fp64" in sw:
        ref, dref = sw["fp64"]["fields"], sw["fp64"]["diags"]
        v64 = pts * sw["fp64"]["steps"] / sw["fp64"]["sec"]
        out["vs_fp64_plain"] = round(value / v64, 3)
        out["accuracy_vs_fp64"] = sweep_errors(insts, h["fields"], ref, h["diags"], dref)
        out["sweep"] = {"fp64_plain": {"value": round(v64, 1), "ms_per_step": round(sw["fp64"]["sec"] * 1e3 /
                                                                                   sw["fp64"]["steps"], 4),
                                       "column_tiles_per_nr": sw["fp64"]["tiles"],
                                       "launches": [{"pass": L["pass"], "size": L["size"], "ms": round(L["ms"], 6)}
                                                    for L in sw["fp64"]["launches"]]}}
        for k, r in sw.items():
            if k in (hp, "fp64"):
                continue
            v = pts * r["steps"] / r["sec"]
            out["sweep"][k] = {"value": round(v, 1), "ms_per_step": round(r["sec"] * 1e3 / r["steps"], 4),
                               "vs_fp64_plain": round(v / v64, 3), "column_tiles_per_nr": r["tiles"],
                               "launches": [{"pass": L["pass"], "size": L["size"], "ms": round(L["ms"], 6)}
                                            for L in r["launches"]],
                               "accuracy_vs_fp64": sweep_errors(insts, r["fields"], ref, r["diags"], dref)}
    del sw
    def progress(what):
        print(f"bench: {what}", file=sys.stderr, flush=True)

    if not args.only_headline:
        progress("extras")
        if not args.no_full_model:
            progress("full-model pulse")
            out["full_model_pulse"] = full_model_measurement(torch, args)
        if not args.no_paper_shapes:
            progress("paper grids")
            out["paper_shapes"] = paper_shapes_measurement(torch, args.tune_cache)
        if not args.no_cartesian:
            progress("Cartesian pulse")
            out["cartesian_3d"] = cartesian_measurement(torch, args.tune_cache)
        if not args.no_long_pulse:
            out["long_pulse"] = long_pulse_measurement(torch, [int(x) for x in args.long_pulse_checkpoints.split(",")])
        if not args.no_parareal:
            progress("parareal")
            out["parareal"] = parareal_measurement(torch, "fp32_cn64")
            out["parareal_fp32_storage"] = parareal_measurement(torch, "fp32_storage")
        if not args.no_net:
            progress("network")
            out["coarse_net"] = coarse_net_measurement(torch)
        if not args.no_cpu_baseline:
            progress("CPU baseline")
            out["cpu_baseline"] = cpu_baseline(insts, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def wl_batch_steps():
    from paper_1507_05988_amd import workloads as wl

    return wl.BATCH_STEPS


if __name__ == "__main__":
    main()

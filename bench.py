#!/usr/bin/env python3
"""Throughput of the FCN z-step on one MI355X, in grid-point z-steps per second.

Workload: the full-model pulse (Nr=512 over [0, 8 mm], Nt=2048 over [-400, 400) fs,
w0 = 2 mm, tau = 100 fs, P = 5 Pcr, Kerr n2 + n4, 8-photon ionisation with plasma
defocusing, multiphoton and collisional absorption, dz = 5 mm), in the FP32 field
precision with FP64 density scan and diagnostics.  One step is one whole Strang z-step
(column CN solve + fused iFFT / two nonlinear half steps / FFT row pass, diagnostics
partials included) on the resident field.  The timed steps run in chunks of at most
500 steps (z <= 2.5 m, before the collapse near 4.2 m), each chunk starting from the
resident initial pulse: past the collapse the trajectory is chaotic and the explicit RK4
density step can leave its stability region (sigma_K I^K dtau > 2.785).
The line also carries the FP64 plain method, the FP32-storage mode (FP32 field, FP64
arithmetic) and the FP32-CN64 mode (FP32 row pass with twiddle pairs, FP64 column solve) on
the same workload, the errors of the three FP32-field modes against FP64 at
checkpoints (with the FP64 run's own sensitivity to FP32 input rounding as the
conditioning floor), parareal along z on a held-out learned-coarse trajectory (classical
and learned coarse propagator, fine steps in FP32-CN64 and in FP32 storage, against the
serial FP64 plain method), the long-distance
pulse (1024 x 8192, adaptive dz) at checkpoints up to 10^4 steps (FP32 modes against FP64,
FP64 against the CPU oracle's stored values; --long-pulse-checkpoints extends it), the
roofline of the dominant kernel and the CPU oracle's rate on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "grid-pt z-steps/s, FP32/parareal vs FP64 plain at 1e-5 rel err; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def weighted_rel_err(a, ref):
    nr = ref.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    return math.sqrt(np.sum(w[:, None] * np.abs(a - ref) ** 2) / np.sum(w[:, None] * np.abs(ref) ** 2))


CHUNK = 500
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fcn_step_fullmodel_512x2048_traffic.json")


def measured_traffic(precision, kernel, tiles):
    """HBM bytes per launch of one kernel of the full-model step (`kernel` "row" or "col") in
    `precision` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs (copy-calibrated), or
    None when no run covers that kernel or its sources changed since."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as fh:
            entries = json.load(fh)["kernels"]
        for t in entries:
            if t["precision"] != precision or t["pass"] != kernel:
                continue
            if kernel == "col" and [t["col_tile"], t["col_rows"]] != [tiles["col_tile"], tiles["col_rows"]]:
                continue
            h = hashlib.sha256()
            for src in t["sources"]:
                with open(os.path.join(ROOT, src), "rb") as fh:
                    h.update(fh.read())
            return int(t["bytes_per_launch"]) if h.hexdigest() == t["sources_sha256"] else None
    except (OSError, KeyError, ValueError):
        pass
    return None


def timed_steps(plan, field, init, steps, torch):
    """`steps` steps in chunks of CHUNK, each chunk restarting from the resident initial
    field `init`; every chunk is bracketed by device synchronisation and timed with events
    on the plan's stream (the restart copies are outside the timed intervals).  Seconds."""
    total = 0.0
    done = 0
    while done < steps:
        n = min(CHUNK, steps - done)
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


def cpu_baseline(inst, a0, seconds: float):
    """The FP64 oracle on the host cores over a bounded sample of the same workload."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pts = int(inst["nr"]) * int(inst["nt"])
    t0 = time.perf_counter()
    a = oracle.propagate(inst, a0, 1, threads=threads)
    t1 = time.perf_counter() - t0
    n = max(1, min(2000, int(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.propagate(inst, a, n, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": pts * n / dt, "unit": "grid-pt z-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} FP64 oracle steps of the {inst['nr']}x{inst['nt']} full-model pulse "
                     f"(after 1 warm step), {dt:.1f} s"}
    # the same oracle on one thread (a few steps), and on the grid of the paper's timing
    # example (Nr = 2112, Nt = 2048, Sec. 5.1 Table 2) on one thread and on all threads
    from paper_1507_05988_amd import workloads as wl

    n1 = max(1, int(min(seconds / 4, 5.0) / max(t1 * threads, 1e-6)))
    t0 = time.perf_counter()
    oracle.propagate(inst, a, n1, threads=1)
    d1 = time.perf_counter() - t0
    out["one_thread"] = {"value": pts * n1 / d1, "steps": n1, "seconds": round(d1, 2)}
    pg = wl.config_paper_timing()
    ag = wl.gaussian_field(pg)
    rec = {"grid": f"{pg['nr']}x{pg['nt']}"}
    for label, th, steps in (("all_threads", threads, 5), ("one_thread", 1, 1)):
        t0 = time.perf_counter()
        oracle.propagate(pg, ag, steps, threads=th)
        d = time.perf_counter() - t0
        rec[label] = {"threads": th, "seconds_per_step": round(d / steps, 3)}
    out["paper_timing_grid"] = rec
    return out


def batched_sweep_measurement(torch):
    """The 64-pulse ragged sweep (Nr in {256, 512, 1024}, Nt in {512 ... 4096}, about 7.5e7
    points, Kerr, one plan with autotuned column tiles), 100 steps, in FP64, FP32 and
    FP32-CN64: aggregate throughput, per-pass kernel times (kernel-own events; one launch per
    distinct Nt or Nr) and the largest per-instance field error against the FP64 GPU run."""
    from paper_1507_05988_amd import autotune, fcn
    from paper_1507_05988_amd import workloads as wl

    insts = wl.config_batch()
    pts = sum(int(i["nr"]) * int(i["nt"]) for i in insts)
    byt = pts * 16
    t64 = autotune.tune(insts, "fp64", steps=10, repeats=2)
    p64 = fcn.Plan(insts, precision="fp64", col_tile=t64["col_tile"], col_rows=t64["col_rows"])
    init64 = p64.pack([wl.gaussian_field(i) for i in insts])
    f64 = init64.clone()
    p64.step(f64, 5)
    sec64 = timed_steps(p64, f64, init64, wl.BATCH_STEPS, torch)
    f64.copy_(init64)
    p64.step(f64, wl.BATCH_STEPS)
    p64.sync()
    ref = p64.unpack(f64)
    del p64, f64, init64
    out = {"points": pts, "instances": len(insts), "steps": wl.BATCH_STEPS, "unit": "grid-pt z-steps/s",
           "fp64_plain": {"value": round(pts * wl.BATCH_STEPS / sec64, 1),
                          "ms_per_step": round(sec64 * 1e3 / wl.BATCH_STEPS, 4),
                          "col_tile": [t64["col_tile"], t64["col_rows"]]}}
    for prec in ("fp32", "fp32_cn64"):
        t = autotune.tune(insts, prec, steps=10, repeats=2)
        plan = fcn.Plan(insts, precision=prec, col_tile=t["col_tile"], col_rows=t["col_rows"])
        init = plan.pack([wl.gaussian_field(i, np.complex64) for i in insts])
        f = init.clone()
        plan.step(f, 5)
        sec = timed_steps(plan, f, init, wl.BATCH_STEPS, torch)
        f.copy_(init)
        krow, kcol, _ = plan.step_timed(f, 20)
        f.copy_(init)
        plan.step(f, wl.BATCH_STEPS)
        plan.sync()
        errs = [weighted_rel_err(g.astype(np.complex128), r) for g, r in zip(plan.unpack(f), ref)]
        value = pts * wl.BATCH_STEPS / sec
        out[prec] = {
            "value": round(value, 1), "ms_per_step": round(sec * 1e3 / wl.BATCH_STEPS, 4),
            "hbm_gbs_algorithmic": round(value * 32 / 1e9, 1), "row_pass_ms": round(krow, 4),
            "col_pass_ms": round(kcol, 4), "col_tile": [t["col_tile"], t["col_rows"]],
            "field_error_vs_fp64_max": max(errs), "field_error_vs_fp64_median": float(np.median(errs)),
            "vs_fp64_plain": round(sec64 / sec, 3),
            "roofline_row_pass": {"bound": "hbm", "achieved": round(byt / (krow * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(byt / (krow * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "roofline_col_pass": {"bound": "hbm", "achieved": round(byt / (kcol * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(byt / (kcol * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
        del plan, f, init
    return out


def paper_shapes_measurement(torch):
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
            t = autotune.tune(inst, prec, steps=10, repeats=2)
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
    FP64 plain method over the same steps (device time):
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
        out = {"fp64_plain_serial": {"seconds": round(t64, 6), "value": round(work / t64, 1)}}
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
                         "iterations": [{"k": h["iter"], "error": h["error"],
                                         "change": h["change"] if h["iter"] else None} for h in hist],
                         "status": hist[-1].get("status"), "final_error": hist[-1]["error"],
                         "native_driver": {"status": nat["status"], "iterations": nat["iterations"]}}
            if m is not None:
                out[name]["weights"] = os.path.relpath(wfile, ROOT)
        res[label] = out
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--no-net", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-paper-shapes", action="store_true")
    ap.add_argument("--headline-precision", default="fp32_cn64", choices=["fp32_cn64", "fp32"],
                    help="mode of the headline line: fp32_cn64 (within 1e-5 of FP64 over the timed "
                         "chunks) or fp32 (faster, within 1e-5 for about 190 steps of this workload)")
    ap.add_argument("--no-long-pulse", action="store_true")
    ap.add_argument("--long-pulse-checkpoints", default="100,1000,10000",
                    help="comma-separated step counts of the long-distance pulse checkpoints")
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
    from paper_1507_05988_amd import fcn
    from paper_1507_05988_amd import workloads as wl

    if args.only_net:
        print(json.dumps({"coarse_net": coarse_net_measurement(torch)}), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "reps": 10}))
        return

    inst = wl.config_full()
    pts = int(inst["nr"]) * int(inst["nt"])
    a0 = wl.gaussian_field(inst)

    # ---- FP32 timed region
    from paper_1507_05988_amd import autotune

    tiles = {prec: autotune.tune(inst, prec, steps=50, repeats=3) for prec in ("fp32", "fp64", "fp32_storage", "fp32_cn64")}
    tile_kw = {prec: dict(col_tile=t["col_tile"], col_rows=t["col_rows"]) for prec, t in tiles.items()}
    print("[bench] column tiles (autotuned): " + ", ".join(f"{k} {t['col_tile']}x{t['col_rows']}" for k, t in tiles.items()),
          file=sys.stderr, flush=True)
    hp = args.headline_precision
    p32 = fcn.Plan(inst, precision=hp, **tile_kw[hp])
    init32 = p32.pack(a0.astype(np.complex64))
    f32 = init32.clone()
    if args.warmup > 0:
        p32.step(f32, min(args.warmup, CHUNK))
    sec = timed_steps(p32, f32, init32, args.steps, torch)
    p32.sync()
    value = pts * args.steps / sec
    ms_per_step = sec * 1e3 / args.steps
    print(f"[bench] {hp} {args.steps} steps in {sec:.4f} s ({ms_per_step * 1e3:.2f} us/step)", file=sys.stderr,
          flush=True)

    # ---- per-kernel durations with HIP events on the plan's stream
    f32.copy_(init32)
    krow, kcol, _ = p32.step_timed(f32, min(args.steps, CHUNK))
    p32.sync()
    bytes_per_launch = pts * 2 * 8  # each pass reads and writes every FP32 complex value once
    row_name = ("row_kernel<float, float, 2048, 8> (iFFT + 2 NL half steps + FFT"
                + (", twiddle pairs)" if hp == "fp32_cn64" else ")"))
    col_name = (f"col_kernel<{'double' if hp == 'fp32_cn64' else 'float'}, float, {tiles[hp]['col_tile']}, "
                f"{tiles[hp]['col_rows']}> (CN solve)")
    dom = "row" if krow >= kcol else "col"
    dom_name, dom_ms = (row_name, krow) if dom == "row" else (col_name, kcol)
    achieved = bytes_per_launch / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(hp, dom, tiles[hp]),
                "kernel": dom_name, "kernel_ms": round(dom_ms, 6), "row_ms": round(krow, 6), "col_ms": round(kcol, 6),
                "bytes_per_launch": bytes_per_launch}
    print(f"[bench] kernel means: row {krow * 1e3:.2f} us, col {kcol * 1e3:.2f} us", file=sys.stderr, flush=True)

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
        "config": {"workload": ("full-model pulse, FP32 field, FP32 FFTs (twiddle pairs) and nonlinear step, "
                                "FP64 CN column solve and density scan" if hp == "fp32_cn64" else
                                "full-model pulse, FP32 field / FP64 density") +
                               f", Nr=512, Nt=2048, dz=5 mm, timed in chunks of {CHUNK} steps from z=0",
                   "precision": hp,
                   "nr": int(inst["nr"]), "nt": int(inst["nt"]), "dz": inst["dz"], "P_over_Pcr": 5.0,
                   "terms": "diffraction+GVD+Kerr(n2,n4)+plasma+MPA(K=8)+collisions"},
        "hbm_gbs_algorithmic": round(value * 32 / 1e9, 1),
        "roofline": roofline,
        "hbm_copy_gbs": copy_bandwidth(torch),
        "column_tiles": {k: {"col_tile": t["col_tile"], "col_rows": t["col_rows"],
                             "col_us": {kk: round(v * 1e3, 2) for kk, v in t["table"].items()}} for k, t in tiles.items()},
    }

    # ---- FP64 plain method on the same workload
    if not args.no_fp64:
        p64 = fcn.Plan(inst, precision="fp64", **tile_kw["fp64"])
        init64 = p64.pack(a0)
        f64 = init64.clone()
        p64.step(f64, min(args.warmup, 50) or 1)
        n64 = min(args.steps, 1000)
        s64 = timed_steps(p64, f64, init64, n64, torch)
        p64.sync()
        f64.copy_(init64)
        r64, c64, _ = p64.step_timed(f64, min(n64, CHUNK))
        out["fp64_plain"] = {"value": round(pts * n64 / s64, 1), "ms_per_step": round(s64 * 1e3 / n64, 6),
                             "steps": n64, "row_ms": round(r64, 6), "col_ms": round(c64, 6),
                             "hbm_gbs_algorithmic": round(pts * n64 / s64 * 64 / 1e9, 1)}
        del p64, f64
        out["vs_fp64_plain"] = round(value / (pts * n64 / s64), 3)
        for mode in ("fp32_storage", "fp32_cn64" if hp == "fp32" else "fp32"):
            pm = fcn.Plan(inst, precision=mode, **tile_kw[mode])
            initm = pm.pack(a0.astype(np.complex64))
            fm = initm.clone()
            pm.step(fm, min(args.warmup, 50) or 1)
            sm = timed_steps(pm, fm, initm, n64, torch)
            pm.sync()
            fm.copy_(initm)
            rm, cm, _ = pm.step_timed(fm, min(n64, CHUNK))
            out[mode] = {"value": round(pts * n64 / sm, 1), "ms_per_step": round(sm * 1e3 / n64, 6),
                         "steps": n64, "row_ms": round(rm, 6), "col_ms": round(cm, 6),
                         "hbm_gbs_algorithmic": round(pts * n64 / sm * 32 / 1e9, 1),
                         "vs_fp64_plain": round(s64 / sm, 3)}
            del pm, fm

    # ---- FP32 error against the FP64 GPU method at checkpoints; the FP64 run started from
    # the FP32-rounded input measures how much the trajectory itself amplifies FP32 rounding
    if not args.no_accuracy:
        checkpoints = (250, 500, 750, 1000, wl.FULL_STEPS)
        q32 = fcn.Plan(inst, precision="fp32")
        q64 = fcn.Plan(inst, precision="fp64")
        qr = fcn.Plan(inst, precision="fp64")
        qm = fcn.Plan(inst, precision="fp32_storage")
        qc = fcn.Plan(inst, precision="fp32_cn64")
        gc = qc.pack(a0.astype(np.complex64))
        ok_c = True
        g32 = q32.pack(a0.astype(np.complex64))
        g64 = q64.pack(a0)
        gr = qr.pack(a0.astype(np.complex64).astype(np.complex128))
        gm = qm.pack(a0.astype(np.complex64))
        ok_m = True
        acc = []
        done = 0
        for cp in checkpoints:
            for q, g in ((q32, g32), (q64, g64), (qr, gr), (qm, gm), (qc, gc)):
                q.step(g, cp - done)
            done = cp
            ok32 = True
            try:
                q32.sync()
            except fcn.FcnError:
                ok32 = False
            q64.sync()
            qr.sync()
            try:
                qm.sync()
            except fcn.FcnError:
                ok_m = False
            try:
                qc.sync()
            except fcn.FcnError:
                ok_c = False
            x64 = q64.unpack(g64)[0]
            d32 = q32.split_diag(q32.diagnostics(g32))[0]
            d64 = q64.split_diag(q64.diagnostics(g64))[0]
            row = {"steps": cp, "z_m": round(cp * inst["dz"], 4),
                   "floor_fp64_from_fp32_input": weighted_rel_err(qr.unpack(gr)[0], x64),
                   "i_max_fp64": d64["i_max"], "rho_max_fp64": d64["rho_max"]}
            if ok32:
                x32 = q32.unpack(g32)[0].astype(np.complex128)
                row.update(field=weighted_rel_err(x32, x64),
                           fluence=float(np.max(np.abs(d32["fluence"] - d64["fluence"])) / np.max(d64["fluence"])),
                           rho_max=abs(d32["rho_max"] - d64["rho_max"]) / max(d64["rho_max"], 1e-300),
                           energy=abs(d32["energy"] / d64["energy"] - 1))
            else:
                row.update(field=None, note="FP32 trajectory left the RK4 density stability region")
            row["field_fp32_storage"] = weighted_rel_err(qm.unpack(gm)[0].astype(np.complex128), x64) if ok_m else None
            row["field_fp32_cn64"] = weighted_rel_err(qc.unpack(gc)[0].astype(np.complex128), x64) if ok_c else None
            acc.append(row)
            if not ok32:
                break
        out["accuracy_fp32_vs_fp64"] = acc

    if not args.no_batch:
        out["batched_sweep"] = batched_sweep_measurement(torch)
    if not args.no_paper_shapes:
        out["paper_shapes"] = paper_shapes_measurement(torch)
    if not args.no_long_pulse:
        out["long_pulse"] = long_pulse_measurement(torch, [int(x) for x in args.long_pulse_checkpoints.split(",")])
    if not args.no_parareal:
        # fine and coarse steps in FP32-CN64 (parareal target 1e-4), and in FP32 storage (1e-5)
        out["parareal"] = parareal_measurement(torch, "fp32_cn64")
        out["parareal_fp32_storage"] = parareal_measurement(torch, "fp32_storage")
    if not args.no_net:
        out["coarse_net"] = coarse_net_measurement(torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, a0, args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

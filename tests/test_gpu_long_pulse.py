"""Long-distance pulse (1024 x 8192, full model, adaptive dz with a 0.05 rad phase limit) at
z checkpoints: the FP64 GPU method against the CPU oracle, and the FP32 modes against the
FP64 GPU method.

The oracle's values after 100, 1000 and 10000 steps (each an independent run from z = 0) are
stored in tests/golden/long_pulse_reference.json, written by
tests/golden/make_long_pulse_reference.py, which calls only oracle/.  The pulse collapses
between z = 10 m and z = 73 m; from there on the trajectory amplifies any perturbation by
about 1e4 (an FP64 run from the FP32-rounded input separates by 2.5e-8 before the collapse
and by 3e-4 after it), so the tolerances at 10000 steps are set by that measured
amplification, not by the per-step rounding.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_1507_05988_amd import fcn
from paper_1507_05988_amd import workloads as wl

pytestmark = pytest.mark.gpu

REF_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_pulse_reference.json")
# FP64 GPU against the oracle, relative: before the collapse the per-step rounding of two
# FP64 codes (measured 2.3e-13 at 1000 steps); after it, that difference amplified ~1e4 times
FP64_TOL = {100: 1e-10, 1000: 1e-10, 10000: 1e-7}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def werr(a, ref):
    nr = ref.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    return math.sqrt(np.sum(w[:, None] * np.abs(a - ref) ** 2) / np.sum(w[:, None] * np.abs(ref) ** 2))


@pytest.fixture(scope="module")
def runs():
    """FP64 adaptive run to every stored checkpoint, its dz log replayed by an FP64 run from the
    FP32-rounded input (the floor), an FP32 run and an FP32-storage run."""
    import torch

    with open(REF_FILE) as fh:
        ref = json.load(fh)
    cps = [c["steps"] for c in ref["checkpoints"]]
    inst = wl.config_long()
    a0 = wl.gaussian_field(inst)
    kw = dict(adaptive=True, max_phase=wl.LONG_MAX_PHASE, dz_min=wl.LONG_DZ_MIN, dz_max=wl.LONG_DZ_MAX)
    p64 = fcn.Plan(inst, precision="fp64", **kw)
    others = {"floor": fcn.Plan(inst, precision="fp64"), "fp32": fcn.Plan(inst, precision="fp32"),
              "fp32_storage": fcn.Plan(inst, precision="fp32_storage"),
              "fp32_cn64": fcn.Plan(inst, precision="fp32_cn64")}
    a32 = a0.astype(np.complex64)
    g64 = p64.pack(a0)
    g = {"floor": others["floor"].pack(a32.astype(np.complex128)), "fp32": others["fp32"].pack(a32),
         "fp32_storage": others["fp32_storage"].pack(a32), "fp32_cn64": others["fp32_cn64"].pack(a32)}
    log = torch.zeros(cps[-1], dtype=torch.float64, device=p64.device)
    out = {}
    done = 0
    for cp in cps:
        say(f"  long pulse 1024x8192: steps {done} -> {cp}")
        p64.propagate(g64, cp - done, dz_log=log[done:cp])
        p64.sync()
        for name, p in others.items():
            p.propagate(g[name], cp - done, dz_log=log[done:cp], replay=True)
            p.sync()
        done = cp
        x64 = p64.unpack(g64)[0]
        rec = {"x64": x64, "log": log[:cp].cpu().numpy(), "diag": p64.split_diag(p64.diagnostics(g64))[0]}
        for name, p in others.items():
            rec[name] = werr(p.unpack(g[name])[0].astype(np.complex128), x64)
        out[cp] = rec
    return ref, out


def test_fp64_against_oracle_checkpoints(runs):
    ref, out = runs
    for c in ref["checkpoints"]:
        n = c["steps"]
        tol = FP64_TOL[n]
        r = out[n]
        lg = r["log"]
        assert abs(lg.sum() / c["z"] - 1) < tol, (n, lg.sum(), c["z"])
        for k, v in c["dz"].items():
            assert abs(lg[int(k)] / v - 1) < tol, (n, k)
        d = r["diag"]
        errs = {k: abs(d[k] / c[k] - 1) for k in ("energy", "i_max", "i_axis", "rho_max", "phi")}
        flu = np.asarray(d["fluence"][::c["fluence_stride"]])
        fr = np.asarray(c["fluence"])
        errs["fluence"] = float(np.max(np.abs(flu - fr)) / fr.max())
        x = r["x64"]
        smp = np.array([x[m, t] for m, t, _, _ in c["field_samples"]])
        want = np.array([complex(re, im) for _, _, re, im in c["field_samples"]])
        errs["field_samples"] = float(np.max(np.abs(smp - want)) / c["abs_max"])
        errs["abs_max"] = abs(np.abs(x).max() / c["abs_max"] - 1)
        say(f"  {n} steps (z = {c['z']:.3f} m): " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        for k, v in errs.items():
            assert v < tol, (n, k, v, tol)


def test_fp32_modes_against_fp64_checkpoints(runs):
    """The FP32-field modes replay the FP64 run's dz log.  Before the collapse: FP32 within the
    per-step bound 1e-6 accumulated over the steps, FP32-CN64 within the 1e-5 target and a third
    of the FP32 error (the column solve sets most of the FP32 error on this wide beam), FP32
    storage within 1e-5.  After it, each mode within a stated multiple of the floor (the FP64 run
    from the same FP32-rounded input)."""
    _, out = runs
    for n, r in out.items():
        say(f"  {n} steps: floor {r['floor']:.2e}, FP32 {r['fp32']:.2e}, FP32-CN64 {r['fp32_cn64']:.2e}, "
            f"FP32 storage {r['fp32_storage']:.2e}")
        if n <= 1000:
            assert r["floor"] < 1e-7
            assert r["fp32"] < n * 1e-6
            assert r["fp32_cn64"] < min(1e-5, r["fp32"] / 3)
            assert r["fp32_storage"] < 1e-5
        else:
            # after the collapse the trajectory amplifies any perturbation ~1e4 times: FP32
            # storage stays at the floor; the FP32-arithmetic row pass of FP32 and FP32-CN64 keeps
            # adding its rounding in the filament and follows a neighbouring trajectory (measured
            # 5.5e-2 and 0.09-0.2 at 1e4 steps, floor 2.9e-4): held to 500 and 2000 times the floor
            assert r["fp32_storage"] < 3 * r["floor"] + 1e-5
            assert r["fp32_cn64"] < 500 * r["floor"]
            assert r["fp32"] < 2000 * r["floor"]

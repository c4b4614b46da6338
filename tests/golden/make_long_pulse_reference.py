"""Writes tests/golden/long_pulse_reference.json: the CPU oracle's long-distance pulse
(1024 x 8192, adaptive dz, full model) after 100, 1000 and 10000 steps, each an independent
run from z = 0.  Stored per checkpoint: z reached, a few dz values, the diagnostics, the
fluence at every 16th radius and the field at 25 fixed grid points.  It calls only oracle/
(and the seeded input builders), so every stored value is the oracle's.

Run: python tests/golden/make_long_pulse_reference.py [--max-steps N]   (about 90 minutes on
8 cores for the 10000-step checkpoint; the file is rewritten after each checkpoint, and a
later run of the same oracle source computes only the checkpoints still missing).  Rewrite
only with a commit that names the passage or reading of the paper that changed the oracle's
arithmetic."""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1507_05988_amd import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "long_pulse_reference.json")
CHECKPOINTS = (100, 1000, 10000)
SAMPLE_ROWS = (0, 8, 32, 128, 512)
SAMPLE_OFFSETS = (-256, -64, 0, 64, 256)  # around the centre of the time window
FLUENCE_STRIDE = 16
DZ_AT = (0, 9, 99, 999, 9999)


def sample_points(nt):
    return [(m, nt // 2 + d) for m in SAMPLE_ROWS for d in SAMPLE_OFFSETS]


def checkpoint(inst, a0, steps):
    t0 = time.time()
    a, log = oracle.propagate_adaptive(inst, a0, steps, wl.LONG_MAX_PHASE, wl.LONG_DZ_MIN, wl.LONG_DZ_MAX)
    d = oracle.diagnostics(inst, a)
    nt = int(inst["nt"])
    return {
        "steps": steps,
        "seconds": round(time.time() - t0, 1),
        "z": float(np.sum(log)),
        "dz": {str(k): float(log[k]) for k in DZ_AT if k < steps},
        "dz_last": float(log[-1]),
        "dz_min": float(np.min(log)),
        "energy": d["energy"], "i_max": d["i_max"], "i_axis": d["i_axis"], "rho_max": d["rho_max"],
        "phi": d["phi"],
        "abs_max": float(np.max(np.abs(a))),
        "fluence_stride": FLUENCE_STRIDE,
        "fluence": [float(x) for x in d["fluence"][::FLUENCE_STRIDE]],
        "field_samples": [[m, n, float(a[m, n].real), float(a[m, n].imag)] for m, n in sample_points(nt)],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-steps", type=int, default=CHECKPOINTS[-1])
    args = ap.parse_args()
    inst = wl.config_long()
    a0 = wl.gaussian_field(inst)
    data = {"about": "CPU oracle, long-distance pulse 1024 x 8192, adaptive dz "
                     f"(max phase {wl.LONG_MAX_PHASE}, dz in [{wl.LONG_DZ_MIN}, {wl.LONG_DZ_MAX}] m), "
                     "independent runs from z = 0",
            "oracle_source_sha256": hashlib.sha256(oracle.source().encode()).hexdigest(),
            "checkpoints": []}
    if os.path.exists(OUT):  # keep the checkpoints an earlier run of the same oracle source wrote
        with open(OUT) as fh:
            old = json.load(fh)
        if old.get("oracle_source_sha256") == data["oracle_source_sha256"]:
            data["checkpoints"] = [c for c in old["checkpoints"] if c["steps"] in CHECKPOINTS]
    have = {c["steps"] for c in data["checkpoints"]}
    for n in CHECKPOINTS:
        if n > args.max_steps:
            break
        if n in have:
            continue
        data["checkpoints"].append(checkpoint(inst, a0, n))
        data["checkpoints"].sort(key=lambda c: c["steps"])
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
            fh.write("\n")
        c = data["checkpoints"][-1]
        print(f"{n} steps: z = {c['z']:.4f} m, dz_last = {c['dz_last']:.3e}, I_max = {c['i_max']:.3e}, "
              f"rho_max = {c['rho_max']:.3e} ({c['seconds']} s)", flush=True)


if __name__ == "__main__":
    main()

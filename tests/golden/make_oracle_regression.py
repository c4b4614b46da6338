"""Writes tests/golden/oracle_regression.json: diagnostics of the CPU oracle on two small seeded
workloads, with the SHA-256 of the oracle's source.  It calls only oracle/ (and the seeded
input builders), so the stored values are the oracle's; tests/test_golden.py recomputes them.
Run: python tests/golden/make_oracle_regression.py  (rewrite only with a commit that names the
passage or reading of the paper that changed the oracle's arithmetic)."""
import hashlib
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1507_05988_amd import workloads as wl  # noqa: E402

CASES = {
    "kerr_pulse_32x128_10_steps": (lambda: wl.config_small(nr=32, nt=128), 1.0, 10),
    "full_model_24x128_6_steps_at_5e17": (lambda: wl.config_full(nr=24, nt=128), None, 6),
}


def compute():
    out = {}
    for name, (make, _, steps) in CASES.items():
        inst = make()
        a0 = wl.gaussian_field(inst)
        if name.startswith("full_model"):
            a0 = a0 * math.sqrt(5e17 / inst["I0"])
        a = oracle.propagate(inst, a0, steps, threads=1)
        d = oracle.diagnostics(inst, a, threads=1)
        out[name] = {"steps": steps, "energy": d["energy"], "i_max": d["i_max"], "i_axis": d["i_axis"],
                     "rho_max": d["rho_max"], "phi": d["phi"],
                     "fluence_first_8": [float(x) for x in d["fluence"][:8]],
                     "field_row0_first_4": [[float(z.real), float(z.imag)] for z in a[0, :4]]}
    return out


def source_hash():
    return hashlib.sha256(oracle.source().encode()).hexdigest()


if __name__ == "__main__":
    data = {"about": "oracle diagnostics after a few steps of two seeded workloads (regression values)",
            "oracle_source_sha256": source_hash(), "cases": compute()}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print("written")

"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

Each workload runs at its real grid (and batch) with the plan options bench.py uses; the CPU
oracle follows the same steps on the whole field where that takes seconds, else on sampled
instances of a batch (each instance of a batch is bit-identical to the instance run alone,
tested separately, so a sampled instance checks the batched launch).  Tolerances: FP64 1e-10;
FP32 and FP32-CN64 the per-step bound 1e-6 accumulated over the steps; FP32 storage 1e-6 over
<= 100 steps.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1507_05988_amd import fcn
from paper_1507_05988_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def werr(a, ref):
    nr = ref.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    return math.sqrt(np.sum(w[:, None] * np.abs(a - ref) ** 2) / np.sum(w[:, None] * np.abs(ref) ** 2))


def _run(insts, precision, nsteps, fields, **kw):
    plan = fcn.Plan(insts, precision=precision, **kw)
    f = plan.pack(fields)
    plan.step(f, nsteps)
    plan.sync()
    return plan.unpack(f)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 60 * 1e-6), ("fp32_storage", 1e-6),
                                           ("fp32_cn64", 60 * 1e-6)])
def test_full_model_pulse_full_size(precision, tol):
    """Full-model pulse, 512 x 2048, 60 steps of 5 mm from z = 0 (the bench workload)."""
    inst = wl.config_full()
    a0 = wl.gaussian_field(inst)
    a_in = a0 if precision == "fp64" else a0.astype(np.complex64)
    got = _run(inst, precision, 60, a_in)[0].astype(np.complex128)
    want = oracle.propagate(inst, a_in.astype(np.complex128), 60)
    e = werr(got, want)
    say(f"  full model 512x2048, 60 steps, {precision}: {e:.3e}")
    assert e < tol


@pytest.mark.parametrize("precision,tol", [("fp32", wl.BATCH_STEPS * 1e-6), ("fp32_cn64", 1e-5)])
def test_batched_sweep_full_size_sampled(precision, tol):
    """The 64-pulse sweep (7.3e7 points) in one plan, 100 steps; the oracle runs the smallest,
    a middle and the largest instance alone.  FP32: the per-step bound; FP32-CN64: the 1e-5
    target over the whole run."""
    insts = wl.config_batch()
    fields = [wl.gaussian_field(i, np.complex64) for i in insts]
    got = _run(insts, precision, wl.BATCH_STEPS, fields)
    sizes = [i["nr"] * i["nt"] for i in insts]
    order = np.argsort(sizes, kind="stable")
    for k in (order[0], order[len(order) // 2], order[-1]):
        inst = insts[k]
        want = oracle.propagate(inst, fields[k].astype(np.complex128), wl.BATCH_STEPS)
        e = werr(got[k].astype(np.complex128), want)
        say(f"  {precision} instance {k} ({inst['nr']}x{inst['nt']}): {e:.3e}")
        assert e < tol


def test_long_pulse_full_size_adaptive():
    """Long-distance pulse, 1024 x 8192, adaptive dz: 16 steps FP64 against the oracle (field and
    dz log), and FP32 replaying that dz log."""
    import torch
    inst = wl.config_long()
    a0 = wl.gaussian_field(inst)
    n = 16
    plan = fcn.Plan(inst, precision="fp64", adaptive=True, max_phase=wl.LONG_MAX_PHASE, dz_min=wl.LONG_DZ_MIN,
                    dz_max=wl.LONG_DZ_MAX)
    log = torch.zeros(n, dtype=torch.float64, device=plan.device)
    f = plan.pack(a0)
    plan.propagate(f, n, dz_log=log)
    plan.sync()
    got = plan.unpack(f)[0]
    want, wlog = oracle.propagate_adaptive(inst, a0, n, wl.LONG_MAX_PHASE, wl.LONG_DZ_MIN, wl.LONG_DZ_MAX)
    glog = log.cpu().numpy()
    e = werr(got, want)
    say(f"  long pulse 1024x8192 FP64 adaptive, {n} steps: {e:.3e}; dz {glog[0]:.3e} .. {glog[-1]:.3e}")
    assert np.max(np.abs(glog / wlog - 1)) < 1e-12
    assert e < 1e-10
    p32 = fcn.Plan(inst, precision="fp32")
    g = p32.pack(a0.astype(np.complex64))
    p32.propagate(g, n, dz_log=log, replay=True)
    p32.sync()
    e32 = werr(p32.unpack(g)[0].astype(np.complex128), want)
    say(f"  FP32 replay: {e32:.3e}")
    assert e32 < n * 1e-6


def test_learned_coarse_trajectory_full_size():
    """A learned-coarse trajectory (512 x 2048, Kerr only), one 50-step window, FP64 and FP32."""
    inst = wl.config_parareal_trajectory(2000)
    a0 = wl.gaussian_field(inst)
    want = oracle.propagate(inst, a0, 50)
    e64 = werr(_run(inst, "fp64", 50, a0)[0], want)
    e32 = werr(_run(inst, "fp32", 50, a0.astype(np.complex64))[0].astype(np.complex128), want)
    say(f"  trajectory 2000, 50 steps: FP64 {e64:.3e}, FP32 {e32:.3e}")
    assert e64 < 1e-10 and e32 < 50 * 1e-6

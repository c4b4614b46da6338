"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

Each workload runs at its real grid (and batch) with the plan options bench.py uses; the CPU
oracle follows the same steps on the whole field where that takes seconds, else on sampled
instances of a batch (each instance of a batch is bit-identical to the instance run alone,
tested separately, so a sampled instance checks the batched launch).  Tolerances: FP64 1e-10;
the FP32-field modes the FP32 target 1e-5 (FP32 storage 1e-6) in the r-weighted field norm, the
relative error the target is stated in.  Element by element (largest element error over the
largest element) the bound is ELEMENTWISE times that: the largest element error sits on the axis
at the focus, where the r-weighted norm gives least weight, and measures 4-9 times the field
error in every FP32 mode.  Plain FP32, which misses the target on the sweep's largest pulses, is
held to the per-step bound 1e-6 accumulated over the steps under a test name that says so.
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


ELEMENTWISE = 10  # element-wise bound over the field-norm bound (see the module docstring)


def elerr(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _run(insts, precision, nsteps, fields, **kw):
    plan = fcn.Plan(insts, precision=precision, **kw)
    f = plan.pack(fields)
    plan.step(f, nsteps)
    plan.sync()
    return plan.unpack(f)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("fp32_storage", 1e-6),
                                           ("fp32_cn64", 1e-5)])
def test_full_model_pulse_full_size(precision, tol):
    """Full-model pulse, 512 x 2048, 60 steps of 5 mm from z = 0 (the bench workload), field
    norm and element by element against the oracle from the same input."""
    inst = wl.config_full()
    a0 = wl.gaussian_field(inst)
    a_in = a0 if precision == "fp64" else a0.astype(np.complex64)
    got = _run(inst, precision, 60, a_in)[0].astype(np.complex128)
    want = oracle.propagate(inst, a_in.astype(np.complex128), 60)
    e, el = werr(got, want), elerr(got, want)
    say(f"  full model 512x2048, 60 steps, {precision}: field {e:.3e}, element-wise {el:.3e}")
    assert e < tol and el < ELEMENTWISE * tol


def _sweep_sampled(precision):
    """The 64-pulse sweep (7.56e7 points) in one graph-replayed plan on its own stream, 100
    steps; the oracle runs the smallest, a middle and the largest instance alone."""
    import torch
    insts = wl.config_batch()
    fields = [wl.gaussian_field(i, np.complex64) for i in insts]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        got = _run(insts, precision, wl.BATCH_STEPS, fields, use_graph=True, stream=stream)
    sizes = [i["nr"] * i["nt"] for i in insts]
    order = np.argsort(sizes, kind="stable")
    out = []
    for k in (order[0], order[len(order) // 2], order[-1]):
        inst = insts[k]
        want = oracle.propagate(inst, fields[k].astype(np.complex128), wl.BATCH_STEPS)
        g = got[k].astype(np.complex128)
        out.append((k, werr(g, want), elerr(g, want)))
        say(f"  {precision} instance {k} ({inst['nr']}x{inst['nt']}): field {out[-1][1]:.3e}, "
            f"element-wise {out[-1][2]:.3e}")
    return insts, fields, got, out


def test_batched_sweep_full_size_fp32_cn64():
    """The headline mode on the headline workload: the sampled instances within the FP32 target
    1e-5 of the oracle (field norm; element-wise within ELEMENTWISE times that), and every one of
    the 64 instances within 1e-5 of the FP64 GPU method (which the oracle pins to 1e-10)."""
    insts, fields, got, out = _sweep_sampled("fp32_cn64")
    for k, e, el in out:
        assert e < 1e-5 and el < ELEMENTWISE * 1e-5, (k, e, el)
    ref = _run(insts, "fp64", wl.BATCH_STEPS, [f.astype(np.complex128) for f in fields])
    k0 = out[0][0]
    assert werr(ref[k0], oracle.propagate(insts[k0], fields[k0].astype(np.complex128), wl.BATCH_STEPS)) < 1e-10
    errs = [werr(g.astype(np.complex128), r) for g, r in zip(got, ref)]
    say(f"  all 64 instances vs FP64: max {max(errs):.3e}, median {np.median(errs):.3e}")
    assert max(errs) < 1e-5


def test_batched_sweep_full_size_plain_fp32_reported_not_at_target():
    """Plain FP32 on the sweep is not at the 1e-5 target on its largest pulses (the FP32
    elimination factors and twiddles repeat the same rounding every step); it is held to the
    per-step bound 1e-6 accumulated over the 100 steps."""
    _, _, _, out = _sweep_sampled("fp32")
    for k, e, el in out:
        assert e < wl.BATCH_STEPS * 1e-6 and el < ELEMENTWISE * wl.BATCH_STEPS * 1e-6, (k, e, el)


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
    for prec, tol in (("fp32", n * 1e-6), ("fp32_cn64", 1e-5)):
        p32 = fcn.Plan(inst, precision=prec)
        g = p32.pack(a0.astype(np.complex64))
        p32.propagate(g, n, dz_log=log, replay=True)
        p32.sync()
        x = p32.unpack(g)[0].astype(np.complex128)
        e32, el32 = werr(x, want), elerr(x, want)
        say(f"  {prec} replay: field {e32:.3e}, element-wise {el32:.3e}")
        assert e32 < tol and el32 < ELEMENTWISE * tol


def test_learned_coarse_trajectory_full_size():
    """A learned-coarse trajectory (512 x 2048, Kerr only), one 50-step window, FP64 and FP32."""
    inst = wl.config_parareal_trajectory(2000)
    a0 = wl.gaussian_field(inst)
    want = oracle.propagate(inst, a0, 50)
    e64 = werr(_run(inst, "fp64", 50, a0)[0], want)
    e32 = werr(_run(inst, "fp32", 50, a0.astype(np.complex64))[0].astype(np.complex128), want)
    say(f"  trajectory 2000, 50 steps: FP64 {e64:.3e}, FP32 {e32:.3e}")
    assert e64 < 1e-10 and e32 < 50 * 1e-6


@pytest.mark.parametrize("name", ["application_1350x1024", "timing_2112x2048"])
def test_paper_grids_full_size(name):
    """The paper's own grids at full size: the 1.1 km application run's Nr = 1350, Nt = 1024
    (Sec. 5.2) and the timing example's Nr = 2112, Nt = 2048 (Sec. 5.1, Table 2), a few full-model
    steps against the oracle on the whole field: FP64 within 1e-10, FP32-CN64 within the 1e-5
    target (field norm and element-wise)."""
    inst = wl.config_paper_application() if name.startswith("application") else wl.config_paper_timing()
    a0 = wl.gaussian_field(inst)
    n = 4
    want = oracle.propagate(inst, a0, n)
    got64 = _run(inst, "fp64", n, a0)[0]
    e64 = werr(got64, want)
    a32 = a0.astype(np.complex64)
    want32 = oracle.propagate(inst, a32.astype(np.complex128), n)
    got32 = _run(inst, "fp32_cn64", n, a32)[0].astype(np.complex128)
    e32, el32 = werr(got32, want32), elerr(got32, want32)
    say(f"  {name}, {n} steps: FP64 {e64:.3e}; FP32-CN64 field {e32:.3e}, element-wise {el32:.3e}")
    assert e64 < 1e-10 and elerr(got64, want) < 1e-10
    assert e32 < 1e-5 and el32 < 1e-5

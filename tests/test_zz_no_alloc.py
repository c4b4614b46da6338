"""The allocation-free entry point fcn_step_scratch (the library's static device scratch in place
of the caller's workspace) gives the same fields as fcn_step on a bound plan, on two calls in a
row of which the second is smaller, through the C ABI."""
import math

import numpy as np
import pytest

from paper_1507_05988_amd import fcn
from paper_1507_05988_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _case(insts, precision, a0s, nsteps):
    """fcn_step on a plan bound to a torch workspace, and fcn_step_scratch on a second plan of the
    same instances: both from the same initial fields."""
    ref_plan = fcn.Plan(insts, precision=precision)
    f_ref = ref_plan.pack(a0s)
    ref_plan.step(f_ref, nsteps)
    ref_plan.sync()
    plan = fcn.Plan(insts, precision=precision)
    f = plan.pack(a0s)
    plan.step_scratch(f, nsteps)
    plan.torch.cuda.synchronize()
    return ref_plan.unpack(f_ref), plan.unpack(f), plan


def test_step_scratch_matches_step_on_two_calls():
    print("[no-alloc] call 1: ragged full-model batch, FP32-CN64", flush=True)
    big = [wl.config_full(nr=96, nt=512), wl.config_full(nr=40, nt=256), wl.config_full(nr=130, nt=1024)]
    a_big = [(wl.gaussian_field(i) * math.sqrt(6e17 / i["I0"])).astype(np.complex64) for i in big]
    ref, got, plan = _case(big, "fp32_cn64", a_big, 7)
    assert plan.workspace_bytes <= fcn.SCRATCH_BYTES
    for r, g, a in zip(ref, got, a_big):
        assert np.array_equal(r.view(np.uint32), g.view(np.uint32))  # the same kernels: bit for bit
        assert np.max(np.abs(g - a)) > 1e-3 * np.max(np.abs(a))  # and the steps did something
    print("[no-alloc] call 2: one smaller Kerr pulse, FP64", flush=True)
    small = [wl.config_small(nr=33, nt=128)]
    a_small = [wl.gaussian_field(small[0])]
    ref2, got2, plan2 = _case(small, "fp64", a_small, 5)
    assert plan2.workspace_bytes < plan.workspace_bytes
    assert np.array_equal(ref2[0].view(np.uint64), got2[0].view(np.uint64))
    assert np.max(np.abs(got2[0] - a_small[0])) > 1e-6 * np.max(np.abs(a_small[0]))


def test_step_scratch_leaves_the_bound_workspace_alone():
    """A bound plan keeps its own step state: fcn_step after fcn_step_scratch continues the plan's
    own counter and gives the same field as the same fcn_step calls without it."""
    print("[no-alloc] bound plan: step, scratch call, step", flush=True)
    inst = wl.config_full(nr=64, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
    p = fcn.Plan(inst, precision="fp64")
    f = p.pack(a0)
    p.step(f, 3)
    other = p.pack(a0)
    p.step_scratch(other, 4)
    p.step(f, 2)
    p.sync()
    q = fcn.Plan(inst, precision="fp64")
    g = q.pack(a0)
    q.step(g, 3)
    q.step(g, 2)
    q.sync()
    assert np.array_equal(p.unpack(f)[0].view(np.uint64), q.unpack(g)[0].view(np.uint64))
    r = q.pack(a0)
    q.step(r, 4)
    q.sync()
    assert np.array_equal(p.unpack(other)[0].view(np.uint64), q.unpack(r)[0].view(np.uint64))

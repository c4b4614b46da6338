"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: FP64 stages <= 1e-12 relative; FP64 whole runs <= 1e-10 relative in the
r-weighted norm; FP32 field error <= 1e-5 (the FP32 target), with per-output errors for
fluence and rho_max at the same target.  The largest element error over the largest element
is held to ELEMENTWISE times the field bound: it sits on the axis at the focus, where the
r-weighted norm gives least weight, and measures 4-9 times the field error in every FP32 mode.
Inputs are seeded synthetic Gaussians or seeded random fields.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1507_05988_amd import fcn
from paper_1507_05988_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def werr(a, ref):
    """r-weighted relative L2 error (weights 1/8, 1, 2, ...; r_max row excluded)."""
    nr = ref.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    num = np.sum(w[:, None] * np.abs(a - ref) ** 2)
    den = np.sum(w[:, None] * np.abs(ref) ** 2)
    return math.sqrt(num / den)


ELEMENTWISE = 10


def relmax(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _plan(insts, precision, **kw):
    return fcn.Plan(insts, precision=precision, **kw)


# ------------------------------------------------------------------ stage parity

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nt", [64, 128, 256, 1024, 2048, 4096, 8192])
def test_fft_stages(precision, nt):
    say(f"fft stage {precision} nt={nt}")
    inst = wl.config_small(nr=19, nt=nt)  # ragged row count: several workgroups and a tail
    a = wl.random_field(19, nt, seed=nt)
    a[-1] = wl.random_field(2, nt, seed=1)[0]
    plan = _plan(inst, precision)
    f = plan.pack(a)
    plan.stage(fcn.STAGE_FFT, f)
    got = plan.unpack(f)[0]
    want = oracle.fft_rows(a)
    tol = 1e-14 * math.log2(nt) * 4 if precision == "fp64" else 3e-7 * math.log2(nt)
    assert relmax(got, want) < tol
    plan.stage(fcn.STAGE_IFFT, f)
    back = plan.unpack(f)[0]
    assert relmax(back, a) < tol
    plan.sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nr", [3, 4, 8, 37, 128, 512, 1024, 2048, 2112, 4096])
def test_cn_stage(precision, nr):
    say(f"cn stage {precision} nr={nr}")
    nt = 64
    inst = wl.config_full(nr=nr, nt=nt)
    a = wl.random_field(nr, nt, seed=nr)
    plan = _plan(inst, precision)
    for dz in (5e-3, 0.2):  # 0.2 m: far from diagonal dominance
        f = plan.pack(a)
        plan.stage(fcn.STAGE_CN, f, dz)
        got = plan.unpack(f)[0]
        want = oracle.cn_columns(inst, a, dz)
        # FP32: the partitioned solve's reduced system has 2 nr / 16 unknowns per column
        tol = 1e-12 if precision == "fp64" else 2e-5 * max(1.0, nr / 2048)
        assert relmax(got, want) < tol, (dz, relmax(got, want))
    plan.sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tiles", [(8, 8), (16, 16), (4, 16), (32, 8), (16, 8), (2, 8), (2, 16), (1, 8), (1, 16),
                                   (8, 6), (4, 6), (2, 6), (1, 6), (8, 4), (4, 4), (2, 4), (1, 4)])
def test_cn_stage_tiles(precision, tiles):
    nr, nt = 120, 128  # W * ceil(nr/L) stays within 512 threads for every tile
    if precision == "fp64" and tiles[1] == 16:
        pytest.skip("FP64 with 16 rows per thread is not a supported tile")
    say(f"cn tiles {precision} {tiles}")
    inst = wl.config_small(nr=nr, nt=nt)
    a = wl.random_field(nr, nt, seed=3)
    plan = _plan(inst, precision, col_tile=tiles[0], col_rows=tiles[1])
    f = plan.pack(a)
    plan.stage(fcn.STAGE_CN, f, 0.05)
    want = oracle.cn_columns(inst, a, 0.05)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert relmax(plan.unpack(f)[0], want) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nt", [64, 256, 2048, 8192])
@pytest.mark.parametrize("terms", [wl.KERR, wl.ALL_TERMS & ~(wl.DIFFRACTION | wl.GVD), "kerr_n8", "avalanche"])
def test_nl_stage(precision, nt, terms):
    """One nonlinear sub-step (Eq. nonlinearpart) against the oracle: Kerr only, every term, the
    whole Kerr sum to j = 4 (n2, n4, n6, n8) with every term, and every term with the avalanche
    rate in the density equation."""
    say(f"nl stage {precision} nt={nt} terms={terms}")
    nr = 6
    inst = wl.config_full(nr=nr, nt=nt)
    if terms == "kerr_n8":
        inst.update(n6=wl.config_higher_kerr()["n6"], n8=wl.config_higher_kerr()["n8"])
        terms = wl.ALL_TERMS & ~(wl.DIFFRACTION | wl.GVD)
    elif terms == "avalanche":
        inst["U_i"] = wl.U_I_O2
        terms = (wl.ALL_TERMS | wl.AVALANCHE) & ~(wl.DIFFRACTION | wl.GVD)
    inst["terms"] = terms
    rng = np.random.default_rng(nt)
    t = inst["t_min"] + np.arange(nt) * (inst["t_max"] - inst["t_min"]) / nt
    env = np.exp(-(t / inst["tau"]) ** 2)
    amp = np.sqrt(6e17) * (0.3 + 0.7 * rng.random((nr, 1))) * env[None, :]
    a = amp * np.exp(2j * np.pi * rng.random((nr, nt))) * (1 + 0.05 * rng.standard_normal((nr, nt)))
    h = 2.5e-3
    plan = _plan(inst, precision)
    f = plan.pack(a)
    plan.stage(fcn.STAGE_NL, f, h)
    got = plan.unpack(f)[0]
    want = oracle.nl_half(inst, a, h)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert relmax(got, want) < tol


# --------------------------------------------------------------- whole-step parity

def _run(inst, precision, nsteps, a0=None, **kw):
    plan = _plan(inst, precision, **kw)
    a0 = wl.gaussian_field(inst) if a0 is None else a0
    f = plan.pack(a0)
    plan.step(f, nsteps)
    plan.sync()
    return plan.unpack(f)[0], plan


def test_small_kerr_fp64_matches_oracle():
    """Plain Kerr case, Nr=128, Nt=256, 100 steps of 1 cm, FP64."""
    inst = wl.config_small()
    say("small kerr fp64")
    got, _ = _run(inst, "fp64", wl.SMALL_STEPS)
    want = oracle.propagate(inst, wl.gaussian_field(inst), wl.SMALL_STEPS)
    e = werr(got, want)
    say(f"  field error {e:.3e}")
    assert e < 1e-10


def test_small_kerr_fp32_matches_oracle():
    inst = wl.config_small()
    say("small kerr fp32")
    got, _ = _run(inst, "fp32", wl.SMALL_STEPS)
    want = oracle.propagate(inst, wl.gaussian_field(inst), wl.SMALL_STEPS)
    e = werr(got.astype(np.complex128), want)
    say(f"  field error {e:.3e}")
    assert e < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_step_error(precision):
    """One full-model step from an ionising state: FP64 to 1e-12, FP32 to 1e-6 (a few FP32
    roundings per pass; this per-step bound is what FP32 guarantees)."""
    inst = wl.config_full(nr=96, nt=512)
    a0 = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
    a0 = oracle.propagate(inst, a0, 5)  # a state with structure in r and t
    got, _ = _run(inst, precision, 1, a0=a0 if precision == "fp64" else a0.astype(np.complex64))
    want = oracle.propagate(inst, a0 if precision == "fp64" else a0.astype(np.complex64).astype(np.complex128), 1)
    e = werr(got.astype(np.complex128), want)
    say(f"  one-step field error {precision}: {e:.3e}")
    assert e < (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("precision", ["fp32_cn64", "fp32"])
@pytest.mark.parametrize("tiles", [(1, 4), (2, 6), (4, 8), (8, 4), (16, 8), (32, 8), (2, 16)])
def test_pair_order_step_tiles(precision, tiles):
    """Two full-model steps of a ragged two-pulse batch (45 x 64 and 37 x 128) with every kind
    of column tile.  Inside a z-step an FP32 spectrum holds columns s and nt - s side by side
    and the column solve moves a pair with one access; the lone columns 0 and nt/2 share the
    first entry and sit in the first and last tile of each pulse (at W = 32 the last tile holds
    column nt/2 alone).  Against the oracle from the same FP32 input, 2e-6 (two steps of the
    FP32 per-step bound)."""
    if precision == "fp32_cn64" and tiles[1] == 16:
        pytest.skip("FP64 arithmetic with 16 rows per thread is not a supported tile")
    say(f"pair order step {precision} tiles {tiles}")
    insts = [wl.config_full(nr=45, nt=64), wl.config_full(nr=37, nt=128)]
    a0 = []
    for inst in insts:
        a = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
        a0.append(oracle.propagate(inst, a, 3).astype(np.complex64))  # structure in r and t
    plan = _plan(insts, precision, col_tile=tiles[0], col_rows=tiles[1])
    f = plan.pack(a0)
    plan.step(f, 2)
    plan.sync()
    got = plan.unpack(f)
    for inst, a, g in zip(insts, a0, got):
        want = oracle.propagate(inst, a.astype(np.complex128), 2)
        e = werr(g.astype(np.complex128), want)
        say(f"  {inst['nr']}x{inst['nt']}: field error {e:.3e}")
        assert e < 2e-6


def _full_physics_40(precision):
    inst = wl.config_full(nr=96, nt=512)
    a0 = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
    a_in = a0 if precision == "fp64" else a0.astype(np.complex64)
    got, plan = _run(inst, precision, 40, a0=a_in)
    want = oracle.propagate(inst, a_in.astype(np.complex128), 40)
    dg = oracle.diagnostics(inst, want)
    assert dg["rho_max"] > 1e20  # the density term is exercised
    g = got.astype(np.complex128)
    d = plan.split_diag(plan.diagnostics(plan.pack(got)))[0]
    errs = {"field": werr(g, want), "elementwise": relmax(g, want),
            "fluence": float(np.max(np.abs(d["fluence"] - dg["fluence"])) / np.max(dg["fluence"])),
            "rho_max": abs(d["rho_max"] / dg["rho_max"] - 1)}
    say(f"  full physics {precision}, 40 steps: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    return errs


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_cn64", 1e-5), ("fp32_storage", 1e-5)])
def test_full_physics_reduced_grid(precision, tol):
    """Full model (Kerr n2+n4, plasma, MPA, collisions) on a reduced grid, 40 steps of 5 mm
    from the ionising regime (the oracle amplifies a 1e-15 input perturbation to ~3e-14 here),
    from the same (FP32-rounded where the field is FP32) input.  Every output within the FP32
    target of 1e-5 of the oracle for the FP32-field modes that claim it, FP64 within 1e-10:
    the r-weighted field error, the fluence and the peak density (the largest element error over
    the largest element within ELEMENTWISE times the bound)."""
    errs = _full_physics_40(precision)
    for k, v in errs.items():
        assert v < (ELEMENTWISE * tol if k == "elementwise" else tol), (k, v)


def test_full_physics_reduced_grid_plain_fp32_reported_not_at_target():
    """Plain FP32 on the same 40 ionising steps is not at the 1e-5 target (its transform and
    elimination roundings repeat from step to step; measured ~2.4e-5 in the field): the test
    holds it to the per-step bound 1e-6 accumulated over the 40 steps, and checks that the two
    precision remedies are both below it."""
    errs = _full_physics_40("fp32")
    assert errs["field"] < 40 * 1e-6 and errs["elementwise"] < ELEMENTWISE * 40 * 1e-6
    assert _full_physics_40("fp32_cn64")["field"] < errs["field"]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_cn64", 1e-5), ("fp32_storage", 1e-5)])
def test_higher_order_kerr_and_chirp(precision, tol):
    """The whole Kerr sum of Eq. nlse (n2, n4, n6, n8 of alternating sign) with plasma, MPA and
    collisions, from a chirped pulse (Eq. gauss with C = -1.5), 30 steps of 5 mm through the
    C ABI against the oracle: field, element-wise, fluence and peak density."""
    inst = wl.config_higher_kerr(nr=96, nt=512)
    a0 = wl.gaussian_field(inst)
    assert abs(np.angle(a0[0, 3 * 512 // 8] / a0[0, 256])) > 0.1  # the input is chirped
    a_in = a0 if precision == "fp64" else a0.astype(np.complex64)
    got, plan = _run(inst, precision, 30, a0=a_in)
    want = oracle.propagate(inst, a_in.astype(np.complex128), 30)
    dg = oracle.diagnostics(inst, want)
    g = got.astype(np.complex128)
    d = plan.split_diag(plan.diagnostics(plan.pack(got)))[0]
    errs = {"field": werr(g, want), "elementwise": relmax(g, want),
            "fluence": float(np.max(np.abs(d["fluence"] - dg["fluence"])) / np.max(dg["fluence"])),
            "rho_max": abs(d["rho_max"] / dg["rho_max"] - 1)}
    # the n6 and n8 terms matter: dropping them moves the oracle's own result far beyond tol
    off = dict(inst, n6=0.0, n8=0.0)
    assert werr(oracle.propagate(off, a_in.astype(np.complex128), 30), want) > 1e-3
    say(f"  higher-order Kerr + chirp {precision}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < (ELEMENTWISE * tol if k == "elementwise" else tol), (k, v)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_cn64", 1e-5), ("fp32_storage", 1e-5)])
def test_avalanche_ionisation_run(precision, tol):
    """Avalanche ionisation (sigma_c / U_i) I rho added to the density rate, with every other term,
    30 steps of 5 mm at 7e17 W/m^2 through the C ABI against the oracle: field, fluence and peak
    density within the bound (element-wise within ELEMENTWISE times it); the avalanche moves the
    oracle's own peak density by more than 1 %."""
    inst = wl.config_avalanche(nr=96, nt=512)
    a0 = wl.gaussian_field(inst)
    a_in = a0 if precision == "fp64" else a0.astype(np.complex64)
    got, plan = _run(inst, precision, 30, a0=a_in)
    want = oracle.propagate(inst, a_in.astype(np.complex128), 30)
    dg = oracle.diagnostics(inst, want)
    g = got.astype(np.complex128)
    d = plan.split_diag(plan.diagnostics(plan.pack(got)))[0]
    errs = {"field": werr(g, want), "elementwise": relmax(g, want),
            "fluence": float(np.max(np.abs(d["fluence"] - dg["fluence"])) / np.max(dg["fluence"])),
            "rho_max": abs(d["rho_max"] / dg["rho_max"] - 1)}
    off = dict(inst, terms=inst["terms"] & ~wl.AVALANCHE)
    d_off = oracle.diagnostics(off, oracle.propagate(off, a_in.astype(np.complex128), 30))
    assert dg["rho_max"] > 1.01 * d_off["rho_max"]
    say(f"  avalanche {precision}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
        + f"; rho_max {dg['rho_max']:.3e} (without avalanche {d_off['rho_max']:.3e})")
    for k, v in errs.items():
        assert v < (ELEMENTWISE * tol if k == "elementwise" else tol), (k, v)


def test_fp64_error_tracks_conditioning_on_unstable_trajectory():
    """40 steps of 2 cm at 6e17 W/m^2 put ~0.5 rad of nonlinear phase in each half step and the
    trajectory is ill-conditioned: the oracle itself turns a 1e-15 relative input perturbation
    into ~1e-6.  The FP64 GPU error must stay within a small factor of that amplification."""
    inst = wl.config_full(nr=96, nt=512)
    inst["dz"] = 2e-2
    a0 = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
    rng = np.random.default_rng(0)
    pert = a0 * (1 + 1e-15 * rng.standard_normal(a0.shape))
    want = oracle.propagate(inst, a0, 40)
    kappa = werr(oracle.propagate(inst, pert, 40), want)
    got, _ = _run(inst, "fp64", 40, a0=a0)
    e = werr(got, want)
    say(f"  amplification of 1e-15: {kappa:.3e}; GPU FP64 error {e:.3e}")
    assert kappa > 1e-9  # the case is the ill-conditioned one
    assert e < 100 * kappa


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diagnostics_match_oracle(precision):
    inst = wl.config_full(nr=64, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    plan = _plan(inst, precision)
    f = plan.pack(a0)
    diag = plan.propagate(f, 6, diag_every=3)
    plan.sync()
    recs = [plan.split_diag(diag[i])[0] for i in range(3)]
    b = a0.copy()
    for i, r in enumerate(recs):
        want = oracle.diagnostics(inst, b)
        tol = 1e-11 if precision == "fp64" else 1e-5
        for key in ("energy", "i_max", "i_axis", "rho_max", "phi"):
            assert abs(r[key] / want[key] - 1) < tol, (i, key, r[key], want[key])
        assert np.max(np.abs(r["fluence"] - want["fluence"])) < tol * np.max(want["fluence"])
        assert r["step"] == 3 * i
        assert abs(r["z"] - 3 * i * inst["dz"]) < 1e-15
        b = oracle.propagate(inst, b, 3)


def test_adaptive_dz_matches_oracle():
    inst = wl.config_full(nr=48, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    plan = _plan(inst, "fp64", adaptive=True, max_phase=0.05, dz_min=1e-6, dz_max=1e-2)
    import torch
    log = torch.zeros(12, dtype=torch.float64, device=plan.device)
    f = plan.pack(a0)
    plan.propagate(f, 12, dz_log=log)
    plan.sync()
    got = plan.unpack(f)[0]
    want, wlog = oracle.propagate_adaptive(inst, a0, 12, 0.05, 1e-6, 1e-2)
    glog = log.cpu().numpy()
    assert np.max(np.abs(glog / wlog - 1)) < 1e-12, (glog, wlog)
    assert len(set(np.round(wlog, 12))) > 1  # the step length actually adapts
    assert werr(got, want) < 1e-10


def test_adaptive_dz_fp32_cn64_tracks_fp64():
    """FP32-CN64 with its own adaptive dz: the phase-rate rule sees the FP32 field, so its dz
    sequence stays within the field error of the FP64 run's and the fields agree to the
    FP32-CN64 accuracy."""
    import torch
    inst = wl.config_full(nr=48, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    kw = dict(adaptive=True, max_phase=0.05, dz_min=1e-6, dz_max=1e-2)
    logs, fields = {}, {}
    for prec in ("fp64", "fp32_cn64"):
        plan = _plan(inst, prec, **kw)
        log = torch.zeros(20, dtype=torch.float64, device=plan.device)
        f = plan.pack(a0 if prec == "fp64" else a0.astype(np.complex64))
        plan.propagate(f, 20, dz_log=log)
        plan.sync()
        logs[prec] = log.cpu().numpy()
        fields[prec] = plan.unpack(f)[0].astype(np.complex128)
    dzerr = float(np.max(np.abs(logs["fp32_cn64"] / logs["fp64"] - 1)))
    e = werr(fields["fp32_cn64"], fields["fp64"])
    say(f"  fp32-cn64 adaptive, 20 steps: dz {dzerr:.2e}, field {e:.2e}")
    assert len(set(np.round(logs["fp64"], 12))) > 1
    assert dzerr < 1e-5 and e < 20 * 1e-6


def test_replay_dz_log_fp32():
    """FP32 run replaying the FP64 run's dz sequence lands on the FP64 trajectory."""
    import torch
    inst = wl.config_full(nr=48, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    p64 = _plan(inst, "fp64", adaptive=True)
    log = torch.zeros(10, dtype=torch.float64, device=p64.device)
    f64 = p64.pack(a0)
    p64.propagate(f64, 10, dz_log=log)
    p64.sync()
    p32 = _plan(inst, "fp32")
    f32 = p32.pack(a0)
    p32.propagate(f32, 10, dz_log=log, replay=True)
    p32.sync()
    e = werr(p32.unpack(f32)[0].astype(np.complex128), p64.unpack(f64)[0])
    assert e < 1e-5


# ------------------------------------------------------------- batching and graphs

def test_ragged_batch_is_bitwise_instance_invariant():
    """Each instance of a ragged batch equals the same instance run alone, bit for bit
    (the decomposition-invariance of the paper's Sec. 5.1, on the GPU)."""
    insts = wl.config_batch(count=6, seed=11)
    for i in insts:
        i["nr"] = min(i["nr"], 256)
    say("ragged batch: " + ", ".join(f"{i['nr']}x{i['nt']}" for i in insts))
    batch = _plan(insts, "fp32")
    f = batch.pack([wl.gaussian_field(i, np.complex64) for i in insts])
    batch.step(f, 5)
    batch.sync()
    outs = batch.unpack(f)
    for k, inst in enumerate(insts):
        single, _ = _run(inst, "fp32", 5, a0=wl.gaussian_field(inst, np.complex64))
        assert np.array_equal(single.view(np.uint32), outs[k].view(np.uint32)), k


def test_ragged_batch_matches_oracle_fp64():
    insts = wl.config_batch(count=3, seed=5)
    for i in insts:
        i["nr"] = min(i["nr"], 128)
        i["nt"] = min(i["nt"], 1024)
    plan = _plan(insts, "fp64")
    f = plan.pack([wl.gaussian_field(i) for i in insts])
    plan.step(f, 4)
    plan.sync()
    for inst, got in zip(insts, plan.unpack(f)):
        want = oracle.propagate(inst, wl.gaussian_field(inst), 4)
        assert werr(got, want) < 1e-11


def test_graph_replay_equals_eager():
    import torch
    inst = wl.config_small()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = _plan(inst, "fp32", stream=stream)
        graph = _plan(inst, "fp32", use_graph=True, stream=stream)
        a0 = wl.gaussian_field(inst, np.complex64)
        fe, fg = eager.pack(a0), graph.pack(a0)
        eager.step(fe, 40)
        graph.step(fg, 40)  # 2 graph replays of 16 steps + eager remainder
        eager.sync()
        graph.sync()
        x = eager.unpack(fe)[0]
        y = graph.unpack(fg)[0]
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        # several replays interleaved with eager work stay identical
        graph.step(fg, 20)
        eager.step(fe, 20)
        eager.sync()
        graph.sync()
        assert np.array_equal(eager.unpack(fe)[0].view(np.uint32), graph.unpack(fg)[0].view(np.uint32))


def test_graph_plans_with_dz_log_match_eager():
    """A graph-enabled plan given a dz log (adaptive logging, or replay) runs eagerly: fields and
    logs equal the eager plan's bit for bit, every step's dz is logged, and replay follows the log."""
    import torch
    inst = wl.config_full(nr=48, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    kw = dict(adaptive=True, max_phase=0.05, dz_min=1e-6, dz_max=1e-2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        out = {}
        for g in (False, True):
            plan = _plan(inst, "fp64", use_graph=g, stream=stream, **kw)
            log = torch.zeros(40, dtype=torch.float64, device=plan.device)
            f = plan.pack(a0)
            plan.propagate(f, 40, dz_log=log)
            plan.sync()
            out[g] = (plan.unpack(f)[0], log.cpu().numpy())
        assert np.array_equal(out[False][0].view(np.uint64), out[True][0].view(np.uint64))
        assert np.array_equal(out[False][1], out[True][1]) and np.all(out[True][1] > 0)
        assert len(set(np.round(out[True][1], 12))) > 1
        log = torch.from_numpy(out[True][1]).to(plan.device)
        rep = {}
        for g in (False, True):
            plan = _plan(inst, "fp32_cn64", use_graph=g, stream=stream)
            f = plan.pack(a0.astype(np.complex64))
            plan.propagate(f, 40, dz_log=log, replay=True)
            plan.sync()
            rep[g] = plan.unpack(f)[0]
        assert np.array_equal(rep[False].view(np.uint32), rep[True].view(np.uint32))
        e = werr(rep[True].astype(np.complex128), out[True][0])
        say(f"  graph plan replaying the adaptive log: {e:.2e} against FP64")
        assert e < 1e-5


def test_lanes_give_the_bits_of_one_lane():
    """Instances split into 3 concurrent lanes (own streams, own step counters) give the same
    bits as one lane: eager and graph-replayed steps, adaptive dz, diagnostics records (which
    run the lanes in turn on the bound stream), and a non-finite intensity in an instance of
    another lane than the first is still reported."""
    import torch
    insts = wl.config_batch(count=7, seed=21)
    for i in insts:
        i["nr"] = min(i["nr"], 256)
    stream = torch.cuda.Stream()
    fields = [wl.gaussian_field(i, np.complex64) for i in insts]
    with torch.cuda.stream(stream):
        outs = {}
        for lanes, graph in ((1, False), (3, False), (3, True), (1, True)):
            p = _plan(insts, "fp32_cn64", lanes=lanes, use_graph=graph, stream=stream)
            f = p.pack(fields)
            p.step(f, 37)
            p.step(f, 20)
            p.sync()
            outs[(lanes, graph)] = p.unpack(f)
        for key, got in outs.items():
            for a, b in zip(outs[(1, False)], got):
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), key
        # adaptive dz without a log (lanes concurrent), then records (lanes in turn)
        res = {}
        for lanes in (1, 3):
            p = _plan(insts, "fp64", lanes=lanes, adaptive=True, stream=stream)
            f = p.pack([x.astype(np.complex128) for x in fields])
            p.step(f, 9)
            d = p.propagate(f, 6, diag_every=3)
            p.sync()
            res[lanes] = (p.unpack(f), d.cpu().numpy())
        for a, b in zip(res[1][0], res[3][0]):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert np.array_equal(res[1][1], res[3][1])
        # flags of every lane reach fcn_sync
        p = _plan(insts, "fp64", lanes=3, stream=stream)
        bad = [x.astype(np.complex128) for x in fields]
        bad[-1][2, 7] = np.nan
        f = p.pack(bad)
        p.step(f, 2)
        with pytest.raises(fcn.FcnError) as ei:
            p.sync()
        assert ei.value.code == fcn.FCN_E_NONFINITE
        p.sync()


@pytest.mark.parametrize("precision,nr,ipk", [("fp64", 40, 5e17), ("fp64", 64, 6e17), ("fp32_cn64", 64, 6e17)])
def test_step_splitting_is_exact(precision, nr, ipk):
    """step(n) then step(m) equals step(n+m) bitwise (state carried in the workspace; the fused
    row pass hands each chunk's neighbour point the density its own thread uses, so two half
    steps in one pass equal two passes bit for bit, also where the density is large)."""
    inst = wl.config_full(nr=nr, nt=256)
    a0 = wl.gaussian_field(inst) * math.sqrt(ipk / inst["I0"])
    if precision != "fp64":
        a0 = a0.astype(np.complex64)
    view = np.uint64 if precision == "fp64" else np.uint32
    p = _plan(inst, precision)
    f1 = p.pack(a0)
    p.step(f1, 7)
    p.sync()
    q = _plan(inst, precision)
    f2 = q.pack(a0)
    q.step(f2, 3)
    q.step(f2, 4)
    q.sync()
    assert np.array_equal(p.unpack(f1)[0].view(view), q.unpack(f2)[0].view(view))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32_cn64", 2e-6)])
def test_step_splitting_kerr_only_agrees_to_rounding(precision, tol):
    """Kerr-only launches apply the two nonlinear half steps of a fused row pass as one rotation
    (the rotations leave |A| unchanged), so step(n) then step(m) differs from step(n+m), where
    they are two rotations, by rounding only; and the fused run matches the oracle."""
    inst = wl.config_small(nr=64, nt=256)
    a0 = wl.gaussian_field(inst)
    if precision != "fp64":
        a0 = a0.astype(np.complex64)
    p = _plan(inst, precision)
    f1 = p.pack(a0)
    p.step(f1, 7)
    q = _plan(inst, precision)
    f2 = q.pack(a0)
    q.step(f2, 3)
    q.step(f2, 4)
    p.sync()
    q.sync()
    x, y = p.unpack(f1)[0].astype(np.complex128), q.unpack(f2)[0].astype(np.complex128)
    assert relmax(x, y) < tol
    want = oracle.propagate(inst, a0.astype(np.complex128), 7)
    assert werr(x, want) < (1e-12 if precision == "fp64" else 7e-6)


def test_nonfinite_is_reported():
    inst = wl.config_small(nr=16, nt=64)
    plan = _plan(inst, "fp64")
    a = wl.gaussian_field(inst)
    a[3, 5] = np.nan
    f = plan.pack(a)
    plan.step(f, 1)
    with pytest.raises(fcn.FcnError) as ei:
        plan.sync()
    assert ei.value.code == fcn.FCN_E_NONFINITE
    plan.sync()  # the flag is cleared once reported


def test_misaligned_field_is_rejected():
    """The step entry points move frequency pairs of the spectrum with 16-byte accesses and
    reject a field pointer that is not 16-byte aligned (here 8 bytes into an allocation)."""
    import ctypes
    import torch

    inst = wl.config_small(nr=16, nt=64)
    plan = _plan(inst, "fp32")
    f = plan.pack(wl.gaussian_field(inst, np.complex64))
    buf = torch.zeros(f.numel() + 1, dtype=f.dtype, device=f.device)
    ptr = ctypes.c_void_p(buf.data_ptr() + 8)
    for call in (lambda: plan.lib.fcn_step(plan._h, ptr, 1),
                 lambda: plan.lib.fcn_propagate(plan._h, ptr, 1, None, 0, None, 0)):
        assert call() == fcn.FCN_E_ARG
    plan.step(f, 1)  # the aligned field still steps
    plan.sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32_cn64"])
def test_density_instability_is_reported(precision):
    """A 30 fs spike above the RK4 density step's stability limit (1.99e18 W/m^2 on the
    full-model time grid) is reported as FCN_E_UNSTABLE; the same spike at 1.9e18 W/m^2 is not
    (the oracle shows the same limit on the CPU)."""
    inst = wl.config_full(nr=16, nt=2048)
    t = inst["t_min"] + np.arange(2048) * (inst["t_max"] - inst["t_min"]) / 2048
    for ipk, stable in ((1.9e18, True), (2.1e18, False)):
        a = np.zeros((16, 2048), dtype=complex)
        a[:4] = np.sqrt(ipk * np.exp(-2 * (t / 30e-15) ** 2))
        plan = _plan(inst, precision)
        f = plan.pack(a if precision == "fp64" else a.astype(np.complex64))
        plan.step(f, 1)
        if stable:
            plan.sync()
        else:
            with pytest.raises(fcn.FcnError) as ei:
                plan.sync()
            assert ei.value.code == fcn.FCN_E_UNSTABLE
            plan.sync()  # both flags are cleared once reported


def test_fp32_energy_drift_is_bounded():
    """Without absorption the step conserves the r-weighted energy exactly (FP64: 1e-16 per
    step).  In FP32 the transforms' rounding moves it by about -2e-8 per step on this smooth
    pulse; the bound 5e-8 per step guards against a regression (a biased constant or twiddle
    gave -6e-8)."""
    inst = wl.config_full(nr=256, nt=1024)
    inst["terms"] = wl.KERR_ONLY
    a0 = wl.gaussian_field(inst)
    plan = _plan(inst, "fp32")
    f = plan.pack(a0.astype(np.complex64))
    diag = plan.propagate(f, 400, diag_every=100)
    plan.sync()
    e = [plan.split_diag(diag[i])[0]["energy"] for i in range(5)]
    drift = max(abs(x / e[0] - 1) for x in e)
    say(f"  FP32 energy drift over 400 steps: {drift:.3e}")
    assert drift < 400 * 5e-8


# ------------------------------------------------- FP32 storage with FP64 arithmetic

@pytest.mark.parametrize("nt", [64, 2048, 8192])
def test_fp32_storage_stages(nt):
    """Each stage in FP32-storage mode: FP64 arithmetic on FP32-rounded input, one FP32
    rounding of the output, so the error is that of two roundings (<= 2^-23 relative to the
    largest element) whatever the transform length or solve size."""
    say(f"fp32-storage stages nt={nt}")
    nr = 37
    inst = wl.config_full(nr=nr, nt=nt)
    a = wl.random_field(nr, nt, seed=nt + 1)
    a32 = a.astype(np.complex64).astype(np.complex128)
    plan = _plan(inst, "fp32_storage")
    tol = 2.0 ** -23
    for stage, want in ((fcn.STAGE_FFT, oracle.fft_rows(a32)),
                        (fcn.STAGE_IFFT, oracle.fft_rows(a32, inverse=True)),
                        (fcn.STAGE_CN, oracle.cn_columns(inst, a32, 0.05))):
        f = plan.pack(a)
        plan.stage(stage, f, 0.05 if stage == fcn.STAGE_CN else 0.0)
        got = plan.unpack(f)[0].astype(np.complex128)
        e = relmax(got, want)
        say(f"  stage {stage}: {e:.2e}")
        assert e < tol
    plan.sync()


def test_fp32_storage_single_step_and_run():
    """One full-model step from an ionising state (two FP32 roundings, ~4e-8), then 40 steps
    of the ionising trajectory: an order of magnitude below FP32 arithmetic (measured
    2.2e-6 against 2.5e-5)."""
    inst = wl.config_full(nr=96, nt=512)
    a0 = wl.gaussian_field(inst) * math.sqrt(6e17 / inst["I0"])
    a5 = oracle.propagate(inst, a0, 5)
    a5_32 = a5.astype(np.complex64)
    got, _ = _run(inst, "fp32_storage", 1, a0=a5_32)
    e1 = werr(got.astype(np.complex128), oracle.propagate(inst, a5_32.astype(np.complex128), 1))
    a0_32 = a0.astype(np.complex64)
    got40, _ = _run(inst, "fp32_storage", 40, a0=a0_32)
    want40 = oracle.propagate(inst, a0_32.astype(np.complex128), 40)
    e40 = werr(got40.astype(np.complex128), want40)
    g32, _ = _run(inst, "fp32", 40, a0=a0_32)
    e40_32 = werr(g32.astype(np.complex128), want40)
    say(f"  fp32-storage: one step {e1:.2e}, 40 steps {e40:.2e} (FP32 arithmetic: {e40_32:.2e})")
    assert e1 < 2e-7
    assert e40 < 1e-5  # the FP32 target
    assert e40 < e40_32 / 5


def test_fp32_storage_long_run_error_vs_fp64():
    """800 steps of a Kerr pulse on a 128 x 512 grid against the FP64 GPU method: the error of
    FP32 storage grows like a random walk of the store roundings (~1e-6 here), far below the
    FP32-arithmetic error, which accumulates coherently (~5e-5)."""
    inst = wl.config_parareal_trajectory(5000, nr=128, nt=512)
    a0 = wl.gaussian_field(inst)
    ref, _ = _run(inst, "fp64", 800, a0=a0)
    got, _ = _run(inst, "fp32_storage", 800, a0=a0)
    g32, _ = _run(inst, "fp32", 800, a0=a0)
    e = werr(got.astype(np.complex128), ref)
    e32 = werr(g32.astype(np.complex128), ref)
    say(f"  800 steps vs FP64: fp32-storage {e:.2e}, fp32 {e32:.2e}")
    assert e < 5e-6
    assert e < e32 / 5


def test_fp32_storage_batch_and_graph():
    """The ragged batch and the graph replay in FP32-storage mode give the same bits as single
    instances stepped eagerly."""
    import torch
    insts = [wl.config_small(nr=40, nt=256), wl.config_small(nr=72, nt=512)]
    fields = [wl.gaussian_field(i, np.complex64) for i in insts]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = _plan(insts, "fp32_storage", use_graph=True, stream=stream)
        f = batch.pack(fields)
        batch.step(f, 37)  # 2 graph replays of 16 steps + eager remainder
        batch.sync()
        got = batch.unpack(f)
    for i, inst in enumerate(insts):
        single, _ = _run(inst, "fp32_storage", 37, a0=fields[i])
        assert np.array_equal(got[i], single)


# ------------------------------- FP32 row pass with twiddle pairs, FP64-arithmetic column solve

def _rms(a, ref):
    return float(np.sqrt(np.mean(np.abs(a - ref) ** 2) / np.mean(np.abs(ref) ** 2)))


@pytest.mark.parametrize("nt", [64, 256, 2048, 8192])
def test_fp32_cn64_stages(nt):
    """FFT and inverse FFT with twiddles as hi + lo pairs: within the FP32 arithmetic bound and,
    on the RMS over the grid, no less accurate than the plain FP32 transforms (whose rounded
    twiddles add a fixed error); the column solve is the FP32-storage kernel, bitwise."""
    say(f"fp32-cn64 stages nt={nt}")
    nr = 37
    inst = wl.config_full(nr=nr, nt=nt)
    a = wl.random_field(nr, nt, seed=nt + 2)
    a32 = a.astype(np.complex64).astype(np.complex128)
    pc = _plan(inst, "fp32_cn64")
    p32 = _plan(inst, "fp32")
    tol = 3e-7 * math.log2(nt)
    for stage, want in ((fcn.STAGE_FFT, oracle.fft_rows(a32)), (fcn.STAGE_IFFT, oracle.fft_rows(a32, inverse=True))):
        got = {}
        for name, p in (("cn64", pc), ("fp32", p32)):
            f = p.pack(a)
            p.stage(stage, f)
            got[name] = p.unpack(f)[0].astype(np.complex128)
        e = relmax(got["cn64"], want)
        r_pair, r_plain = _rms(got["cn64"], want), _rms(got["fp32"], want)
        say(f"  stage {stage}: max {e:.2e}, rms {r_pair:.2e} (plain FP32 twiddles {r_plain:.2e})")
        assert e < tol
        assert r_pair <= r_plain * 1.05
    ps = _plan(inst, "fp32_storage")
    f, g = pc.pack(a), ps.pack(a)
    pc.stage(fcn.STAGE_CN, f, 0.05)
    ps.stage(fcn.STAGE_CN, g, 0.05)
    got_c, got_s = pc.unpack(f)[0], ps.unpack(g)[0]
    assert np.array_equal(got_c, got_s)
    assert relmax(got_c.astype(np.complex128), oracle.cn_columns(inst, a32, 0.05)) < 2.0 ** -23
    pc.sync()


def test_fp32_cn64_run_errors_vs_fp64():
    """Full-model pulse on a 128 x 512 grid, 300 steps, and the Kerr trajectory of the FP32-
    storage test, 800 steps, against the FP64 GPU method: FP32-CN64 sits between FP32 and
    FP32 storage, well below FP32."""
    cases = ((wl.config_full(nr=128, nt=512), 300), (wl.config_parareal_trajectory(5000, nr=128, nt=512), 800))
    for inst, n in cases:
        a0 = wl.gaussian_field(inst)
        ref, _ = _run(inst, "fp64", n, a0=a0)
        e = {}
        for mode in ("fp32", "fp32_cn64", "fp32_storage"):
            got, _ = _run(inst, mode, n, a0=a0.astype(np.complex64))
            e[mode] = werr(got.astype(np.complex128), ref)
        say(f"  {inst['nr']}x{inst['nt']}, {n} steps vs FP64: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
        assert e["fp32_cn64"] < e["fp32"] / 2
        assert e["fp32_storage"] < e["fp32_cn64"]
        assert e["fp32_cn64"] < 1e-5  # the FP32 target, over the whole run


def test_fp32_cn64_batch_and_graph():
    """The ragged batch and the graph replay in FP32-CN64 mode give the same bits as single
    instances stepped eagerly (instances with and without a density term)."""
    import torch
    insts = [wl.config_small(nr=40, nt=256), wl.config_full(nr=72, nt=512)]
    fields = [wl.gaussian_field(i, np.complex64) for i in insts]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = _plan(insts, "fp32_cn64", use_graph=True, stream=stream)
        f = batch.pack(fields)
        batch.step(f, 37)  # 2 graph replays of 16 steps + eager remainder
        batch.sync()
        got = batch.unpack(f)
    for i, inst in enumerate(insts):
        single, _ = _run(inst, "fp32_cn64", 37, a0=fields[i])
        assert np.array_equal(got[i], single)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 10 * 1e-6)])
def test_paper_grid_nr_2112(precision, tol):
    """The radial size of the paper's timing example (Nr = 2112, Table 2): tall columns solved
    with 2 (FP32) or 1 (FP64) frequencies per workgroup, 10 full-model steps against the oracle."""
    inst = wl.config_full(nr=2112, nt=128)
    a0 = wl.gaussian_field(inst) * math.sqrt(5e17 / inst["I0"])
    got, plan = _run(inst, precision, 10, a0=a0 if precision == "fp64" else a0.astype(np.complex64))
    want = oracle.propagate(inst, a0 if precision == "fp64" else a0.astype(np.complex64).astype(np.complex128), 10)
    e = werr(got.astype(np.complex128), want)
    say(f"  2112 x 128 {precision} tiles {plan.tiles()}: {e:.3e}")
    assert e < tol

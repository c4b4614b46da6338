"""Seeded synthetic inputs for the FCN z-step: instance parameters and initial fields.

This module is shared by the tests, the benchmark and the CPU oracle's callers.  It
holds input recipes only: the physical parameters of each workload, the Gaussian
initial pulse (Sec. 5, Eq. gauss) and the seeded draws of the batched sweep.  It
holds none of the solver's arithmetic (no transforms, no Crank-Nicholson matrices,
no nonlinear operator) and it imports nothing from the HIP binding or the oracle.

Units are SI throughout.  A workload is a list of instance dicts whose keys match
the ``fcn_instance`` struct of ``include/fcn.h``:
``nr, nt, r_max, t_min, t_max, lambda0, n0, k2, n2, n4, n6, n8, K, sigma_K, rho_at,
sigma_c, U_i, dz, terms`` plus the pulse keys ``w0, tau, P, I0, chirp`` that only the
initial field uses.
"""
from __future__ import annotations

import math

import numpy as np

# Term switches (same bit values as the FCN_* enum in include/fcn.h).
DIFFRACTION = 1  # transverse Laplacian of the linear operator (Eq. linearpart)
GVD = 2          # group-velocity dispersion of the linear operator (Eq. linearpart)
KERR = 4         # sum_j n_{2j} |A|^{2j} of Eq. nonlinearpart
PLASMA = 8       # plasma defocusing term of Eq. nonlinearpart
MPA = 16         # multiphoton absorption term of Eq. nonlinearpart
COLL = 32        # collisional absorption, -(sigma_c/2) rho (not in the paper)
AVALANCHE = 64   # avalanche ionisation, (sigma_c / U_i) I rho in the density rate (not in the paper)
ALL_TERMS = DIFFRACTION | GVD | KERR | PLASMA | MPA | COLL
KERR_ONLY = DIFFRACTION | GVD | KERR

FS = 1e-15
MM = 1e-3
LAMBDA0 = 800e-9
K2_AIR = 2e-29            # k'' [s^2/m] = 0.2 fs^2/cm (Sec. 2, after Eq. nlse)
# Collisional cross-section from the Drude model with tau_c = 350 fs at 800 nm,
# sigma_c = k0 w0 tau_c / (n0 rho_c (1 + w0^2 tau_c^2)); evaluated once with CODATA
# constants and stored as a plain input coefficient.
SIGMA_C_800NM = 5.471072962824351e-24
# Ionisation potential of O2, 12.06 eV, for the avalanche rate (sigma_c / U_i) I rho.
U_I_O2 = 12.06 * 1.602176634e-19


def critical_power(lambda0: float, n0: float, n2: float) -> float:
    """Critical self-focusing power Pcr = 3.77 lambda0^2 / (8 pi n0 n2) (Sec. 2, after Eq. kerrsource)."""
    return 3.77 * lambda0 ** 2 / (8.0 * math.pi * n0 * n2)


def peak_intensity(power: float, w0: float) -> float:
    """I0 such that the pulse peak carries ``power``: |A|^2 = I0 exp(-2 r^2/w0^2) integrates to I0 pi w0^2/2."""
    return 2.0 * power / (math.pi * w0 ** 2)


def rayleigh_range(w0: float, lambda0: float, n0: float = 1.0) -> float:
    return math.pi * n0 * w0 ** 2 / lambda0


def marburger_distance(w0: float, lambda0: float, p_over_pcr: float) -> float:
    """Marburger's empirical collapse distance; inf when P is at or below the threshold."""
    x = (math.sqrt(p_over_pcr) - 0.852) ** 2 - 0.0219
    if p_over_pcr <= 1.0 or x <= 0.0:
        return math.inf
    return 0.367 * rayleigh_range(w0, lambda0) / math.sqrt(x)


def gaussian_field(inst: dict, dtype=np.complex128) -> np.ndarray:
    """Initial pulse A(r,0,t) = sqrt(I0) exp(-r^2/r0^2 - t^2/tp^2 - i C t^2/tp^2) (Sec. 5, Eq. gauss).

    Grid: r_m = m r_max/(nr-1) for 0 <= m < nr and t_p = t_min + p (t_max - t_min)/nt for
    0 <= p < nt (periodic window, right end excluded).  The row at r_max is set to zero,
    the Dirichlet condition of Eq. bound.  Layout ``[nr][nt]``, t contiguous.
    """
    nr, nt = int(inst["nr"]), int(inst["nt"])
    r = np.arange(nr, dtype=np.float64) * (inst["r_max"] / (nr - 1))
    t = inst["t_min"] + np.arange(nt, dtype=np.float64) * ((inst["t_max"] - inst["t_min"]) / nt)
    w0, tau, chirp = inst["w0"], inst["tau"], inst.get("chirp", 0.0)
    amp = math.sqrt(inst["I0"])
    radial = np.exp(-(r / w0) ** 2)
    temporal = np.exp(-(t / tau) ** 2 - 1j * chirp * (t / tau) ** 2)
    a = amp * radial[:, None] * temporal[None, :]
    a[nr - 1, :] = 0.0
    return a.astype(dtype)


def _pulse(inst: dict, w0: float, tau: float, p_over_pcr: float) -> dict:
    pcr = critical_power(inst["lambda0"], inst["n0"], inst["n2"])
    out = dict(inst)
    out.update(w0=w0, tau=tau, P=p_over_pcr * pcr, I0=peak_intensity(p_over_pcr * pcr, w0),
               chirp=0.0, p_over_pcr=p_over_pcr)
    return out


def _base(nr, nt, w0, tau, *, r_max=None, t_half=None, n2=0.0, n4=0.0, k2=K2_AIR,
          K=8, sigma_K=0.0, rho_at=0.0, sigma_c=0.0, U_i=0.0, dz=0.0, terms=KERR_ONLY):
    r_max = 4.0 * w0 if r_max is None else r_max
    t_half = 4.0 * tau if t_half is None else t_half
    return dict(nr=nr, nt=nt, r_max=r_max, t_min=-t_half, t_max=t_half, lambda0=LAMBDA0, n0=1.0,
                k2=k2, n2=n2, n4=n4, n6=0.0, n8=0.0, K=K, sigma_K=sigma_K, rho_at=rho_at,
                sigma_c=sigma_c, U_i=U_i, dz=dz, terms=terms)


# Full-model coefficient set: Kerr n2 and the alternating-sign n4, 8-photon ionisation
# of O2 with sigma_K given in cm^2 units and converted to SI (2.9e-99 s^-1 cm^16 W^-8),
# neutral density 5.4e24 m^-3 and collisional absorption.
FULL_PHYSICS = dict(n2=1e-23, n4=-3.6e-42, K=8, sigma_K=2.9e-99 * (1e-4) ** 8, rho_at=5.4e24,
                    sigma_c=SIGMA_C_800NM, terms=ALL_TERMS)


def config_small(nr=128, nt=256) -> dict:
    """Plain Kerr case: Nr=128 over [0,4 w0], Nt=256 over [-4 tau, 4 tau), w0=1 mm, tau=50 fs,
    P=3 Pcr, n2=3.2e-23 m^2/W, k''=2e-29 s^2/m, dz=1 cm (100 steps)."""
    inst = _base(nr, nt, 1 * MM, 50 * FS, n2=3.2e-23, dz=1e-2, terms=KERR_ONLY)
    return _pulse(inst, 1 * MM, 50 * FS, 3.0)


SMALL_STEPS = 100


def config_full(nr=512, nt=2048) -> dict:
    """Full model: Nr=512 over [0,4 w0], Nt=2048 over [-4 tau, 4 tau), w0=2 mm, tau=100 fs,
    P=5 Pcr, n2+n4, K=8 ionisation, plasma, MPA and collisional absorption; dz=5 mm (2000 steps)."""
    inst = _base(nr, nt, 2 * MM, 100 * FS, dz=5e-3, **FULL_PHYSICS)
    return _pulse(inst, 2 * MM, 100 * FS, 5.0)


FULL_STEPS = 2000


def config_batch(count=64, seed=3) -> list[dict]:
    """Batched sweep of ``count`` Kerr-only pulses of uneven grids.

    Draws, in order per instance from ``default_rng(seed)``: Nr in {256,512,1024}, Nt in
    {512,1024,2048,4096}, P/Pcr ~ U[1,10], tau ~ U[30,200] fs; w0 ~ U[0.5,3] mm from
    ``default_rng(1000 + i)``.  Windows are [0, 4 w0] and [-4 tau, 4 tau).  Each instance
    steps with dz_i = min(1 cm, z_c,i / 200), z_c being Marburger's collapse distance.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nr = int(rng.choice([256, 512, 1024]))
        nt = int(rng.choice([512, 1024, 2048, 4096]))
        p = float(rng.uniform(1.0, 10.0))
        tau = float(rng.uniform(30.0, 200.0)) * FS
        w0 = float(np.random.default_rng(1000 + i).uniform(0.5, 3.0)) * MM
        zc = marburger_distance(w0, LAMBDA0, p)
        dz = min(1e-2, 0.5 * zc / 100.0)
        inst = _base(nr, nt, w0, tau, n2=3.2e-23, dz=dz, terms=KERR_ONLY)
        out.append(_pulse(inst, w0, tau, p))
    return out


BATCH_STEPS = 100


def config_long(nr=1024, nt=8192) -> dict:
    """Long single pulse: Nr=1024 over [0, 20 mm], Nt=8192 over [-200, 200) fs, w0=5 mm,
    tau=50 fs, P=8 Pcr with the full-model coefficient set; adaptive dz (0.05 rad)."""
    inst = _base(nr, nt, 5 * MM, 50 * FS, r_max=20 * MM, dz=1e-2, **FULL_PHYSICS)
    return _pulse(inst, 5 * MM, 50 * FS, 8.0)


LONG_MAX_PHASE = 0.05
LONG_DZ_MIN = 1e-6
LONG_DZ_MAX = 1e-2


def config_parareal_trajectory(j: int, nr=512, nt=2048) -> dict:
    """Trajectory j of the learned-coarse workload: Kerr only, Nr=512 over [0, 4 mm],
    Nt=2048 over [-600, 600) fs, w0=1 mm, dz=0.2 mm, P/Pcr ~ U[2,8] and tau ~ U[50,150] fs
    drawn from ``default_rng(5000 + j)``."""
    rng = np.random.default_rng(5000 + j)
    p = float(rng.uniform(2.0, 8.0))
    tau = float(rng.uniform(50.0, 150.0)) * FS
    inst = _base(nr, nt, 1 * MM, tau, r_max=4 * MM, t_half=600 * FS, n2=3.2e-23, dz=2e-4,
                 terms=KERR_ONLY)
    return _pulse(inst, 1 * MM, tau, p)


PARAREAL_WINDOWS = 32
PARAREAL_STEPS_PER_WINDOW = 50
# Learned-coarse variant of the same trajectories: 8 windows of 250 steps (5 cm, 0.4 m in
# all).  Over 1 cm windows the classical coarse step is within 5e-8..3e-7 of the fine steps
# (FP64), below FP32 field resolution, so a learned correction has nothing to learn there;
# over 5 cm its error is 1e-6..1e-3 per window.
LEARNED_WINDOWS = 8
LEARNED_STEPS_PER_WINDOW = 250


def config_higher_kerr(nr=256, nt=1024, chirp=-1.5) -> dict:
    """Full-model pulse with the whole Kerr sum of Eq. nlse (n2, n4, n6, n8 of alternating sign)
    and a chirped input (Sec. 5, Eq. gauss, C != 0): the full-model grid and coefficients, plus
    synthetic n6 = 4e-60 m^6/W^3 and n8 = -2e-77 m^8/W^4 (the paper gives no values; these make
    every order turn the phase appreciably near 5e17 W/m^2), scaled to 5e17 W/m^2 peak."""
    inst = config_full(nr=nr, nt=nt)
    inst.update(n6=4e-60, n8=-2e-77, chirp=chirp)
    inst["I0"] = 5e17
    return inst


def config_avalanche(nr=256, nt=1024, peak=7e17) -> dict:
    """Full-model pulse with avalanche ionisation added to the density rate: the full-model grid
    and coefficients, U_i of O2, scaled to `peak` W/m^2 (where the avalanche rate sigma_c I / U_i,
    about 2e12 1/s, turns a few percent of the pulse's density over its length)."""
    inst = config_full(nr=nr, nt=nt)
    inst.update(U_i=U_I_O2, terms=ALL_TERMS | AVALANCHE)
    inst["I0"] = peak
    return inst


def config_paper_timing(nr=2112, nt=2048) -> dict:
    """The grid of the paper's timing example (Sec. 5.1, Table 2: Nr = 2112, Nt = 2048, 1000
    steps); the paper gives no physics or ranges for it, so the full-model pulse's are used
    (r in [0, 8 mm], t in [-400, 400) fs, w0 = 2 mm, tau = 100 fs, 5 Pcr, dz = 5 mm)."""
    return config_full(nr=nr, nt=nt)


def config_paper_application(nr=1350, nt=1024) -> dict:
    """The paper's 1.1 km run (Sec. 5.2): I0 = 3.14e14 W/m^2, r0 = 18 mm, tau0 = 300 fs, C = 0,
    Nr = 1350, Nt = 1024, 1.1e6 steps (dz = 1 mm).  Unstated and read here: r in [0, 4 r0],
    t in [-4 tau0, 4 tau0), the full-model coefficient set."""
    inst = _base(nr, nt, 18 * MM, 300 * FS, dz=1e-3, **FULL_PHYSICS)
    pcr = critical_power(inst["lambda0"], inst["n0"], inst["n2"])
    power = 3.14e14 * math.pi * (18 * MM) ** 2 / 2.0  # I0 = 2P / (pi r0^2)
    return _pulse(inst, 18 * MM, 300 * FS, power / pcr)


def config_cartesian(nx=255, ny=255, nt=256, p_over_pcr=30.0) -> dict:
    """Cartesian 3D+1 pulse (Delta_perp = d2/dx2 + d2/dy2, Sec. 2): an elliptic Gaussian beam,
    w_x = 3 mm, w_y = 2 mm, tau = 50 fs, `p_over_pcr` critical powers (I0 = 2P / (pi w_x w_y)),
    on x, y in [-12, 12] mm (nx, ny points; odd counts put x = y = 0 on a grid point) and
    t in [-200, 200) fs, the full-model coefficients, dz = 1 cm.  With the seeded transverse
    noise of ``cartesian_field`` the beam breaks up into several filaments (the regime that needs
    the Cartesian form)."""
    wx, wy, tau = 3 * MM, 2 * MM, 50 * FS
    inst = _base(3, nt, wx, tau, dz=1e-2, **FULL_PHYSICS)
    del inst["nr"], inst["r_max"]
    pcr = critical_power(inst["lambda0"], inst["n0"], inst["n2"])
    inst.update(geometry="cartesian", nx=nx, ny=ny, x_max=12 * MM, y_max=12 * MM, wx=wx, wy=wy, tau=tau,
                P=p_over_pcr * pcr, I0=2.0 * p_over_pcr * pcr / (math.pi * wx * wy), p_over_pcr=p_over_pcr,
                chirp=0.0, noise=0.05, noise_seed=11)
    return inst


def cartesian_field(inst: dict, dtype=np.complex128) -> np.ndarray:
    """Initial Cartesian pulse [ny][nx][nt]: sqrt(I0) exp(-x^2/wx^2 - y^2/wy^2 - t^2/tau^2)
    times (1 + noise eta(x, y)), eta a seeded real Gaussian field smoothed over about 0.3 mm
    (unit standard deviation); grid x_i = -x_max + i 2 x_max/(nx-1), y likewise,
    t_p = t_min + p (t_max - t_min)/nt; the four walls are zero (A = 0 there)."""
    nx, ny, nt = int(inst["nx"]), int(inst["ny"]), int(inst["nt"])
    x = -inst["x_max"] + np.arange(nx) * (2.0 * inst["x_max"] / (nx - 1))
    y = -inst["y_max"] + np.arange(ny) * (2.0 * inst["y_max"] / (ny - 1))
    t = inst["t_min"] + np.arange(nt, dtype=np.float64) * ((inst["t_max"] - inst["t_min"]) / nt)
    env = np.exp(-(y[:, None] / inst["wy"]) ** 2 - (x[None, :] / inst["wx"]) ** 2)
    if inst.get("noise", 0.0) > 0.0:
        rng = np.random.default_rng(int(inst.get("noise_seed", 0)))
        white = rng.standard_normal((ny, nx))
        kx = np.fft.fftfreq(nx, d=x[1] - x[0])
        ky = np.fft.fftfreq(ny, d=y[1] - y[0])
        corr = 0.3 * MM
        filt = np.exp(-((kx[None, :] ** 2 + ky[:, None] ** 2) * (math.pi * corr) ** 2))
        eta = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
        eta /= np.std(eta)
        env = env * (1.0 + inst["noise"] * eta)
    temporal = np.exp(-(t / inst["tau"]) ** 2 - 1j * inst.get("chirp", 0.0) * (t / inst["tau"]) ** 2)
    a = math.sqrt(inst["I0"]) * env[:, :, None] * temporal[None, None, :]
    a[0], a[-1] = 0.0, 0.0
    a[:, 0], a[:, -1] = 0.0, 0.0
    return a.astype(dtype)


def random_field(nr: int, nt: int, seed: int, scale: float = 1.0, dtype=np.complex128) -> np.ndarray:
    """Seeded complex normal field (stage tests on random spectra); last row zero."""
    rng = np.random.default_rng(seed)
    a = scale * (rng.standard_normal((nr, nt)) + 1j * rng.standard_normal((nr, nt)))
    a[nr - 1, :] = 0.0
    return a.astype(dtype)


def points(insts) -> int:
    if isinstance(insts, dict):
        insts = [insts]
    return int(sum((int(i["nx"]) * int(i["ny"]) if i.get("geometry") == "cartesian" else int(i["nr"])) * int(i["nt"])
                   for i in insts))

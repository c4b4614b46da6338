"""Dense brute-force forms of the FCN step for tiny grids -- TEST INFRASTRUCTURE ONLY.

These are deliberately different constructions of the same mathematics, used to pin
the C oracle:
  * the DFT as an explicit O(N^2) matrix;
  * the Crank-Nicholson matrices assembled from the discrete operator itself
    (Eqs. diff1-diff3 with the boundary conditions of Eq. bound), i.e. M_abc = I - dz/2 L
    and M_def = I + dz/2 L, instead of from the printed coefficient list, and solved by
    dense LU (numpy.linalg.solve);
  * the nonlinear half step with a direct RK4 loop (Eqs. ionization, nonlinearpart).
Nothing here is used by the HIP path.
"""
from __future__ import annotations

import math

import numpy as np

C = 299792458.0
HBAR = 1.054571817e-34
ME = 9.1093837015e-31
QE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def constants(inst):
    k0 = 2 * math.pi * inst["n0"] / inst["lambda0"]
    w0 = 2 * math.pi * C / inst["lambda0"]
    rho_c = EPS0 * ME * w0 ** 2 / QE ** 2
    beta = inst["K"] * HBAR * w0 * inst["sigma_K"] * inst["rho_at"]
    return k0, w0, rho_c, beta


def dft_matrix(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def radial_laplacian(nr: int, dr: float) -> np.ndarray:
    """Discrete d2/dr2 + (1/r) d/dr on rows 0..nr-2; row nr-1 (r = r_max, A = 0) is zero.

    Row m >= 1: centred second difference plus the centred first difference over r_m.
    Row 0: the axis limit 2 d2A/dr2 with the mirror value A_{-1} = A_1 (dA/dr = 0)."""
    L = np.zeros((nr, nr))
    L[0, 0] = -4.0 / dr ** 2
    L[0, 1] = 4.0 / dr ** 2
    for m in range(1, nr - 1):
        r = m * dr
        L[m, m - 1] = 1.0 / dr ** 2 - 1.0 / (2.0 * dr * r)
        L[m, m] = -2.0 / dr ** 2
        L[m, m + 1] = 1.0 / dr ** 2 + 1.0 / (2.0 * dr * r)
    return L


def omegas(nt: int, dtau: float) -> np.ndarray:
    q = np.where(np.arange(nt) < nt // 2, np.arange(nt), np.arange(nt) - nt)
    return 2 * np.pi * q / (nt * dtau)


def cn_dense(inst, dz: float, omega: float, terms=None):
    terms = inst["terms"] if terms is None else terms
    nr = int(inst["nr"])
    k0 = constants(inst)[0]
    dr = inst["r_max"] / (nr - 1)
    lin = np.zeros((nr, nr), dtype=np.complex128)
    if terms & 1:
        lin += 1j / (2 * k0) * radial_laplacian(nr, dr)
    if terms & 2:
        lin += np.diag(np.full(nr, 1j * inst["k2"] * omega ** 2 / 2))
    ident = np.eye(nr, dtype=np.complex128)
    m_abc = ident - dz / 2 * lin
    m_def = ident + dz / 2 * lin
    m_abc[nr - 1, :] = 0.0
    m_abc[nr - 1, nr - 1] = 1.0
    m_def[nr - 1, :] = 0.0
    return m_abc, m_def


def linear_dense(inst, a: np.ndarray, dz: float, terms=None) -> np.ndarray:
    nr, nt = a.shape
    dtau = (inst["t_max"] - inst["t_min"]) / nt
    F = dft_matrix(nt)
    spec = a @ F.T
    w = omegas(nt, dtau)
    out = np.empty_like(spec)
    for p in range(nt):
        m_abc, m_def = cn_dense(inst, dz, w[p], terms)
        out[:, p] = np.linalg.solve(m_abc, m_def @ spec[:, p])
    return (out @ np.conj(F).T) / nt


def rho_rk4(inst, inten_row: np.ndarray) -> np.ndarray:
    k0, w0, rho_c, beta = constants(inst)
    K = int(inst["K"])
    rho_at = inst["rho_at"]
    nt = inten_row.shape[0]
    h = (inst["t_max"] - inst["t_min"]) / nt
    rho = np.zeros(nt)
    if rho_at <= 0:
        return rho

    aval = inst["sigma_c"] / inst["U_i"] if inst["terms"] & 64 else 0.0

    def f(i, r):
        return beta / (K * HBAR * w0) * i ** K * (1 - r / rho_at) + aval * i * r

    for q in range(nt - 1):
        i0, i1 = inten_row[q], inten_row[q + 1]
        ih = 0.5 * (i0 + i1)
        r = rho[q]
        k1 = f(i0, r)
        k2 = f(ih, r + h / 2 * k1)
        k3 = f(ih, r + h / 2 * k2)
        k4 = f(i1, r + h * k3)
        rho[q + 1] = r + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return rho


def nl_half_dense(inst, a: np.ndarray, hz: float, terms=None) -> np.ndarray:
    terms = inst["terms"] if terms is None else terms
    k0, w0, rho_c, beta = constants(inst)
    K = int(inst["K"])
    out = a.copy()
    for m in range(a.shape[0]):
        inten = np.abs(a[m]) ** 2
        rho = rho_rk4(inst, inten) if terms & (8 | 32) else np.zeros_like(inten)
        nhat = np.zeros(inten.shape, dtype=np.complex128)
        if terms & 4:
            nhat += 1j * k0 / inst["n0"] * (inst["n2"] * inten + inst["n4"] * inten ** 2
                                             + inst["n6"] * inten ** 3 + inst["n8"] * inten ** 4)
        if terms & 8:
            nhat += -1j * k0 / 2 * rho / rho_c
        if terms & 16:
            nhat += -beta / 2 * inten ** (K - 1)
        if terms & 32:
            nhat += -inst["sigma_c"] / 2 * rho
        out[m] = a[m] * np.exp(hz * nhat)
    return out


def step_dense(inst, a: np.ndarray, dz: float, terms=None) -> np.ndarray:
    a = nl_half_dense(inst, a, dz / 2, terms)
    a = linear_dense(inst, a, dz, terms)
    return nl_half_dense(inst, a, dz / 2, terms)


def weighted_norm(a: np.ndarray) -> float:
    """sum_p [ |A_0p|^2 / 8 + sum_{m=1}^{nr-2} m |A_mp|^2 ]: the norm the CN step conserves."""
    nr = a.shape[0]
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[nr - 1] = 0.0
    return float(np.sum(w[:, None] * np.abs(a) ** 2))

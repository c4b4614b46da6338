"""CPU FP64 oracle of the FCN z-step on a Cartesian transverse grid -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this module.  It shares no code with the HIP path.

A Cartesian instance is a dict with the keys of a radial one (see ``oracle.params``) except
that the transverse grid is ``nx`` points over [-x_max, x_max] and ``ny`` points over
[-y_max, y_max]; the field is complex [ny][nx][nt].  One z-step follows Sec. 3 of the paper in
its order: nonlinear half step, forward transform of every row along t, Crank-Nicholson along
x then along y for every frequency (``fcn_cartesian.c``; the reading is in its header), inverse
transform, nonlinear half step.  The transforms and the nonlinear half steps are the radial
oracle's routines applied to the nx * ny rows (they do not depend on the geometry).

Parity status: the axis solves are pinned by the exact eigenvalues of the Dirichlet second
difference (sine modes), unitarity, the astigmatic Gaussian beam's closed form at second order,
and a dense brute force on tiny grids (tests/test_oracle_cartesian.py).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

import oracle as _radial

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcn_cartesian.c")
_LIB = os.path.join(_HERE, "_build", "liborc_cart.so")


class CartParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nt", ctypes.c_int32),
        ("x_max", ctypes.c_double), ("y_max", ctypes.c_double),
        ("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
        ("lambda0", ctypes.c_double), ("n0", ctypes.c_double), ("k2", ctypes.c_double),
        ("terms", ctypes.c_uint32),
    ]


def _compile(src: str, out: str):
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                           "-fno-fast-math", "-ffp-contract=off", "-o", out, src, "-lm"])


def build(force: bool = False) -> str:
    """Compile fcn_cartesian.c with gcc (-O2, OpenMP, no fast-math) into oracle/_build/."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        _compile(_SRC, tmp)
        os.replace(tmp, _LIB)
    return _LIB


def _load(path: str):
    h = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    cp = ctypes.POINTER(CartParams)
    h.orc_cart_matrices.argtypes = [cp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
    h.orc_cart_cn_axis.argtypes = [cp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    h.orc_cart_matrices.restype = ctypes.c_int
    h.orc_cart_cn_axis.restype = ctypes.c_int
    return h


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


class use_library:
    """Context manager: route the axis solves through another build of fcn_cartesian.c (the
    mutation tests compile copies with a planted mistake)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_variant(source_text: str, out_path: str) -> str:
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    _compile(src, out_path)
    return out_path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def params(inst: dict, terms: int | None = None) -> CartParams:
    p = CartParams()
    p.nx, p.ny, p.nt = int(inst["nx"]), int(inst["ny"]), int(inst["nt"])
    for k in ("x_max", "y_max", "t_min", "t_max", "lambda0", "n0", "k2"):
        setattr(p, k, float(inst[k]))
    p.terms = int(inst["terms"] if terms is None else terms)
    return p


def row_view(inst: dict) -> dict:
    """The radial-oracle instance whose nr rows are the nx * ny transverse points (for the
    transforms and the nonlinear half steps, which do not depend on the geometry)."""
    r = dict(inst)
    r["nr"] = int(inst["nx"]) * int(inst["ny"])
    r["r_max"] = float(inst["x_max"])
    return r


def spacing(inst: dict):
    return 2.0 * inst["x_max"] / (inst["nx"] - 1), 2.0 * inst["y_max"] / (inst["ny"] - 1)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _threads(threads):
    return threads or _radial.default_threads()


def _rows(inst, a):
    return np.ascontiguousarray(a, dtype=np.complex128).reshape(int(inst["ny"]) * int(inst["nx"]), int(inst["nt"]))


def _shape(inst, a):
    return a.reshape(int(inst["ny"]), int(inst["nx"]), int(inst["nt"]))


def axis_matrices(inst: dict, axis: int, dz: float, p: int, terms=None):
    """(a, b, c, d, e, f) of the Crank-Nicholson matrices of axis 0 (x) or 1 (y), column p."""
    n = int(inst["nx"] if axis == 0 else inst["ny"])
    buf = np.zeros(6 * n, dtype=np.complex128)
    pr = params(inst, terms)
    if lib().orc_cart_matrices(ctypes.byref(pr), int(axis), float(dz), int(p), _dptr(buf)) != 0:
        raise ValueError("oracle cartesian matrices rejected its arguments")
    return tuple(buf[k * n:(k + 1) * n].copy() for k in range(6))


def cn_axis(inst: dict, spectrum: np.ndarray, dz: float, axis: int, threads=None, terms=None) -> np.ndarray:
    """One axis (0: x, 1: y) of the linear part on a spectrum [ny][nx][nt]."""
    out = np.ascontiguousarray(spectrum, dtype=np.complex128).copy()
    pr = params(inst, terms)
    if lib().orc_cart_cn_axis(ctypes.byref(pr), _dptr(out), float(dz), int(axis), _threads(threads)) != 0:
        raise ValueError("oracle cartesian cn rejected its arguments")
    return out


def linear_part(inst: dict, a: np.ndarray, dz: float, threads=None, terms=None) -> np.ndarray:
    """Forward transform of every row, Crank-Nicholson along x then y, inverse transform."""
    spec = _radial.fft_rows(_rows(inst, a), inverse=False, threads=threads)
    spec = cn_axis(inst, _shape(inst, spec), dz, 0, threads, terms)
    spec = cn_axis(inst, spec, dz, 1, threads, terms)
    return _shape(inst, _radial.fft_rows(_rows(inst, spec), inverse=True, threads=threads))


def nl_half(inst: dict, a: np.ndarray, hz: float, threads=None, terms=None) -> np.ndarray:
    out = _radial.nl_half(row_view(inst), _rows(inst, a), hz, threads=threads, terms=terms)
    return _shape(inst, out)


def step(inst: dict, a: np.ndarray, dz: float | None = None, threads=None, terms=None) -> np.ndarray:
    dz = float(inst["dz"] if dz is None else dz)
    a = nl_half(inst, a, 0.5 * dz, threads, terms)
    a = linear_part(inst, a, dz, threads, terms)
    return nl_half(inst, a, 0.5 * dz, threads, terms)


def propagate(inst: dict, a: np.ndarray, nsteps: int, dz=None, threads=None, terms=None) -> np.ndarray:
    dzs = np.broadcast_to(np.asarray(inst["dz"] if dz is None else dz, dtype=np.float64), (nsteps,))
    out = np.ascontiguousarray(a, dtype=np.complex128).reshape(int(inst["ny"]), int(inst["nx"]), int(inst["nt"]))
    for n in range(nsteps):
        out = step(inst, out, float(dzs[n]), threads, terms)
    return out


def axis_row(inst: dict) -> int:
    """Row index of the transverse point ((nx-1)/2, (ny-1)/2): x = y = 0 for odd nx, ny."""
    return (int(inst["ny"]) - 1) // 2 * int(inst["nx"]) + (int(inst["nx"]) - 1) // 2


def diagnostics(inst: dict, a: np.ndarray, threads=None, terms=None) -> dict:
    """energy dx dy dtau sum |A|^2; peak and on-axis (axis_row) intensity; peak density and
    phase rate (the radial oracle's per-row routine on the nx * ny rows); fluence per row."""
    rows = _rows(inst, a)
    d = _radial.diagnostics(row_view(inst), rows, threads=threads, terms=terms)
    dx, dy = spacing(inst)
    d["energy"] = dx * dy * float(np.sum(d["fluence"]))
    d["i_axis"] = float(np.max(np.abs(rows[axis_row(inst)]) ** 2))
    return d


def propagate_adaptive(inst: dict, a: np.ndarray, nsteps: int, max_phase: float, dz_min: float, dz_max: float,
                       threads=None, terms=None):
    """Adaptive steps with the radial oracle's rule: dz_n = clamp(max_phase / Phi, dz_min, dz_max)
    with Phi measured on A^{n-1} (A^0 for the first step)."""
    out = np.ascontiguousarray(a, dtype=np.complex128).reshape(int(inst["ny"]), int(inst["nx"]), int(inst["nt"]))
    log = np.zeros(nsteps)
    phi_prev = 0.0
    for n in range(nsteps):
        phi_now = diagnostics(inst, out, threads, terms)["phi"]
        phi = phi_now if n == 0 else phi_prev
        dz = dz_max if phi <= 0.0 else min(max(max_phase / phi, dz_min), dz_max)
        log[n] = dz
        out = step(inst, out, dz, threads, terms)
        phi_prev = phi_now
    return out, log


def gaussian_beam(inst: dict, z: float, wx: float, wy: float, amp: float = 1.0) -> np.ndarray:
    """Linear diffraction of an astigmatic Gaussian beam (no GVD, time-independent envelope):
    the product over the two axes of (1 + i z / z_u)^(-1/2) exp(-u^2 / (w_u^2 (1 + i z / z_u))),
    z_u = k0 w_u^2 / 2 (the textbook paraxial solution), on the grid of ``inst`` [ny][nx]."""
    k0 = 2.0 * math.pi * inst["n0"] / inst["lambda0"]
    x = np.linspace(-inst["x_max"], inst["x_max"], int(inst["nx"]))
    y = np.linspace(-inst["y_max"], inst["y_max"], int(inst["ny"]))

    def axis(u, w):
        q = 1.0 + 1j * z / (k0 * w * w / 2.0)
        return q ** -0.5 * np.exp(-u * u / (w * w * q))

    return amp * axis(y, wy)[:, None] * axis(x, wx)[None, :]

"""CPU FP64 oracle of the FCN z-step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path and never
imports it.  ``fcn_oracle.c`` holds the arithmetic (see its header for the paper
passages each routine follows); ``brute.py`` holds dense numpy brute-force checks
for tiny grids.

Parity status: every routine is pinned by the closed forms, invariants and brute-force
checks in ``tests/test_oracle_*.py``.  The full-physics trajectory after collapse has no
independent pin ("parity unpinned" for that regime); there the piecewise-pinned
oracle is the only judge.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcn_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liborc.so")

DIFFRACTION, GVD, KERR, PLASMA, MPA, COLL, AVALANCHE = 1, 2, 4, 8, 16, 32, 64


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32), ("nt", ctypes.c_int32),
        ("r_max", ctypes.c_double), ("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
        ("lambda0", ctypes.c_double), ("n0", ctypes.c_double), ("k2", ctypes.c_double),
        ("n2", ctypes.c_double), ("n4", ctypes.c_double), ("n6", ctypes.c_double), ("n8", ctypes.c_double),
        ("K", ctypes.c_int32),
        ("sigma_K", ctypes.c_double), ("rho_at", ctypes.c_double), ("sigma_c", ctypes.c_double),
        ("U_i", ctypes.c_double), ("terms", ctypes.c_uint32),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math) into oracle/_build/."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load(path: str):
    handle = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(OrcParams)
    sig = {
        "orc_fft_rows": [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
        "orc_cn_columns": [pp, dp, ctypes.c_double, ctypes.c_int],
        "orc_cn_matrices": [pp, ctypes.c_double, ctypes.c_int, dp],
        "orc_nl_half": [pp, dp, ctypes.c_double, ctypes.c_int],
        "orc_rho_row": [pp, dp, dp],
        "orc_step": [pp, dp, ctypes.c_double, ctypes.c_int],
        "orc_propagate": [pp, dp, ctypes.c_int, dp, ctypes.c_int],
        "orc_diagnostics": [pp, dp, dp, dp, ctypes.c_int],
        "orc_propagate_adaptive": [pp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, dp, ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(handle, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    return handle


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


class use_library:
    """Context manager: route every oracle call through another build of fcn_oracle.c
    (the mutation tests compile copies with a planted mistake)."""

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
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                           "-fno-fast-math", "-ffp-contract=off", "-o", out_path, src, "-lm"])
    return out_path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def params(inst: dict, terms: int | None = None) -> OrcParams:
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name == "terms":
            p.terms = int(inst["terms"] if terms is None else terms)
        elif name in ("nr", "nt", "K"):
            setattr(p, name, int(inst[name]))
        else:
            setattr(p, name, float(inst.get(name, 0.0) if name == "U_i" else inst[name]))
    return p


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(a: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.complex128).copy()
    return out


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


def default_threads() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def fft_rows(a: np.ndarray, inverse: bool = False, threads: int | None = None) -> np.ndarray:
    out = _field(a)
    nr, nt = out.shape
    _check(lib().orc_fft_rows(_dptr(out), nr, nt, int(inverse), threads or default_threads()), "fft")
    return out


def cn_columns(inst: dict, a_freq: np.ndarray, dz: float, threads: int | None = None, terms=None) -> np.ndarray:
    out = _field(a_freq)
    p = params(inst, terms)
    _check(lib().orc_cn_columns(ctypes.byref(p), _dptr(out), float(dz), threads or default_threads()), "cn")
    return out


def cn_matrices(inst: dict, dz: float, col: int, terms=None):
    """(a, b, c, d, e, f) of M_abc and M_def for frequency column ``col``."""
    nr = int(inst["nr"])
    buf = np.zeros(6 * nr, dtype=np.complex128)
    p = params(inst, terms)
    _check(lib().orc_cn_matrices(ctypes.byref(p), float(dz), int(col), _dptr(buf)), "cn_matrices")
    return tuple(buf[k * nr:(k + 1) * nr].copy() for k in range(6))


def nl_half(inst: dict, a: np.ndarray, hz: float, threads: int | None = None, terms=None) -> np.ndarray:
    out = _field(a)
    p = params(inst, terms)
    _check(lib().orc_nl_half(ctypes.byref(p), _dptr(out), float(hz), threads or default_threads()), "nl_half")
    return out


def rho_row(inst: dict, intensity: np.ndarray) -> np.ndarray:
    inten = np.ascontiguousarray(intensity, dtype=np.float64)
    rho = np.zeros_like(inten)
    p = params(inst)
    _check(lib().orc_rho_row(ctypes.byref(p), _dptr(inten), _dptr(rho)), "rho_row")
    return rho


def step(inst: dict, a: np.ndarray, dz: float | None = None, threads: int | None = None, terms=None) -> np.ndarray:
    out = _field(a)
    p = params(inst, terms)
    dz = float(inst["dz"] if dz is None else dz)
    _check(lib().orc_step(ctypes.byref(p), _dptr(out), dz, threads or default_threads()), "step")
    return out


def propagate(inst: dict, a: np.ndarray, nsteps: int, dz=None, threads: int | None = None, terms=None) -> np.ndarray:
    out = _field(a)
    p = params(inst, terms)
    if dz is None:
        dz = inst["dz"]
    dzs = np.ascontiguousarray(np.broadcast_to(np.asarray(dz, dtype=np.float64), (nsteps,)).copy())
    _check(lib().orc_propagate(ctypes.byref(p), _dptr(out), int(nsteps), _dptr(dzs),
                               threads or default_threads()), "propagate")
    return out


def propagate_adaptive(inst: dict, a: np.ndarray, nsteps: int, max_phase: float, dz_min: float,
                       dz_max: float, threads: int | None = None, terms=None):
    out = _field(a)
    p = params(inst, terms)
    log = np.zeros(nsteps, dtype=np.float64)
    _check(lib().orc_propagate_adaptive(ctypes.byref(p), _dptr(out), int(nsteps), float(max_phase),
                                        float(dz_min), float(dz_max), _dptr(log),
                                        threads or default_threads()), "propagate_adaptive")
    return out, log


def diagnostics(inst: dict, a: np.ndarray, threads: int | None = None, terms=None) -> dict:
    f = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.zeros(5, dtype=np.float64)
    flu = np.zeros(int(inst["nr"]), dtype=np.float64)
    p = params(inst, terms)
    _check(lib().orc_diagnostics(ctypes.byref(p), _dptr(f), _dptr(out), _dptr(flu),
                                 threads or default_threads()), "diagnostics")
    return dict(energy=out[0], i_max=out[1], i_axis=out[2], rho_max=out[3], phi=out[4], fluence=flu)

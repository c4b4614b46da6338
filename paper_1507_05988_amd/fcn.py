"""Python binding of the C ABI in include/fcn.h (argument marshalling only).

Every step of the z-step runs in the HIP kernels of libfcn.so; this module only packs
arguments, allocates device buffers with torch and passes raw pointers and the current
torch stream.  There is no CPU fallback: without the built library (or without a GPU)
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcn.so")

FCN_OK, FCN_E_ARG, FCN_E_SIZE, FCN_E_HIP, FCN_E_NONFINITE, FCN_E_STATE, FCN_E_UNSUPPORTED, FCN_E_UNSTABLE = range(8)
FCN_FP64, FCN_FP32, FCN_FP32_STORAGE, FCN_FP32_CN64 = 0, 1, 2, 3
GEOMETRY_RADIAL, GEOMETRY_CARTESIAN = 0, 1  # FCN_RADIAL, FCN_CARTESIAN
PRECISIONS = {"fp64": FCN_FP64, "fp32": FCN_FP32, "fp32_storage": FCN_FP32_STORAGE, "fp32_cn64": FCN_FP32_CN64}
STAGE_FFT, STAGE_IFFT, STAGE_CN, STAGE_NL = 0, 1, 2, 3
DIAG_SCALARS = 8
DIAG_NAMES = ("energy", "i_max", "i_axis", "rho_max", "phi", "z", "step", "dz_prev")

EXPORTED = (
    "fcn_plan_create", "fcn_plan_workspace_size", "fcn_field_size", "fcn_field_offset",
    "fcn_diag_record_size", "fcn_plan_bind", "fcn_step", "fcn_propagate", "fcn_diagnostics",
    "fcn_stage", "fcn_sync", "fcn_last_error", "fcn_plan_destroy", "fcn_plan_tiles", "fcn_step_timed",
    "fcn_net_create", "fcn_net_param_count", "fcn_net_workspace_size", "fcn_net_bind", "fcn_net_refresh",
    "fcn_net_input", "fcn_net_forward", "fcn_net_target", "fcn_net_loss", "fcn_net_backward", "fcn_net_adam",
    "fcn_net_apply", "fcn_net_last_error", "fcn_net_destroy", "fcn_parareal_update",
    "fcn_parareal_workspace_size", "fcn_parareal", "fcn_step_scratch", "fcn_step_timed_launches",
)
SCRATCH_BYTES = 4 << 20  # FCN_SCRATCH_BYTES
PARAREAL_MAX_ITER = 64
PARAREAL_STATUS = {0: "converged", 1: "diverging", 2: "nonfinite", 3: "kmax", 4: "fallback"}


class FcnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"FCN error {code}: {msg}")
        self.code = code


class Instance(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32), ("nt", ctypes.c_int32),
        ("r_max", ctypes.c_double), ("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
        ("lambda0", ctypes.c_double), ("n0", ctypes.c_double), ("k2", ctypes.c_double),
        ("n2", ctypes.c_double), ("n4", ctypes.c_double), ("n6", ctypes.c_double), ("n8", ctypes.c_double),
        ("K", ctypes.c_int32),
        ("sigma_K", ctypes.c_double), ("rho_at", ctypes.c_double), ("sigma_c", ctypes.c_double),
        ("U_i", ctypes.c_double), ("dz", ctypes.c_double),
        ("terms", ctypes.c_uint32),
        ("geometry", ctypes.c_int32), ("ny", ctypes.c_int32), ("y_max", ctypes.c_double),
    ]


class PararealOptions(ctypes.Structure):
    _fields_ = [("windows", ctypes.c_int32), ("steps_per_window", ctypes.c_int32), ("kmax", ctypes.c_int32),
                ("judge", ctypes.c_int32), ("fallback", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double)]


class PararealResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("change", ctypes.c_double * (PARAREAL_MAX_ITER + 1))]


class NetSample(ctypes.Structure):
    _fields_ = [("field_off", ctypes.c_int64), ("coarse_off", ctypes.c_int64), ("row0", ctypes.c_int32),
                ("col0", ctypes.c_int32), ("in_scale", ctypes.c_float), ("out_scale", ctypes.c_float)]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("adaptive", ctypes.c_int32),
        ("max_phase", ctypes.c_double), ("dz_min", ctypes.c_double), ("dz_max", ctypes.c_double),
        ("use_graph", ctypes.c_int32), ("col_tile", ctypes.c_int32), ("col_rows", ctypes.c_int32),
        ("lanes", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfcn.so and declare its signatures; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FcnError(FCN_E_STATE, f"{path} is missing: run `python -m paper_1507_05988_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    plan_p = ctypes.POINTER(vp)
    sig = {
        "fcn_plan_create": ([ctypes.POINTER(Instance), i32, ctypes.POINTER(Options), plan_p], ctypes.c_int),
        "fcn_plan_workspace_size": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_field_size": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_field_offset": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_diag_record_size": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_plan_bind": ([vp, vp, sz, vp], ctypes.c_int),
        "fcn_step": ([vp, vp, i64], ctypes.c_int),
        "fcn_step_scratch": ([vp, vp, i64, vp], ctypes.c_int),
        "fcn_step_timed_launches": ([vp, vp, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                     ctypes.POINTER(i64)], ctypes.c_int),
        "fcn_propagate": ([vp, vp, i64, vp, i32, vp, i32], ctypes.c_int),
        "fcn_diagnostics": ([vp, vp, vp], ctypes.c_int),
        "fcn_stage": ([vp, i32, vp, dbl], ctypes.c_int),
        "fcn_sync": ([vp], ctypes.c_int),
        "fcn_last_error": ([vp], ctypes.c_char_p),
        "fcn_plan_destroy": ([vp], ctypes.c_int),
        "fcn_plan_tiles": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "fcn_step_timed": ([vp, vp, i64, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
                           ctypes.c_int),
        "fcn_net_create": ([i32, i32, plan_p], ctypes.c_int),
        "fcn_net_param_count": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_net_workspace_size": ([vp, i32, i32, i32, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "fcn_net_bind": ([vp, vp, vp, vp, vp, vp, sz, i32, i32, i32, i32, vp], ctypes.c_int),
        "fcn_net_refresh": ([vp], ctypes.c_int),
        "fcn_net_input": ([vp, vp, vp, i32, i32, i32, i32, i32], ctypes.c_int),
        "fcn_net_forward": ([vp, i32, i32, i32, vp], ctypes.c_int),
        "fcn_net_target": ([vp, vp, vp, vp, i32, i32, i32, i32, i32, vp], ctypes.c_int),
        "fcn_net_loss": ([vp, vp, ctypes.POINTER(i32), i32, i32, i32, i32, ctypes.POINTER(dbl)], ctypes.c_int),
        "fcn_net_backward": ([vp, i32, i32, i32], ctypes.c_int),
        "fcn_net_adam": ([vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float], ctypes.c_int),
        "fcn_net_apply": ([vp, vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "fcn_net_last_error": ([vp], ctypes.c_char_p),
        "fcn_net_destroy": ([vp], ctypes.c_int),
        "fcn_parareal_update": ([vp, vp, vp, vp, vp, i32, i32, vp, i32, vp], ctypes.c_int),
        "fcn_parareal_workspace_size": ([i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "fcn_parareal": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, ctypes.c_size_t, ctypes.POINTER(PararealOptions),
                          ctypes.POINTER(PararealResult)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def is_cartesian(inst: dict) -> bool:
    """A Cartesian instance dict has geometry "cartesian" and nx, ny, x_max, y_max in place of
    nr and r_max (field [ny][nx][nt]); any other dict is radial (field [nr][nt])."""
    return inst.get("geometry", "radial") == "cartesian"


def field_shape(inst: dict) -> tuple:
    nt = int(inst["nt"])
    return (int(inst["ny"]), int(inst["nx"]), nt) if is_cartesian(inst) else (int(inst["nr"]), nt)


def rows(inst: dict) -> int:
    """Rows of the row pass: nr, or the nx * ny transverse points of a Cartesian instance."""
    return int(inst["ny"]) * int(inst["nx"]) if is_cartesian(inst) else int(inst["nr"])


def make_instance(inst: dict) -> Instance:
    c = Instance()
    cart = is_cartesian(inst)
    for name, _ in Instance._fields_:
        if name == "geometry":
            c.geometry = GEOMETRY_CARTESIAN if cart else GEOMETRY_RADIAL
            continue
        if name in ("ny", "y_max"):
            setattr(c, name, (int if name == "ny" else float)(inst[name]) if cart else 0)
            continue
        key = {"nr": "nx", "r_max": "x_max"}.get(name, name) if cart else name
        val = inst.get(key, 0.0) if name == "U_i" else inst[key]
        setattr(c, name, int(val) if name in ("nr", "nt", "K", "terms") else float(val))
    return c


class Plan:
    """A batch of pulses stepped together on one GPU.

    instances: list of instance dicts (see workloads.py); precision "fp64", "fp32",
    "fp32_storage" (FP32 field, FP64 arithmetic in the kernels) or "fp32_cn64" (FP32 field and
    row pass with twiddles as hi + lo pairs, FP64-arithmetic column solve).
    The field is one flat complex torch tensor on the device (complex128 for fp64, else complex64),
    instance i occupying [offset(i), offset(i) + nr*nt) as a row-major [nr][nt] matrix (a
    Cartesian instance: nx*ny*nt elements, row-major [ny][nx][nt]).
    """

    def __init__(self, instances, precision: str = "fp64", adaptive: bool = False, max_phase: float = 0.05,
                 dz_min: float = 1e-6, dz_max: float = 1e-2, use_graph: bool = False, col_tile: int = 0,
                 col_rows: int = 0, device: int = 0, stream=None, tune_cache: str | None = None, lanes: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise FcnError(FCN_E_STATE, "no GPU: the FCN library has no CPU path")
        self.torch = torch
        self.lib = load_library()
        if isinstance(instances, dict):
            instances = [instances]
        self.instances = [dict(i) for i in instances]
        self.batch = len(self.instances)
        if precision not in PRECISIONS:
            raise FcnError(FCN_E_ARG, f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        arr = (Instance * self.batch)(*[make_instance(i) for i in self.instances])
        opt = Options(precision=PRECISIONS[precision], adaptive=int(adaptive),
                      max_phase=max_phase, dz_min=dz_min, dz_max=dz_max, use_graph=int(use_graph),
                      col_tile=col_tile, col_rows=col_rows, lanes=lanes,
                      tune_cache=tune_cache.encode() if tune_cache else None)
        self._h = ctypes.c_void_p()
        rc = self.lib.fcn_plan_create(arr, self.batch, ctypes.byref(opt), ctypes.byref(self._h))
        if rc != FCN_OK:
            raise FcnError(rc, "fcn_plan_create rejected the instances or options")
        sz = ctypes.c_size_t()
        self._check(self.lib.fcn_plan_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = sz.value
        self._check(self.lib.fcn_field_size(self._h, ctypes.byref(sz)))
        self.field_elems = sz.value
        self._check(self.lib.fcn_diag_record_size(self._h, ctypes.byref(sz)))
        self.diag_record = sz.value
        self.offsets = []
        for i in range(self.batch):
            self._check(self.lib.fcn_field_offset(self._h, i, ctypes.byref(sz)))
            self.offsets.append(sz.value)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            # 256-byte aligned workspace carved from a torch allocation
            self._ws_buf = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws_buf.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._check(self.lib.fcn_plan_bind(self._h, ctypes.c_void_p(self._ws_ptr), self.workspace_bytes,
                                           ctypes.c_void_p(self.stream.cuda_stream)))

    # ---------------------------------------------------------------- helpers
    def _check(self, rc: int):
        if rc != FCN_OK:
            msg = self.lib.fcn_last_error(self._h).decode() if self._h else ""
            raise FcnError(rc, msg)

    def tiles(self):
        w, l, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.fcn_plan_tiles(self._h, ctypes.byref(w), ctypes.byref(l), ctypes.byref(e)))
        return w.value, l.value, e.value

    def empty_field(self):
        return self.torch.zeros(self.field_elems, dtype=self.cdtype, device=self.device)

    def pack(self, fields) -> "torch.Tensor":
        """List of [nr][nt] (Cartesian: [ny][nx][nt]) numpy arrays, one per instance -> flat
        device field."""
        if isinstance(fields, np.ndarray):
            fields = [fields]
        host = np.zeros(self.field_elems, dtype=np.complex128 if self.precision == "fp64" else np.complex64)
        for i, (f, inst) in enumerate(zip(fields, self.instances)):
            n = rows(inst) * int(inst["nt"])
            host[self.offsets[i]:self.offsets[i] + n] = np.asarray(f).reshape(-1)
        return self.torch.from_numpy(host).to(self.device)

    def unpack(self, field) -> list:
        host = field.detach().to("cpu").numpy()
        out = []
        for i, inst in enumerate(self.instances):
            n = rows(inst) * int(inst["nt"])
            out.append(host[self.offsets[i]:self.offsets[i] + n].reshape(field_shape(inst)).copy())
        return out

    def _field_ptr(self, field):
        if field.device != self.device or field.dtype != self.cdtype or not field.is_contiguous():
            raise FcnError(FCN_E_ARG, "field must be a contiguous device tensor of the plan's dtype")
        if field.numel() < self.field_elems:
            raise FcnError(FCN_E_SIZE, "field tensor is smaller than the plan's field")
        return ctypes.c_void_p(field.data_ptr())

    # ---------------------------------------------------------------- entry points
    def step(self, field, nsteps: int):
        self._check(self.lib.fcn_step(self._h, self._field_ptr(field), int(nsteps)))

    def step_scratch(self, field, nsteps: int, stream=None):
        """fcn_step on the library's static device scratch instead of the plan's workspace
        (the allocation-free entry point); enqueued on `stream` (default: the plan's)."""
        s = self.stream if stream is None else stream
        self._check(self.lib.fcn_step_scratch(self._h, self._field_ptr(field), int(nsteps),
                                              ctypes.c_void_p(s.cuda_stream)))

    def propagate(self, field, nsteps: int, diag_every: int = 0, dz_log=None, replay: bool = False):
        """Steps and returns (diag tensor [records][diag_record] or None)."""
        diag = None
        dptr = None
        if diag_every > 0:
            nrec = nsteps // diag_every + 1
            diag = self.torch.zeros((nrec, self.diag_record), dtype=self.torch.float64, device=self.device)
            dptr = ctypes.c_void_p(diag.data_ptr())
        lptr = None
        if dz_log is not None:
            if dz_log.dtype != self.torch.float64 or dz_log.numel() < nsteps * self.batch:
                raise FcnError(FCN_E_ARG, "dz_log must be float64 with nsteps*batch entries")
            lptr = ctypes.c_void_p(dz_log.data_ptr())
        self._check(self.lib.fcn_propagate(self._h, self._field_ptr(field), int(nsteps), dptr,
                                           int(diag_every), lptr, int(replay)))
        return diag

    def step_timed(self, field, nsteps: int):
        """Steps with HIP events between passes; returns (row_ms, col_ms, total_ms) means."""
        r, c, t = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.fcn_step_timed(self._h, self._field_ptr(field), int(nsteps), ctypes.byref(r),
                                            ctypes.byref(c), ctypes.byref(t)))
        return r.value, c.value, t.value

    def step_timed_launches(self, field, nsteps: int):
        """Steps with HIP events around every launch; returns a list of dicts
        {pass: "row"|"col"|"col_x"|"col_y", size: nt or the system length, points, tile, ms} in
        launch order (tile: elements per thread and rows per workgroup of a row launch, [W, L] of
        a column launch; col_x / col_y: the x and y solves of Cartesian instances)."""
        cap = 64
        n = ctypes.c_int32()
        ms = (ctypes.c_double * cap)()
        info = (ctypes.c_int64 * (5 * cap))()
        self._check(self.lib.fcn_step_timed_launches(self._h, self._field_ptr(field), int(nsteps), cap,
                                                     ctypes.byref(n), ms, info))
        names = ("row", "col", "col_x", "col_y")
        return [{"pass": names[info[5 * i]], "size": int(info[5 * i + 1]),
                 "points": int(info[5 * i + 2]), "tile": [int(info[5 * i + 3]), int(info[5 * i + 4])],
                 "ms": ms[i]} for i in range(n.value)]

    def stage(self, stage: int, field, length: float = 0.0):
        self._check(self.lib.fcn_stage(self._h, int(stage), self._field_ptr(field), float(length)))

    def diagnostics(self, field):
        diag = self.torch.zeros(self.diag_record, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.fcn_diagnostics(self._h, self._field_ptr(field), ctypes.c_void_p(diag.data_ptr())))
        return diag

    def split_diag(self, record) -> list:
        """One diagnostics record -> list of per-instance dicts (scalars + fluence array)."""
        rec = record.detach().to("cpu").numpy() if hasattr(record, "detach") else np.asarray(record)
        out, off = [], 0
        for inst in self.instances:
            nr = rows(inst)
            d = {k: float(rec[off + j]) for j, k in enumerate(DIAG_NAMES)}
            d["fluence"] = rec[off + DIAG_SCALARS:off + DIAG_SCALARS + nr].copy()
            out.append(d)
            off += DIAG_SCALARS + nr
        return out

    def sync(self):
        self._check(self.lib.fcn_sync(self._h))

    def close(self):
        if self._h:
            self.lib.fcn_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

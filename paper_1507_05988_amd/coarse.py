"""Learned coarse z-propagator and parareal along z (additions of this project, not in the paper).

G(U) = C(U) + kappa s Net(U/s): C is one classical FCN step over the whole window length
(50 fine steps of dz in one step of 50 dz), Net the complex convolutional operator of
include/fcn.h (fcn_net_*), s = sqrt(I_ref) one fixed field scale for every pulse (the Kerr
response depends on the absolute intensity, so the network must see it: a per-pulse scale
would hide the pulse power from it) and kappa a fixed output scale (the typical relative
size of F - C over one window) so that the network predicts values of order one.  Parareal over N windows:
U_{j+1}^{k+1} = G(U_j^{k+1}) + F(U_j^k) - G(U_j^k), F = 50 fine FCN steps, with the fine
sweep of all windows batched in one plan.  Every numerical step runs in the HIP kernels of
libfcn.so; this module only orchestrates calls and holds buffers (torch device tensors).
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import fcn
from . import workloads as wl

HALO = 8  # receptive-field radius of 4 layers of 5x5
# field scale of the network: the peak field of a 5 Pcr pulse with w0 = 1 mm (the middle of
# the learned-coarse trajectory family)
S_REF = math.sqrt(wl.peak_intensity(5.0 * wl.critical_power(800e-9, 1.0, 3.2e-23), 1e-3))


def init_params(channels: int, seed: int) -> np.ndarray:
    """Seeded complex initialisation, flat in the layout of include/fcn.h: weights
    (N(0,1) + i N(0,1)) sqrt(1/(2 fan_in)), fan_in = 25 ci; hidden biases 0.01 (1 + i) so
    every CReLU unit starts active, output bias 0; the last layer is scaled by 0.1 so the
    untrained G starts close to the classical coarse step."""
    rng = np.random.default_rng(seed)
    cin = [1, channels, channels, channels]
    cout = [channels, channels, channels, 1]
    parts = []
    for l, (ci, co) in enumerate(zip(cin, cout)):
        std = math.sqrt(1.0 / (2.0 * 25 * ci)) * (0.1 if l == 3 else 1.0)
        w = rng.standard_normal((co, ci, 5, 5, 2)) * std
        parts.append(w.reshape(-1))
        parts.append(np.full(2 * co, 0.01 if l < 3 else 0.0))
    return np.concatenate(parts).astype(np.float32)


def samples_tensor(torch, device, rows):
    """rows: list of (field_off, coarse_off, row0, col0, in_scale, out_scale) -> device NetSample array."""
    arr = (fcn.NetSample * len(rows))()
    for i, (fo, co, r0, c0, isc, osc) in enumerate(rows):
        arr[i] = fcn.NetSample(int(fo), int(co), int(r0), int(c0), float(isc), float(osc))
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


class CoarseNet:
    def __init__(self, channels=32, bf16=True, max_batch=1, max_h=64, max_w=64, training=False, params=None,
                 seed=0, device=0, stream=None, mfma=True):
        import torch

        self.torch = torch
        self.lib = fcn.load_library()
        self.channels = channels
        self.bf16 = bool(bf16)
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        act = (1 if mfma else 2) if bf16 else 0
        self._check(self.lib.fcn_net_create(channels, act, ctypes.byref(self._h)))
        n = ctypes.c_size_t()
        self._check(self.lib.fcn_net_param_count(self._h, ctypes.byref(n)))
        self.nparams = n.value
        p = init_params(channels, seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.size != self.nparams:
            raise fcn.FcnError(fcn.FCN_E_ARG, f"parameter vector has {p.size} floats, network needs {self.nparams}")
        self.params = torch.from_numpy(p.copy()).to(self.device)
        self.training = training
        if training:
            self.grads = torch.zeros_like(self.params)
            self.m = torch.zeros_like(self.params)
            self.v = torch.zeros_like(self.params)
        self._check(self.lib.fcn_net_workspace_size(self._h, max_batch, max_h, max_w, int(training), ctypes.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        self._check(self.lib.fcn_net_bind(self._h, ptr(self.params), ptr(self.grads) if training else None,
                                          ptr(self.m) if training else None, ptr(self.v) if training else None,
                                          ctypes.c_void_p(ws_ptr), n.value, max_batch, max_h, max_w, int(training),
                                          ctypes.c_void_p(self.stream.cuda_stream)))
        self.max_batch, self.max_h, self.max_w = max_batch, max_h, max_w

    def _check(self, rc):
        if rc != fcn.FCN_OK:
            msg = self.lib.fcn_net_last_error(self._h).decode() if self._h else ""
            raise fcn.FcnError(rc, msg)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, p: np.ndarray):
        self.params.copy_(self.torch.from_numpy(np.asarray(p, dtype=np.float32)))
        self._check(self.lib.fcn_net_refresh(self._h))

    def input(self, fields, samples, batch, nr, nt, h, w):
        self._check(self.lib.fcn_net_input(self._h, self._p(fields), self._p(samples), batch, nr, nt, h, w))

    def forward(self, batch, h, w, out=None):
        self._check(self.lib.fcn_net_forward(self._h, batch, h, w, self._p(out) if out is not None else None))

    def target(self, fine, coarse, samples, batch, nr, nt, h, w, target):
        self._check(self.lib.fcn_net_target(self._h, self._p(fine), self._p(coarse), self._p(samples), batch, nr, nt,
                                            h, w, self._p(target)))

    def loss(self, target, row0, batch, h, w, with_grad=True) -> float:
        r = (ctypes.c_int32 * batch)(*[int(x) for x in row0])
        out = ctypes.c_double()
        self._check(self.lib.fcn_net_loss(self._h, self._p(target), r, batch, h, w, int(with_grad),
                                          ctypes.byref(out)))
        return out.value

    def backward(self, batch, h, w):
        self._check(self.lib.fcn_net_backward(self._h, batch, h, w))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.fcn_net_adam(self._h, lr, beta1, beta2, eps))

    def apply(self, coarse, samples, batch, nr, nt, dst):
        self._check(self.lib.fcn_net_apply(self._h, self._p(coarse), self._p(samples), batch, nr, nt, self._p(dst)))

    def params_numpy(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()

    def save(self, path, kappa, s_ref=S_REF, **meta):
        np.savez(path, params=self.params_numpy(), channels=np.int32(self.channels), kappa=np.float64(kappa),
                 s_ref=np.float64(s_ref), bf16=np.int32(1 if self.bf16 else 0), **meta)

    @staticmethod
    def load(path):
        """dict(params, channels, kappa, s_ref, bf16) of a saved network (plain arrays, no pickles)."""
        d = np.load(path, allow_pickle=False)
        return {"params": d["params"], "channels": int(d["channels"]), "kappa": float(d["kappa"]),
                "s_ref": float(d["s_ref"]), "bf16": bool(int(d["bf16"]))}

    def close(self):
        if self._h:
            self.lib.fcn_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CoarseOperator:
    """G(U) on full fields of one grid: the classical coarse step C (`coarse_steps` FCN steps of
    dz * steps_per_window / coarse_steps, one step by default) plus, when a network is given,
    kappa s Net(U/s)."""

    def __init__(self, inst: dict, steps_per_window: int, net_params=None, channels=32, bf16=True, kappa=1.0,
                 coarse_steps=1, precision="fp32", s_ref=S_REF, stream=None):
        import torch

        self.torch = torch
        self.inst = dict(inst)
        self.nr, self.nt = int(inst["nr"]), int(inst["nt"])
        c = dict(inst)
        if steps_per_window % coarse_steps:
            raise ValueError("coarse_steps must divide steps_per_window")
        c["dz"] = inst["dz"] * (steps_per_window // coarse_steps)
        self.coarse_steps = coarse_steps
        self.plan = fcn.Plan(c, precision=precision, stream=stream)
        self.net = None
        if net_params is not None:
            self.net = CoarseNet(channels=channels, bf16=bf16, max_batch=1, max_h=self.nr, max_w=self.nt,
                                 training=False, params=net_params, stream=self.plan.stream)
            self.samples = samples_tensor(torch, self.plan.device, [(0, 0, 0, 0, 1.0 / s_ref, kappa * s_ref)])
        self.tmp = self.plan.empty_field()

    def __call__(self, u, out):
        """out = G(u); u and out are flat complex64 fields of one instance."""
        self.tmp.copy_(u)
        self.plan.step(self.tmp, self.coarse_steps)
        if self.net is None:
            out.copy_(self.tmp)
            return
        self.net.input(u, self.samples, 1, self.nr, self.nt, self.nr, self.nt)
        self.net.forward(1, self.nr, self.nt)
        self.net.apply(self.tmp, self.samples, 1, self.nr, self.nt, out)


def train_coarse(net: CoarseNet, traj_ids, kappa, s_ref=S_REF, batch_traj=16, crops_per_traj=4, crop_h=128,
                 crop_w=128, lr=1e-3,
                 windows=wl.LEARNED_WINDOWS, steps_per_window=wl.LEARNED_STEPS_PER_WINDOW, seed=0, log=None,
                 time_budget=None, make_inst=wl.config_parareal_trajectory, lr_end=None, precision="fp32_storage",
                 warmup=100, updates_per_window=4):
    """Trains `net` on FCN trajectories generated on the fly: for each group of `batch_traj`
    trajectories (one batched fine plan and one batched coarse plan), at every window boundary
    the crops of U_j / s_ref are the inputs and the crops of (F(U_j) - C(U_j)) / (kappa s_ref) the
    targets; `updates_per_window` Adam steps per window, each on freshly drawn crops.  Crops
    cover r rows [0, nr/2) and t columns within nt/8 of the window centre, where the pulse
    is.  `make_inst(j)` gives trajectory j.  The learning rate rises linearly over the first
    `warmup` steps, then decays by cosine from lr to lr_end (default lr/20).  The FCN steps
    run in `precision`: FP32-storage by default, because the coherent error of FP32
    arithmetic over one window is comparable to F - C itself.
    Returns the loss of every step."""
    torch = net.torch
    rng = np.random.default_rng(seed)
    traj_ids = list(traj_ids)
    history = []
    t0 = time.time()
    nb = crops_per_traj
    lr_end = lr / 20 if lr_end is None else lr_end
    total = max(1, ((len(traj_ids) + batch_traj - 1) // batch_traj) * windows * updates_per_window)
    step_no = 0
    for g0 in range(0, len(traj_ids), batch_traj):
        ids = traj_ids[g0:g0 + batch_traj]
        insts = [make_inst(j) for j in ids]
        nr, nt = int(insts[0]["nr"]), int(insts[0]["nt"])
        fine = fcn.Plan(insts, precision=precision, stream=net.stream)
        coarse = fcn.Plan([dict(i, dz=i["dz"] * steps_per_window) for i in insts], precision=precision,
                          stream=net.stream)
        u = fine.pack([wl.gaussian_field(i, np.complex64) for i in insts])
        cbuf = torch.empty_like(u)
        B = len(ids) * nb
        target = torch.empty((B, 2, crop_h, crop_w), dtype=torch.float32, device=u.device)
        ubuf = torch.empty_like(u)
        r_hi = max(1, nr // 2 - crop_h + 1)
        c_span = nt // 8
        for j in range(windows):
            ubuf.copy_(u)
            cbuf.copy_(u)
            coarse.step(cbuf, 1)
            fine.step(u, steps_per_window)
            for _ in range(updates_per_window):
                rows, row0 = [], []
                for k in range(len(insts)):
                    for _ in range(nb):
                        r0 = int(rng.integers(0, r_hi))
                        c0 = int(nt // 2 - crop_w // 2 + rng.integers(-c_span, c_span + 1))
                        rows.append((fine.offsets[k], coarse.offsets[k], r0, c0, 1.0 / s_ref, kappa * s_ref))
                        row0.append(r0)
                smp = samples_tensor(torch, u.device, rows)
                net.input(ubuf, smp, B, nr, nt, crop_h, crop_w)
                net.target(u, cbuf, smp, B, nr, nt, crop_h, crop_w, target)
                net.forward(B, crop_h, crop_w)
                loss = net.loss(target, row0, B, crop_h, crop_w, with_grad=True)
                net.backward(B, crop_h, crop_w)
                frac = min(1.0, step_no / total)
                rate = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * frac))
                net.adam(rate * min(1.0, (step_no + 1) / max(1, warmup)))
                step_no += 1
                history.append(loss)
        fine.sync()
        if log:
            log(f"trajectories {ids[0]}..{ids[-1]}: mean loss over the group "
                f"{np.mean(history[-windows * updates_per_window:]):.4e}, "
                f"{time.time() - t0:.1f} s")
        if time_budget is not None and time.time() - t0 > time_budget:
            break
    return history


def parareal(inst: dict, net_params=None, windows=wl.PARAREAL_WINDOWS, steps_per_window=wl.PARAREAL_STEPS_PER_WINDOW,
             kmax=None, tol=1e-4, reference=None, channels=32, bf16=True, kappa=1.0, coarse_steps=1, fallback=True,
             judge=True, precision="fp32", s_ref=S_REF, stream=None, log=None):
    """Parareal along z for one pulse, with the fine FCN as corrector and judge.

    Iteration k runs the fine FCN over all windows in one batched plan from U^{k-1}, then the
    sequential sweep U_{j+1}^k = G(U_j^k) + F(U_j^{k-1}) - G(U_j^{k-1}).  The judge is the
    r-weighted relative change max_j |U_j^k - U_j^{k-1}| / |U_j^k|: below `tol` the iteration
    has converged; if it grows from one iteration to the next (round-off in grid-scale modes,
    where fine and coarse steps disagree, is being amplified) the previous iterate is kept and
    the iteration stops (judge=False turns this off).  Without convergence and with
    `fallback`, the serial fine solution is
    returned instead.  Returns (fields at the window boundaries U[0..windows], history);
    history[k] = dict(iter, change, error (vs `reference[j]` for U[j+1] if given), seconds);
    iteration 0 is the coarse sweep alone.  The last record carries `status`: "converged",
    "diverging", "nonfinite" (a NaN or Inf change; the iterate is discarded), "kmax" or
    "fallback".  `precision` ("fp32", "fp32_storage" or "fp32_cn64") is that of the
    fine and classical coarse FCN steps; fields are complex64 either way."""
    import torch

    kmax = windows if kmax is None else kmax
    fine = fcn.Plan([inst] * windows, precision=precision, stream=stream)
    st = fine.stream
    G = CoarseOperator(inst, steps_per_window, net_params=net_params, channels=channels, bf16=bf16,
                       kappa=kappa, coarse_steps=coarse_steps, precision=precision, s_ref=s_ref, stream=st)
    nr, nt = int(inst["nr"]), int(inst["nt"])
    n = nr * nt
    off = fine.offsets
    dev = fine.device
    u0 = torch.from_numpy(wl.gaussian_field(inst, np.complex64).reshape(-1)).to(dev)
    U = [u0.clone()] + [torch.empty_like(u0) for _ in range(windows)]
    Gold = [torch.empty_like(u0) for _ in range(windows)]
    t0 = time.time()
    for j in range(windows):  # iteration 0: coarse sweep
        G(U[j], Gold[j])
        U[j + 1].copy_(Gold[j])
    history = []

    def record(k, change, status=None):
        torch.cuda.synchronize(dev)
        rec = dict(iter=k, change=change, seconds=time.time() - t0)
        if reference is not None:
            rec["error"] = max(_werr(U[j + 1], reference[j], nr, nt) for j in range(windows))
        if status:
            rec["status"] = status
        history.append(rec)
        if log:
            log(f"parareal iter {k}: change {change:.3e}" + (f", error {rec['error']:.3e}" if "error" in rec else ""))

    record(0, float("inf"))
    batch = torch.empty(fine.field_elems, dtype=torch.complex64, device=dev)
    gnew = torch.empty_like(u0)
    unew = [u0.clone()] + [torch.empty_like(u0) for _ in range(windows)]
    parts = torch.zeros(2 * 256, dtype=torch.float64, device=dev)
    lib = fine.lib
    prev_change = float("inf")
    status = "kmax"
    for k in range(1, kmax + 1):
        for j in range(windows):
            batch[off[j]:off[j] + n].copy_(U[j])
        fine.step(batch, steps_per_window)
        change = 0.0
        for j in range(windows):
            G(unew[j], gnew)
            rc = lib.fcn_parareal_update(ctypes.c_void_p(gnew.data_ptr()),
                                         ctypes.c_void_p(batch[off[j]:off[j] + n].data_ptr()),
                                         ctypes.c_void_p(Gold[j].data_ptr()), ctypes.c_void_p(U[j + 1].data_ptr()),
                                         ctypes.c_void_p(unew[j + 1].data_ptr()), nr, nt,
                                         ctypes.c_void_p(parts.data_ptr()), 256, ctypes.c_void_p(st.cuda_stream))
            if rc != fcn.FCN_OK:
                raise fcn.FcnError(rc, "parareal update")
            p = parts.view(256, 2).sum(0).cpu().numpy()
            c = math.sqrt(p[0] / max(p[1], 1e-300)) if math.isfinite(p[0]) and math.isfinite(p[1]) else math.nan
            change = math.nan if math.isnan(c) or math.isnan(change) else max(change, c)  # NaN is kept
            Gold[j].copy_(gnew)
        if not math.isfinite(change):  # a non-finite coarse or fine result: never accept it
            status = "nonfinite"
            break
        if judge and change > prev_change:  # growing corrections: keep U^{k-1}
            status = "diverging"
            if history:
                history[-1]["status_next"] = f"iteration {k} change {change:.3e} grew"
            break
        for j in range(1, windows + 1):
            U[j].copy_(unew[j])
        prev_change = change
        if change < tol:
            status = "converged"
            record(k, change, status)
            break
        record(k, change)
    if status != "converged" and fallback:
        ref = serial_fine(inst, windows=windows, steps_per_window=steps_per_window, precision=precision,
                          stream=stream)
        for j in range(windows):
            U[j + 1].copy_(ref[j])
        status = "fallback"
        record(len(history), 0.0, status)
    elif "status" not in history[-1]:
        history[-1]["status"] = status
    return U, history


def parareal_native(inst: dict, net_params=None, windows=wl.PARAREAL_WINDOWS,
                    steps_per_window=wl.PARAREAL_STEPS_PER_WINDOW, kmax=None, tol=1e-4, channels=32, bf16=True,
                    kappa=1.0, fallback=True, judge=True, precision="fp32", s_ref=S_REF, stream=None):
    """Parareal by the library's own driver (fcn_parareal; same iteration, judge and fallback as
    `parareal`, one host synchronisation per iteration).  Returns (U as a [windows + 1, nr*nt]
    complex64 tensor, dict(iterations, status, change, seconds)), seconds the wall time of the
    fcn_parareal call alone."""
    import torch

    kmax = windows if kmax is None else kmax
    nr, nt = int(inst["nr"]), int(inst["nt"])
    fine = fcn.Plan([inst] * windows, precision=precision, stream=stream)
    st = fine.stream
    c = dict(inst, dz=inst["dz"] * steps_per_window)
    crs = fcn.Plan(c, precision=precision, stream=st)
    serial = fcn.Plan(inst, precision=precision, stream=st) if fallback else None
    lib = fine.lib
    net = None
    smp = None
    if net_params is not None:
        net = CoarseNet(channels=channels, bf16=bf16, max_batch=1, max_h=nr, max_w=nt, training=False,
                        params=net_params, stream=st)
        smp = samples_tensor(torch, fine.device, [(0, 0, 0, 0, 1.0 / s_ref, kappa * s_ref)])
    U = torch.zeros((windows + 1, nr * nt), dtype=torch.complex64, device=fine.device)
    U[0].copy_(torch.from_numpy(wl.gaussian_field(inst, np.complex64).reshape(-1)))
    nbytes = ctypes.c_size_t()
    rc = lib.fcn_parareal_workspace_size(nr, nt, windows, ctypes.byref(nbytes))
    if rc != fcn.FCN_OK:
        raise fcn.FcnError(rc, "fcn_parareal_workspace_size")
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=fine.device)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    opt = fcn.PararealOptions(windows, steps_per_window, kmax, int(judge), int(fallback), 0, float(tol))
    res = fcn.PararealResult()
    torch.cuda.synchronize(fine.device)
    t0 = time.perf_counter()
    rc = lib.fcn_parareal(fine._h, crs._h, net._h if net is not None else None,
                          ctypes.c_void_p(smp.data_ptr()) if smp is not None else None,
                          serial._h if serial is not None else None, nr, nt, ctypes.c_void_p(U.data_ptr()),
                          ctypes.c_void_p(ws_ptr), nbytes.value, ctypes.byref(opt), ctypes.byref(res))
    seconds = time.perf_counter() - t0  # the call is synchronous
    if rc != fcn.FCN_OK:
        raise fcn.FcnError(rc, "fcn_parareal")
    out = {"iterations": res.iterations, "status": fcn.PARAREAL_STATUS[res.status],
           "change": [res.change[k] for k in range(1, kmax + 1)], "seconds": seconds}
    return U, out


def _werr(a, ref, nr, nt):
    """r-weighted relative L2 difference (weights m, 1/8 on the axis, 0 on the r_max row)."""
    import torch

    a = a.reshape(nr, nt)
    ref = ref.reshape(nr, nt)
    w = np.arange(nr, dtype=np.float64)
    w[0] = 0.125
    w[-1] = 0.0
    wt = torch.from_numpy(w).to(a.device)[:, None]
    d = (a.to(torch.complex128) - ref.to(torch.complex128)).abs() ** 2
    r = ref.to(torch.complex128).abs() ** 2
    return float(torch.sqrt((wt * d).sum() / (wt * r).sum()))


def serial_fine(inst: dict, windows=wl.PARAREAL_WINDOWS, steps_per_window=wl.PARAREAL_STEPS_PER_WINDOW,
                precision="fp32", stream=None):
    """The serial fine solution at every window boundary (list of `windows` flat fields)."""
    p = fcn.Plan(inst, precision=precision, stream=stream)
    dt = np.complex128 if precision == "fp64" else np.complex64
    f = p.pack(wl.gaussian_field(inst, dt))
    out = []
    for _ in range(windows):
        p.step(f, steps_per_window)
        out.append(f.clone())
    p.sync()
    return out

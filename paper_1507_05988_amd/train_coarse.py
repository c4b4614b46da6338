"""Train the learned coarse z-propagator on FCN trajectories and evaluate it on held-out ones.

Usage: python -m paper_1507_05988_amd.train_coarse [--trajectories 2000] [--channels 32]
           [--fp32-activations] [--out FILE.npz] [--time-budget SECONDS]
(default output: paper_1507_05988_amd/weights/coarse_c<channels>_<bf16|fp32>.npz)

Trajectory j (seeded, see workloads.config_parareal_trajectory) is generated on the GPU by the
fine FCN solver (FP32 storage, FP64 arithmetic by default) over the learned-coarse windows
(workloads.LEARNED_WINDOWS of LEARNED_STEPS_PER_WINDOW steps); training uses j < 2000 and
evaluation the held-out 2000 <= j < 2016.  The output scale kappa is the r-weighted RMS of
|F - C| / |U| over the windows of the first group, so that the network predicts values of
order one; the field scale is coarse.S_REF.  The saved .npz holds plain arrays only.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import coarse, fcn
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights")
HELD_OUT = range(2000, 2016)


def estimate_kappa(ids, steps_per_window=wl.LEARNED_STEPS_PER_WINDOW, windows=wl.LEARNED_WINDOWS,
                   precision="fp32_storage"):
    """r-weighted RMS over the windows of trajectories `ids` of |F(U) - C(U)| / |U| (relative)."""
    import torch

    insts = [wl.config_parareal_trajectory(j) for j in ids]
    nr, nt = int(insts[0]["nr"]), int(insts[0]["nt"])
    fine = fcn.Plan(insts, precision=precision)
    crs = fcn.Plan([dict(i, dz=i["dz"] * steps_per_window) for i in insts], precision=precision)
    u = fine.pack([wl.gaussian_field(i, np.complex64) for i in insts])
    c = torch.empty_like(u)
    vals = []
    for _ in range(windows):
        c.copy_(u)
        crs.step(c, 1)
        fine.step(u, steps_per_window)
        for k in range(len(insts)):
            o = fine.offsets[k]
            vals.append(coarse._werr(c[o:o + nr * nt], u[o:o + nr * nt], nr, nt))
    return float(np.sqrt(np.mean(np.square(vals))))


def coarse_errors(ids, params=None, channels=32, bf16=True, kappa=1.0, s_ref=coarse.S_REF,
                  steps_per_window=wl.LEARNED_STEPS_PER_WINDOW, windows=wl.LEARNED_WINDOWS, precision="fp32_storage"):
    """Per trajectory and window: r-weighted relative error of G(U_j) against F(U_j), U_j on
    the fine trajectory.  Returns an array [len(ids)][windows]."""
    import torch

    out = np.zeros((len(ids), windows))
    for a, j in enumerate(ids):
        inst = wl.config_parareal_trajectory(j)
        nr, nt = int(inst["nr"]), int(inst["nt"])
        G = coarse.CoarseOperator(inst, steps_per_window, net_params=params, channels=channels, bf16=bf16,
                                  kappa=kappa, precision=precision, s_ref=s_ref)
        fine = fcn.Plan(inst, precision=precision, stream=G.plan.stream)
        u = fine.pack(wl.gaussian_field(inst, np.complex64))
        g = torch.empty_like(u)
        for w in range(windows):
            G(u, g)
            fine.step(u, steps_per_window)
            out[a, w] = coarse._werr(g, u, nr, nt)
        fine.sync()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trajectories", type=int, default=2000)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--fp32-activations", action="store_true")
    ap.add_argument("--batch-traj", type=int, default=16)
    ap.add_argument("--crops", type=int, default=4)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--updates-per-window", type=int, default=4)
    ap.add_argument("--windows", type=int, default=wl.LEARNED_WINDOWS)
    ap.add_argument("--steps-per-window", type=int, default=wl.LEARNED_STEPS_PER_WINDOW)
    ap.add_argument("--time-budget", type=float, default=None)
    ap.add_argument("--eval", type=int, default=len(HELD_OUT), help="held-out trajectories to evaluate")
    ap.add_argument("--out", default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32_storage", choices=["fp32", "fp32_storage", "fp32_cn64"],
                    help="precision of the FCN steps that generate the targets")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    bf16 = not args.fp32_activations
    if args.out is None:
        args.out = os.path.join(WEIGHTS, f"coarse_c{args.channels}_{'bf16' if bf16 else 'fp32'}.npz")
    t0 = time.time()
    kappa = estimate_kappa(range(min(args.batch_traj, args.trajectories)), steps_per_window=args.steps_per_window,
                           windows=args.windows, precision=args.precision)
    log(f"kappa (RMS relative |F - C| per window) = {kappa:.4e}")
    B = args.batch_traj * args.crops
    net = coarse.CoarseNet(channels=args.channels, bf16=bf16, max_batch=B, max_h=args.crop, max_w=args.crop,
                           training=True, seed=args.seed)
    hist = coarse.train_coarse(net, range(args.trajectories), kappa=kappa, batch_traj=args.batch_traj,
                               crops_per_traj=args.crops, crop_h=args.crop, crop_w=args.crop, lr=args.lr,
                               seed=args.seed, log=log, time_budget=args.time_budget, precision=args.precision,
                               warmup=args.warmup, updates_per_window=args.updates_per_window,
                               windows=args.windows, steps_per_window=args.steps_per_window)
    t_train = time.time() - t0
    n_traj = min(args.trajectories, (len(hist) // (args.windows * args.updates_per_window)) * args.batch_traj)
    log(f"trained on {n_traj} trajectories, {len(hist)} Adam steps, {t_train:.1f} s")
    params = net.params_numpy()
    ids = list(HELD_OUT)[:args.eval]
    kw = dict(steps_per_window=args.steps_per_window, windows=args.windows, precision=args.precision)
    e_cls = coarse_errors(ids, **kw)
    e_net = coarse_errors(ids, params, channels=args.channels, bf16=bf16, kappa=kappa, **kw)
    log(f"held-out coarse error per window: classical {e_cls.mean():.4e}, learned {e_net.mean():.4e} "
        f"(ratio {e_net.mean() / e_cls.mean():.3f})")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out, kappa, trajectories=np.int32(n_traj), adam_steps=np.int32(len(hist)),
             loss_history=np.asarray(hist, dtype=np.float32), crop=np.int32(args.crop),
             heldout_ids=np.asarray(ids, dtype=np.int32), heldout_err_classical=e_cls, heldout_err_learned=e_net,
             train_seconds=np.float64(t_train), precision=np.array(args.precision),
             windows=np.int32(args.windows), steps_per_window=np.int32(args.steps_per_window))
    log(f"saved {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())

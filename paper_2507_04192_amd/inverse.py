"""Inverse problems through the solver's adjoint (Sec. 3.2): record
observations of a ground-truth run, then fit a parameter field -- a small
MLP on the matrix cores or the plain per-cell table -- by Adam with a
decaying step (Sec. 5: Adam with a decaying learning rate).

Every numerical step runs in the HIP library: the field (MLP or table
gather), the rollout and its adjoint, the network backward and the Adam
update.  This module only sequences the calls.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import native
from . import workloads as W


@dataclasses.dataclass
class History:
    loss: List[float] = dataclasses.field(default_factory=list)
    seconds: float = 0.0


def record(solver, x0, v0, mu, steps, frames, obs):
    """Run the solver from (x0, v0) with floor friction mu and return the
    extraction operators' values at each frame: (lagrangian, eulerian),
    arrays [frame][dim][count] or None."""
    torch = solver.torch
    solver.mpm_init_particles(x0, v0)
    solver.mpm_set_floor_mu(mu)
    d = solver.cfg.dim
    ntr = 0 if obs.get("tracer_pid") is None else len(obs["tracer_pid"])
    nb = 0 if obs.get("box_lo") is None else len(obs["box_lo"])
    dummy = dict(obs)
    if ntr:
        dummy["lag_target"] = np.zeros((len(frames), d, ntr))
    if nb:
        dummy["eul_target"] = np.zeros((len(frames), d, nb))
    solver.mpm_set_observations(frames=frames, **{k: v for k, v in dummy.items() if k != "frames"})
    lag, eul = [], []
    t = 0
    for f in frames:
        solver.mpm_step(f - t)
        t = f
        lq, eq = solver.mpm_extract()
        if lq is not None:
            lag.append(lq.clone())
        if eq is not None:
            eul.append(eq.clone())
    rc, bad = solver.mpm_sync_status()
    if rc != 0:
        raise native.MPMError(rc, f"ground-truth run went non-finite (pid {bad})")
    return (torch.stack(lag) if lag else None), (torch.stack(eul) if eul else None)


def train(solver, x0, steps, frames, obs, targets, field_apply, theta, epochs, lr, decay=0.98,
          target_field: str = "v0", log_every: int = 0):
    """Fit theta: field_apply(theta) gives v0 ([dim, N], when target_field is
    'v0') or the floor friction per node ('mu').  Returns the history."""
    torch = solver.torch
    MLPFunction, MPMRollout = native.autograd_functions()
    lag_t, eul_t = targets
    o = dict(obs)
    if lag_t is not None:
        o["lag_target"] = lag_t
    if eul_t is not None:
        o["eul_target"] = eul_t
    solver.mpm_set_observations(frames=frames, **{k: v for k, v in o.items() if k != "frames"})
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    hist = History()
    t0 = time.perf_counter()
    zeros_v = torch.zeros((solver.cfg.dim, x0.shape[1]), dtype=solver.dtype, device=solver.device)
    for ep in range(epochs):
        th = theta.detach().requires_grad_(True)
        field = field_apply(th)
        if target_field == "v0":
            loss = MPMRollout.apply(field, None, solver, x0, steps)
        else:
            loss = MPMRollout.apply(zeros_v, field.reshape(-1), solver, x0, steps)
        loss.backward()
        native.adam_step(theta, th.grad.contiguous(), m, v, ep + 1, lr * decay ** ep)
        hist.loss.append(float(loss.item()))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            print(f"  epoch {ep:4d} loss {hist.loss[-1]:.6e}", flush=True)
    torch.cuda.synchronize()
    hist.seconds = time.perf_counter() - t0
    return hist


def rel_err(est, true, mask=None):
    """Relative L2 error of a field estimate (arrays or tensors)."""
    e = np.asarray(est.detach().cpu().numpy() if hasattr(est, "detach") else est, dtype=np.float64)
    t = np.asarray(true, dtype=np.float64)
    if mask is not None:
        e, t = e[..., mask], t[..., mask]
    return float(np.linalg.norm(e - t) / np.linalg.norm(t))


def learned_velocity_2d(epochs: int = 60, seed: int = 5, math: str = "bf16", mlp_lr: float = 1e-2,
                        mlp_decay: float = 0.99, cell_lr: float = 0.1, cell_decay: float = 0.98,
                        log_every: int = 0, fit=("mlp", "cells")):
    """Hidden initial velocity of a granular block (Sec. 5 inverse setting):
    v0 = four seeded Gaussian bumps; observations are the velocities of 200
    tracers and the mean velocities in 8 boxes every 20 steps over 400
    steps (FP32 solver, checkpoint every 50).  Fits a 2-64-64-2 tanh MLP
    (MFMA) and a 16 x 8 per-cell table from zero, by the same loss; returns
    their losses and field errors against the hidden field."""
    import torch
    cfg, x0, lo, hi = W.granular_block_2d()
    x0 = x0.astype(np.float32).astype(np.float64)
    n = x0.shape[1]
    v_true = W.eval_bumps(W.gaussian_bumps(seed, lo, hi), x0)
    steps, frames = 400, list(range(20, 401, 20))
    blo, bhi = W.block_boxes(lo, hi)
    obs = dict(tracer_pid=W.pick_tracers(n, 200, seed + 1), lag_field="v", box_lo=blo, box_hi=bhi,
               eul_field="v")
    s = native.Solver(cfg, "f32", capacity=n, tape_steps=steps, ckpt_every=50)
    targets = record(s, x0, v_true, None, steps, frames, obs)
    xin = torch.as_tensor(x0, dtype=torch.float32, device=s.device)
    widths = [2, 64, 64, 2]
    net = native.MLP(widths, in_scale=[2 / (hi[0] - lo[0]), 2 / (hi[1] - lo[1])],
                     in_shift=[-1 - 2 * lo[0] / (hi[0] - lo[0]), -1 - 2 * lo[1] / (hi[1] - lo[1])], math=math)
    out = {"particles": n, "epochs": epochs}
    if "mlp" in fit:
        theta = torch.as_tensor(W.mlp_init_params(widths, seed + 2), device=s.device)
        fa = mlp_field(net, xin)
        with torch.no_grad():
            err0 = rel_err(fa(theta), v_true)
        hm = train(s, x0, steps, frames, obs, targets, fa, theta, epochs, mlp_lr, mlp_decay, log_every=log_every)
        with torch.no_grad():
            out["mlp"] = {"loss": hm.loss, "field_err": rel_err(fa(theta), v_true), "start_err": err0,
                          "seconds": hm.seconds}
    if "cells" in fit:
        cf = native.CellField(2, 16, 8, lo, hi)
        tab = torch.zeros(cf.n_params, dtype=torch.float32, device=s.device)
        fc = cell_field(cf, xin)
        hc = train(s, x0, steps, frames, obs, targets, fc, tab, epochs, cell_lr, cell_decay, log_every=log_every)
        with torch.no_grad():
            out["cells"] = {"loss": hc.loss, "field_err": rel_err(fc(tab), v_true), "seconds": hc.seconds}
    s.close()
    return out


def learned_friction_3d(scale_div: int = 1, epochs: int = 30, steps: int = 2000, ckpt_every: int = 100,
                        n_tracers: int = 500, frame_every: int = 100, seed: int = 8, math: str = "bf16",
                        mlp_lr: float = 3e-3, mlp_decay: float = 0.99, cell_lr: float = 0.02,
                        cell_decay: float = 0.98, cells=(48, 24), log_every: int = 0):
    """Hidden base friction under a 3-D dam-break: mu(x, y) = 0.3 + 0.2
    sin(2 pi x / L) cos(2 pi y / W) + seeded noise per floor node; tracer
    positions every frame_every steps.  Fits a 2-128-128-1 MLP with a
    sigmoid output (friction in [0, 1]) and a per-cell table over the floor,
    both starting at 0.5, through the checkpointed adjoint (FP32).  Field
    errors are over the floor nodes under the initial water column.
    Returns losses, errors, timings and the device memory high-water mark."""
    import torch
    cfg, x0 = W.dam_break_3d(scale_div=scale_div, seed=0)
    x0 = x0.astype(np.float32).astype(np.float64)
    n = x0.shape[1]
    mu_true = W.sinusoid_friction(cfg, seed)
    xy = W.floor_node_coords(cfg)
    L, Wd = cfg.n[0] * cfg.dx, cfg.n[1] * cfg.dx
    col = x0.max(axis=1)
    mask = (xy[0] >= 0) & (xy[0] <= col[0]) & (xy[1] >= 0) & (xy[1] <= col[1])
    frames = list(range(frame_every, steps + 1, frame_every))
    obs = dict(tracer_pid=W.pick_tracers(n, n_tracers, seed + 1), lag_field="x")
    torch.cuda.reset_peak_memory_stats()
    s = native.Solver(cfg, "f32", capacity=n, tape_steps=steps, ckpt_every=ckpt_every)
    targets = record(s, x0, None, mu_true, steps, frames, obs)
    xin = torch.as_tensor(xy, dtype=torch.float32, device=s.device).contiguous()
    widths = [2, 128, 128, 1]
    net = native.MLP(widths, "sigmoid", 1.0, 0.0, in_scale=[2 / L, 2 / Wd], in_shift=[-1.0, -1.0], math=math)
    theta = torch.as_tensor(W.mlp_init_params(widths, seed + 2), device=s.device)
    # start at mu = 0.5 everywhere: zero output-layer weights and bias
    theta[-(widths[-2] + 1):] = 0.0
    fa = mlp_field(net, xin)
    with torch.no_grad():
        err0 = rel_err(fa(theta)[0], mu_true, mask)
    hm = train(s, x0, steps, frames, obs, targets, fa, theta, epochs, mlp_lr, mlp_decay, target_field="mu",
               log_every=log_every)
    with torch.no_grad():
        err_mlp = rel_err(fa(theta)[0], mu_true, mask)
    cf = native.CellField(1, cells[0], cells[1], (0.0, 0.0), (L, Wd))
    tab = torch.full((cf.n_params,), 0.5, dtype=torch.float32, device=s.device)
    fc = cell_field(cf, xin)
    hc = train(s, x0, steps, frames, obs, targets, fc, tab, epochs, cell_lr, cell_decay, target_field="mu",
               log_every=log_every)
    with torch.no_grad():
        err_cell = rel_err(fc(tab)[0], mu_true, mask)
    ws = s.ws.numel()
    s.close()
    return {"particles": n, "grid": list(cfg.n), "steps": steps, "ckpt_every": ckpt_every, "epochs": epochs,
            "workspace_bytes": ws, "max_memory_allocated": torch.cuda.max_memory_allocated(),
            "mlp": {"loss": hm.loss, "field_err": err_mlp, "start_err": err0, "seconds": hm.seconds},
            "cells": {"loss": hc.loss, "field_err": err_cell, "seconds": hc.seconds}}


def mlp_field(net, x_in):
    """field_apply for a network evaluated at fixed inputs x_in [d_in, n]."""
    MLPFunction, _ = native.autograd_functions()
    return lambda th: MLPFunction.apply(th, x_in, net)


def cell_field(field, x_in):
    fn = native.cell_field_function()
    return lambda th: fn.apply(th, x_in, field)


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Learned-field inverse problems through the MPM adjoint")
    ap.add_argument("case", choices=["velocity2d", "friction3d"])
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--scale-div", type=int, default=1, help="friction3d: shrink the dam-break")
    ap.add_argument("--steps", type=int, default=2000, help="friction3d: rollout length")
    ap.add_argument("--log-every", type=int, default=10)
    a = ap.parse_args(argv)
    if a.case == "velocity2d":
        r = learned_velocity_2d(epochs=a.epochs or 60, log_every=a.log_every)
    else:
        r = learned_friction_3d(scale_div=a.scale_div, epochs=a.epochs or 30, steps=a.steps,
                                log_every=a.log_every)
    for k in ("mlp", "cells"):
        if k not in r:
            continue
        r[k]["loss_first"], r[k]["loss_last"] = r[k]["loss"][0], r[k]["loss"][-1]
        del r[k]["loss"]
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()


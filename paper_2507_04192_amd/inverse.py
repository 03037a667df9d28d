"""Inverse problems through the solver's adjoint (Sec. 3.2): record
observations of a ground-truth run, then fit a parameter field -- a small
MLP on the matrix cores or the plain per-cell table -- by Adam with a
decaying step (Sec. 5: Adam with a decaying learning rate).

Every step of the method runs in the HIP library: the field (MLP or table
gather), the rollout and its adjoint, the network backward and the Adam
update.  This module sequences the calls; the only arithmetic it leaves to
torch is the glue of a parameter form (a scalar times a fixed profile, a
zero component appended, a clamp onto [0, 1]).
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
          target_field: str = "v0", log_every: int = 0, trace=None, project=None):
    """Fit theta: field_apply(theta) gives v0 ([dim, N], when target_field is
    'v0') or the floor friction per node ('mu').  trace (a list) receives a
    host copy of theta after every update; project(theta), when given, maps
    theta back into its admissible set after every update.  Returns the
    history."""
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
        if project is not None:
            project(theta)
        if trace is not None:
            trace.append(theta.detach().cpu().numpy().copy())
        hist.loss.append(float(loss.item()))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            print(f"  epoch {ep:4d} loss {hist.loss[-1]:.6e}", flush=True)
    torch.cuda.synchronize()
    hist.seconds = time.perf_counter() - t0
    return hist


def paper_solver(cfg, precision, n, steps, ckpt_every=200, budget=32 << 30):
    """Solver for the paper's 2-D inverse problems (10,000 steps): a
    checkpoint every 200 steps and as many trailing segments on the tape as
    fit in budget bytes -- all 50 at these sizes (8-13 GiB in binary64) --
    so the backward sweep recomputes none."""
    ns = native.max_tape_segments(cfg, precision, n, steps, ckpt_every, budget)
    return native.Solver(cfg, precision, capacity=n, tape_steps=steps, ckpt_every=ckpt_every, tape_segments=ns)


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
                        n_tracers: int = 500, frame_every: int = 20, seed: int = 8, math: str = "bf16",
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


# ---------------------------------------------------------------------------
# The paper's own inverse experiments (Sec. 5.1-5.3), synthetic reproductions
# ---------------------------------------------------------------------------

ALPHA_CASES = {1: "all particle positions (Lagrangian)", 2: "100 particle positions (Lagrangian)",
               3: "mean velocity in 9 monitors (Eulerian)"}


def _last_frames(steps, count, every):
    return list(range(steps - (count - 1) * every, steps + 1, every))


def alpha_inverse(case: int, epochs: int = 60, alpha0: float = 0.1, alpha_true: float = 2.0, lr: float = 0.1,
                  decay: float = 0.98, precision: str = "f64", seed: int = 11, steps: int = 10000,
                  log_every: int = 0):
    """Sec. 5.1: the scalar alpha of the initial velocity v_x = alpha (H0 - y),
    v_y = 0, of a 0.5 x 0.5 m water column, recovered from observations of a
    run with alpha = 2 over its last 100 frames (every 10 steps of the last
    1000 of 10,000 steps, t = 0.3 s): case 1 every particle's position,
    case 2 the positions of 100 random particles, case 3 the mean velocity
    in the nine monitors.  Adam with a decaying rate from alpha = 0.1.
    Returns the loss and alpha histories."""
    import torch
    cfg, x0, H0 = W.inverse_dam_break_2d()
    n = x0.shape[1]
    frames = _last_frames(steps, 100, 10)
    if case == 1:
        obs = dict(tracer_pid=np.arange(n, dtype=np.int32), lag_field="x")
    elif case == 2:
        obs = dict(tracer_pid=W.pick_tracers(n, 100, seed), lag_field="x")
    elif case == 3:
        lo, hi = W.velocity_monitors_2d()
        obs = dict(box_lo=lo, box_hi=hi, eul_field="v")
    else:
        raise ValueError("case is 1, 2 or 3")
    prof = np.stack([H0 - x0[1], np.zeros(n)])
    s = paper_solver(cfg, precision, n, steps)
    targets = record(s, x0, alpha_true * prof, None, steps, frames, obs)
    prof_t = torch.as_tensor(prof, dtype=torch.float32, device=s.device)
    theta = torch.tensor([alpha0], dtype=torch.float32, device=s.device)
    trace = []
    h = train(s, x0, steps, frames, obs, targets, lambda th: th[0] * prof_t, theta, epochs, lr, decay,
              log_every=log_every, trace=trace)
    s.close()
    return {"case": case, "observations": ALPHA_CASES[case], "particles": n, "steps": steps, "epochs": epochs,
            "loss": h.loss, "alpha": [float(a[0]) for a in trace], "alpha_true": alpha_true,
            "seconds": h.seconds}


def profile_inverse(n_obs: int = 1000, epochs: int = 400, lr: float = 1e-2, decay: float = 0.995,
                    precision: str = "f64", math: str = "f32", seed: int = 12, steps: int = 10000,
                    log_every: int = 0):
    """Sec. 5.2: the initial horizontal velocity profile v_x(y) = 2 (1 -
    (y/H0)^2) + 0.2 sin(4 pi y/H0) of the same water column, represented by a
    1-30-30-30-1 ReLU network of y (MFMA kernels), recovered from the
    positions of n_obs random particles over the last 100 frames.  Returns
    the loss history and the relative L2 error of the profile over the
    particles."""
    import torch
    MLPFunction, _ = native.autograd_functions()
    cfg, x0, H0 = W.inverse_dam_break_2d()
    n = x0.shape[1]
    frames = _last_frames(steps, 100, 10)
    obs = dict(tracer_pid=W.pick_tracers(n, n_obs, seed), lag_field="x")
    v_true = np.stack([W.velocity_profile(x0[1], H0), np.zeros(n)])
    s = paper_solver(cfg, precision, n, steps)
    targets = record(s, x0, v_true, None, steps, frames, obs)
    widths = [1, 30, 30, 30, 1]
    net = native.MLP(widths, in_scale=[2.0 / H0], in_shift=[-1.0], math=math, hidden_act="relu")
    y_in = torch.as_tensor(x0[1:2], dtype=torch.float32, device=s.device).contiguous()
    zeros = torch.zeros((1, n), dtype=torch.float32, device=s.device)
    theta = torch.as_tensor(W.mlp_init_params(widths, seed + 1), device=s.device)

    def field(th):
        return torch.cat([MLPFunction.apply(th, y_in, net), zeros], dim=0)

    with torch.no_grad():
        err0 = rel_err(field(theta)[0], v_true[0])
    errs = []
    h = train(s, x0, steps, frames, obs, targets, field, theta, epochs, lr, decay, log_every=log_every)
    with torch.no_grad():
        est = field(theta)[0]
        err = rel_err(est, v_true[0])
        # the learned profile on a uniform grid of heights, for the record
        yg = torch.linspace(0.0, H0, 51, device=s.device, dtype=torch.float32).reshape(1, -1).contiguous()
        prof = MLPFunction.apply(theta, yg, net)[0].cpu().numpy()
    s.close()
    errs.append(err)
    return {"n_obs": n_obs, "particles": n, "epochs": epochs, "loss": h.loss, "start_err": err0,
            "field_err": err, "profile_y": np.linspace(0.0, H0, 51).tolist(), "profile": prof.tolist(),
            "profile_true": W.velocity_profile(np.linspace(0.0, H0, 51), H0).tolist(), "seconds": h.seconds}


def friction_segments_inverse(n_tracers: int = 500, epochs: int = 100, mu0: float = 0.3, lr: float = 0.1,
                              decay: float = 0.98, precision: str = "f64", seed: int = 13, steps: int = 10000,
                              frame_every: int = 10, log_every: int = 0):
    """Sec. 5.3: the Coulomb friction of four equal floor segments under a
    dam-break (truth 0.0, 0.5, 0.1, 0.2), recovered from the positions of
    n_tracers random particles at 1000 frames over 10,000 steps (t = 0.4 s).
    The segments are a 4 x 1 piecewise-constant field over the floor nodes
    (gather/scatter kernels); Adam with a decaying rate from mu0, projected
    onto [0, 1] after every update.  Returns the loss and segment
    histories."""
    import torch
    cfg, x0, seg = W.friction_segments_2d()
    n = x0.shape[1]
    frames = list(range(frame_every, steps + 1, frame_every))
    obs = dict(tracer_pid=W.pick_tracers(n, n_tracers, seed), lag_field="x")
    true = np.asarray(W.FRICTION_SEGMENTS_TRUE)
    mu_true = W.segment_mu(cfg, true, seg_len=seg)
    s = paper_solver(cfg, precision, n, steps)
    targets = record(s, x0, None, mu_true, steps, frames, obs)
    nd = cfg.node_dims()
    xs = (np.arange(nd[0]) - cfg.ghost) * cfg.dx
    nodes = torch.as_tensor(np.stack([xs, np.zeros_like(xs)]), dtype=torch.float32, device=s.device).contiguous()
    L = cfg.n[0] * cfg.dx
    cf = native.CellField(1, len(true), 1, (0.0, -1.0), (L, 1.0))
    theta = torch.full((len(true),), mu0, dtype=torch.float32, device=s.device)
    trace = []
    h = train(s, x0, steps, frames, obs, targets, cell_field(cf, nodes), theta, epochs, lr, decay,
              target_field="mu", log_every=log_every, trace=trace, project=lambda t: t.clamp_(0.0, 1.0))
    s.close()
    return {"n_tracers": n_tracers, "particles": n, "steps": steps, "frames": len(frames), "epochs": epochs,
            "loss": h.loss, "mu": [a.tolist() for a in trace], "mu_true": true.tolist(), "seconds": h.seconds}


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
    ap.add_argument("case", choices=["velocity2d", "friction3d", "alpha", "profile", "segments"])
    ap.add_argument("--alpha-case", type=int, default=3, help="alpha: 1, 2 or 3 (observation strategy)")
    ap.add_argument("--n-obs", type=int, default=500, help="profile: observed particles; segments: tracers")
    ap.add_argument("--out", default=None, help="also write the result as JSON to this file")
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--scale-div", type=int, default=1, help="friction3d: shrink the dam-break")
    ap.add_argument("--steps", type=int, default=2000, help="friction3d: rollout length")
    ap.add_argument("--log-every", type=int, default=10)
    a = ap.parse_args(argv)
    if a.case == "velocity2d":
        r = learned_velocity_2d(epochs=a.epochs or 60, log_every=a.log_every)
    elif a.case == "alpha":
        r = alpha_inverse(a.alpha_case, epochs=a.epochs or 60, log_every=a.log_every)
    elif a.case == "profile":
        r = profile_inverse(n_obs=a.n_obs, epochs=a.epochs or 400, log_every=a.log_every)
    elif a.case == "segments":
        r = friction_segments_inverse(n_tracers=a.n_obs, epochs=a.epochs or 100, log_every=a.log_every)
    else:
        r = learned_friction_3d(scale_div=a.scale_div, epochs=a.epochs or 30, steps=a.steps,
                                log_every=a.log_every)
    for k in ("mlp", "cells"):
        if k not in r:
            continue
        r[k]["loss_first"], r[k]["loss_last"] = r[k]["loss"][0], r[k]["loss"][-1]
        del r[k]["loss"]
    if a.out:
        with open(a.out, "w") as f:
            json.dump(r, f)
    if "loss" in r:
        r = dict(r, loss=[r["loss"][0], r["loss"][-1]])
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()


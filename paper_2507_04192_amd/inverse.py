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


def mlp_field(net, x_in):
    """field_apply for a network evaluated at fixed inputs x_in [d_in, n]."""
    MLPFunction, _ = native.autograd_functions()
    return lambda th: MLPFunction.apply(th, x_in, net)


def cell_field(field, x_in):
    fn = native.cell_field_function()
    return lambda th: fn.apply(th, x_in, field)

"""Shared helpers for the parity tests: run the oracle and the HIP solver on
the very same seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

from paper_2507_04192_amd import workloads as W


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def oracle_state(orc, cfg, x, v=None, C=None, G=None, S=None, Jm1=None):
    d = cfg.dim
    N = x.shape[1]
    F = None
    if G is not None:
        F = np.asarray(G, dtype=np.float64).copy()
        for a in range(d):
            F[a * d + a] += 1.0
    J = None if Jm1 is None else 1.0 + np.asarray(Jm1, dtype=np.float64).reshape(N)
    return orc.State(cfg, x, v=v, C=C, F=F, J=J, S=S)


def gpu_solver(cfg, precision, x, v=None, C=None, G=None, S=None, Jm1=None, keep_grid=False,
               floor_mu=None, capacity=None):
    from paper_2507_04192_amd.native import Solver
    N = x.shape[1]
    s = Solver(cfg, precision, capacity=max(N, 1) if capacity is None else capacity, keep_grid=keep_grid)
    s.mpm_init_particles(x, v)
    if C is not None:
        s.mpm_write_state("C", C, "pid")
    if G is not None:
        s.mpm_write_state("FmI", G, "pid")
    if Jm1 is not None:
        s.mpm_write_state("Jm1", np.asarray(Jm1).reshape(1, -1), "pid")
    if S is not None:
        s.mpm_write_state("stress", S, "pid")
    if floor_mu is not None:
        s.mpm_set_floor_mu(floor_mu)
    return s


def gpu_fields(s):
    st = s.state_numpy("pid")
    return st


def oracle_fields(cfg, st):
    d = cfg.dim
    out = {"x": st.by_pid("x"), "v": st.by_pid("v"), "C": st.by_pid("C"), "stress": st.by_pid("S")}
    if cfg.material in (W.FLUID, W.DP_JAUMANN):
        out["Jm1"] = (st.by_pid("J") - 1.0).reshape(1, -1)
    else:
        F = st.by_pid("F").copy()
        for a in range(d):
            F[a * d + a] -= 1.0
        out["FmI"] = F
    return out


def displacement_error(x_gpu, x_ref, x0, steps, precision):
    """Relative L2 error of the displacement x - x0 and the bound it is held
    to: the stated tolerance (1e-10 binary64, 1e-4 binary32) plus the
    rounding floor of storing positions in the working precision, two units
    of rounding of the largest coordinate per step accumulated as a random
    walk over the steps, relative to the rms displacement.  Positions alone
    (rel-L2 of x) cannot test a short run: its displacement is far below
    the positions' size."""
    x_gpu = np.asarray(x_gpu, dtype=np.float64)
    x_ref = np.asarray(x_ref, dtype=np.float64)
    x0 = np.asarray(x0, dtype=np.float64)
    d_ref = x_ref - x0
    err = rel_l2(x_gpu - x0, d_ref)
    eps = np.finfo(np.float32 if precision == "f32" else np.float64).eps
    rms = np.sqrt(np.mean(d_ref ** 2))
    floor = 2.0 * eps * np.abs(x0).max() * np.sqrt(steps) / max(rms, 1e-300)
    tol = (1e-4 if precision == "f32" else 1e-10) + floor
    return err, tol

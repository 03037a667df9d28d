"""Oracle: plain binary64 CPU reference of the MPM step, its adjoint and the
learned-field network.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The solver never
imports it and the two share no code: this package and the HIP library are
independent implementations of the same equations.

``build()`` compiles ``mpm_oracle.c`` (and the adjoint) with gcc into
``liborc.so`` beside this file; ``lib()`` loads it.  It also compiles the
forward step a second time with complex binary64 data into
``liborc_cs.so`` (``cs_lib()``), for complex-step derivatives of the
forward step that check the hand-written adjoint.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["mpm_oracle.c", "mpm_oracle_adjoint.c"]
LIB_PATH = os.path.join(HERE, "liborc.so")
CS_LIB_PATH = os.path.join(HERE, "liborc_cs.so")

ORC_FLUID, ORC_DP_HENCKY, ORC_HENCKY_ELASTIC, ORC_DP_JAUMANN = 0, 1, 2, 3
_MAT = {"fluid": ORC_FLUID, "sand": ORC_DP_HENCKY, "elastic": ORC_HENCKY_ELASTIC,
        "dp_jaumann": ORC_DP_JAUMANN}
_WALL = {"slip": 0, "stick": 1, "coulomb": 2}
_XFER = {"apic": 0, "pic": 1, "flip": 2, "tpic": 3}
MAX_OBSTACLES = 4


def build(opt: str = "-O2", extra=()) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", opt, "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC",
           "-shared", *extra, *srcs, "-o", LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    # the forward step with complex data; -Bsymbolic keeps its calls inside it
    cmd = ["gcc", opt, "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC",
           "-shared", "-DORC_COMPLEX_STEP", "-Wl,-Bsymbolic", *extra, os.path.join(HERE, "mpm_oracle.c"),
           "-o", CS_LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(CS_LIB_PATH + ".tmp", CS_LIB_PATH)
    return LIB_PATH


class OrcConfig(ct.Structure):
    _fields_ = [
        ("dim", ct.c_int32), ("n", ct.c_int32 * 3), ("ghost", ct.c_int32),
        ("tile", ct.c_int32), ("material", ct.c_int32), ("key_f32", ct.c_int32),
        ("wall_mode", ct.c_int32 * 6),
        ("dx", ct.c_double), ("gravity", ct.c_double * 3), ("wall_mu", ct.c_double * 6),
        ("rho0", ct.c_double), ("bulk", ct.c_double), ("gamma", ct.c_double),
        ("youngs", ct.c_double), ("poisson", ct.c_double), ("phi_deg", ct.c_double),
        ("vol0", ct.c_double), ("mass", ct.c_double),
        ("transfer", ct.c_int32), ("n_obstacles", ct.c_int32),
        ("flip_alpha", ct.c_double), ("viscosity", ct.c_double),
        ("psi_deg", ct.c_double), ("cohesion", ct.c_double), ("tension", ct.c_double),
        ("obst_lo", (ct.c_double * 3) * 4), ("obst_hi", (ct.c_double * 3) * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ct.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_cs_lib = None


def cs_lib():
    """The complex-step build of the forward step (orc_step and its stages
    with complex binary64 data; branches taken on the real parts)."""
    global _cs_lib
    if _cs_lib is None:
        if not os.path.exists(CS_LIB_PATH):
            build()
        _cs_lib = ct.CDLL(CS_LIB_PATH)
        P = ct.c_void_p
        _cs_lib.orc_step.restype = ct.c_int
        _cs_lib.orc_step.argtypes = [P, ct.c_int64, ct.c_double] + [P] * 13
        _cs_lib.orc_node_dims.restype = ct.c_int64
        _cs_lib.orc_node_dims.argtypes = [P, P]
    return _cs_lib


def _declare(L):
    P = ct.c_void_p
    i64, i32, f64 = ct.c_int64, ct.c_int32, ct.c_double
    L.orc_phibar.restype = f64
    L.orc_phibar.argtypes = [f64]
    L.orc_dphibar.restype = f64
    L.orc_dphibar.argtypes = [f64]
    L.orc_stencil_1d.argtypes = [f64, f64, ct.c_int, P, P, P]
    L.orc_node_dims.restype = i64
    L.orc_node_dims.argtypes = [P, P]
    L.orc_num_keys.restype = i64
    L.orc_num_keys.argtypes = [P]
    L.orc_cell_keys.argtypes = [P, i64, P, P]
    L.orc_cells_per_tile.restype = ct.c_int32
    L.orc_cells_per_tile.argtypes = [P]
    L.orc_sort_perm.argtypes = [i64, P, ct.c_int32, P]
    L.orc_p2g.argtypes = [P, i64, f64, P, P, P, P, P, P]
    L.orc_p2g_ex.argtypes = [P, i64, f64, P, P, P, P, P, P, P]
    L.orc_grid_update.argtypes = [P, f64, P, P, P, P]
    L.orc_g2p.argtypes = [P, i64, f64, P, P, P, P, P]
    L.orc_g2p_ex.argtypes = [P, i64, f64, P, P, P, P, P, P]
    L.orc_obstacles.argtypes = [P, P, P]
    L.orc_dp_jaumann.restype = ct.c_int
    L.orc_dp_jaumann.argtypes = [P, f64, P, P, P]
    L.orc_fluid_stress.argtypes = [P, f64, P, P]
    L.orc_sym_eig.argtypes = [ct.c_int, P, P, P]
    L.orc_fluid_pressure.restype = f64
    L.orc_fluid_pressure.argtypes = [P, f64]
    L.orc_cone_alpha.restype = f64
    L.orc_cone_alpha.argtypes = [P]
    L.orc_hencky_return.restype = ct.c_int
    L.orc_hencky_return.argtypes = [P, ct.c_int, P, P, P, P]
    L.orc_constitutive.argtypes = [P, i64, f64, P, P, P, P, P]
    L.orc_step.restype = ct.c_int
    L.orc_step.argtypes = [P, i64, f64, P, P, P, P, P, P, P, P, P, P, P, P, P]
    if hasattr(L, "orc_adjoint_step"):
        _declare_adjoint(L)


def _declare_adjoint(L):
    P = ct.c_void_p
    i64, f64 = ct.c_int64, ct.c_double
    L.orc_adjoint_step.restype = ct.c_int
    L.orc_adjoint_step.argtypes = [P, i64, f64, P] + [P] * 6 + [P] * 6 + [P] * 6 + [P]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def make_config(cfg, key_f32: bool = False) -> OrcConfig:
    """Translate a workloads.SimConfig into the oracle's C struct."""
    c = OrcConfig()
    c.dim = cfg.dim
    for a in range(3):
        c.n[a] = int(cfg.n[a])
        c.gravity[a] = float(cfg.gravity[a])
    c.ghost = cfg.ghost
    c.tile = cfg.tile
    c.material = _MAT[cfg.material]
    c.key_f32 = 1 if key_f32 else 0
    for f in range(6):
        c.wall_mode[f] = _WALL[cfg.wall_mode[f]]
        c.wall_mu[f] = float(cfg.wall_mu[f])
    c.dx = float(cfg.dx)
    c.rho0, c.bulk, c.gamma = float(cfg.rho0), float(cfg.bulk), float(cfg.gamma)
    c.youngs, c.poisson, c.phi_deg = float(cfg.youngs), float(cfg.poisson), float(cfg.phi_deg)
    c.vol0, c.mass = float(cfg.vol0), float(cfg.mass)
    c.transfer = _XFER[cfg.transfer]
    c.flip_alpha = float(cfg.flip_alpha)
    c.viscosity = float(cfg.viscosity)
    c.psi_deg, c.cohesion, c.tension = float(cfg.psi_deg), float(cfg.cohesion), float(cfg.tension)
    obs = list(cfg.obstacles)
    if len(obs) > MAX_OBSTACLES:
        raise ValueError("too many obstacles")
    c.n_obstacles = len(obs)
    for o, (lo, hi) in enumerate(obs):
        for a in range(3):
            c.obst_lo[o][a] = float(lo[a]) if a < len(lo) else 0.0
            c.obst_hi[o][a] = float(hi[a]) if a < len(hi) else 0.0
    return c


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class State:
    """Particle state in the oracle's layout (component-major float64);
    eps is the accumulated equivalent plastic strain."""

    def __init__(self, cfg, x, v=None, C=None, F=None, J=None, S=None, pid=None, eps=None):
        d = cfg.dim
        x = _f64(x).reshape(d, -1)
        N = x.shape[1]
        self.N = N
        self.x = x.copy()
        self.v = np.zeros((d, N)) if v is None else _f64(v).reshape(d, N).copy()
        self.C = np.zeros((d * d, N)) if C is None else _f64(C).reshape(d * d, N).copy()
        if F is None:
            F = np.zeros((d * d, N))
            for a in range(d):
                F[a * d + a] = 1.0
        self.F = _f64(F).reshape(d * d, N).copy()
        self.J = np.ones(N) if J is None else _f64(J).reshape(N).copy()
        self.S = np.zeros((d * d, N)) if S is None else _f64(S).reshape(d * d, N).copy()
        self.pid = np.arange(N, dtype=np.int32) if pid is None else \
            np.ascontiguousarray(pid, dtype=np.int32).copy()
        self.eps = np.zeros(N) if eps is None else _f64(eps).reshape(N).copy()

    def copy(self):
        s = State.__new__(State)
        s.N = self.N
        for k in ("x", "v", "C", "F", "J", "S", "pid", "eps"):
            setattr(s, k, getattr(self, k).copy())
        return s

    def by_pid(self, name):
        """Field reordered so that column p belongs to particle id p."""
        a = getattr(self, name)
        out = np.empty_like(a)
        if a.ndim == 1:
            out[self.pid] = a
        else:
            out[:, self.pid] = a
        return out


class Oracle:
    def __init__(self, cfg, key_f32: bool = False):
        self.cfg = cfg
        self.c = make_config(cfg, key_f32)
        self.L = lib()
        dims = (ct.c_int32 * 3)()
        self.NN = int(self.L.orc_node_dims(ct.byref(self.c), dims))
        self.dims = tuple(dims)

    # single stages -------------------------------------------------------
    def keys(self, x):
        x = _f64(x)
        N = x.shape[-1]
        k = np.empty(N, dtype=np.int32)
        self.L.orc_cell_keys(ct.byref(self.c), N, _ptr(x), _ptr(k))
        return k

    def num_keys(self):
        return int(self.L.orc_num_keys(ct.byref(self.c)))

    def cells_per_tile(self):
        return int(self.L.orc_cells_per_tile(ct.byref(self.c)))

    @staticmethod
    def sort_perm(key, cells_per_tile=64):
        """The step's order of particles with cell keys `key` (tile =
        key // cells_per_tile; every workload here has 64 cells per tile)."""
        key = np.ascontiguousarray(key, dtype=np.int32)
        perm = np.empty_like(key)
        lib().orc_sort_perm(key.shape[0], _ptr(key), int(cells_per_tile), _ptr(perm))
        return perm

    def p2g(self, st: State, dt, with_momentum=False):
        """Nodal mass and momentum-plus-force; with_momentum also returns the
        momentum without the force (FLIP's v^n = that / mass)."""
        d = self.cfg.dim
        gm = np.empty(self.NN)
        gp = np.empty((d, self.NN))
        gq = np.empty((d, self.NN)) if with_momentum else None
        self.L.orc_p2g_ex(ct.byref(self.c), st.N, dt, _ptr(st.x), _ptr(st.v), _ptr(st.C),
                          _ptr(st.S), _ptr(gm), _ptr(gp), _ptr(gq))
        return (gm, gp, gq) if with_momentum else (gm, gp)

    def grid_update(self, gm, gp, dt, floor_mu=None):
        d = self.cfg.dim
        gv = np.empty((d, self.NN))
        fm = None if floor_mu is None else _f64(floor_mu)
        self.L.orc_grid_update(ct.byref(self.c), dt, _ptr(fm), _ptr(_f64(gm)), _ptr(_f64(gp)),
                               _ptr(gv))
        return gv

    def g2p(self, st: State, gv, dt, gv_old=None):
        """Updates st.x, st.v, st.C in place with the configured transfer
        (gv_old: the grid velocity before the update, needed by FLIP); returns
        the velocity gradient L."""
        d = self.cfg.dim
        L = np.empty((d * d, st.N))
        go = None if gv_old is None else _f64(gv_old)
        self.L.orc_g2p_ex(ct.byref(self.c), st.N, dt, _ptr(_f64(gv)), _ptr(go), _ptr(st.x),
                          _ptr(st.v), _ptr(st.C), _ptr(L))
        return L

    def obstacles(self, I, vel):
        """The obstacle rule applied to one node (stored index I) velocity."""
        Ii = (ct.c_int32 * 3)(*[int(v) for v in (list(I) + [0, 0, 0])[:3]])
        v = np.zeros(3)
        v[:len(vel)] = vel
        self.L.orc_obstacles(ct.byref(self.c), Ii, _ptr(v))
        return v[:self.cfg.dim]

    def dp_jaumann(self, L, sigma, dt):
        """One stress update of the hypoelastic Drucker-Prager material:
        returns (sigma', zone, equivalent plastic strain increment)."""
        d = self.cfg.dim
        Lf = _f64(L).reshape(d * d).copy()
        sg = _f64(sigma).reshape(d * d).copy()
        de = ct.c_double(0.0)
        zone = self.L.orc_dp_jaumann(ct.byref(self.c), float(dt), _ptr(Lf), _ptr(sg), ct.byref(de))
        return sg.reshape(d, d), int(zone), de.value

    def fluid_stress(self, J, L):
        """Kirchhoff stress J sigma of the (viscous) fluid at J and velocity gradient L."""
        d = self.cfg.dim
        Lf = _f64(L).reshape(d * d).copy()
        tau = np.empty(d * d)
        self.L.orc_fluid_stress(ct.byref(self.c), float(J), _ptr(Lf), _ptr(tau))
        return tau.reshape(d, d)

    def constitutive(self, st: State, L, dt):
        self.L.orc_constitutive(ct.byref(self.c), st.N, dt, _ptr(_f64(L)), _ptr(st.F),
                                _ptr(st.J), _ptr(st.S), _ptr(st.eps))

    def hencky_return(self, Ftr, elastic_only=False):
        d = self.cfg.dim
        Ftr = _f64(Ftr).reshape(d * d)
        Fe = np.empty(d * d)
        tau = np.empty(d * d)
        dg = ct.c_double(0.0)
        cas = self.L.orc_hencky_return(ct.byref(self.c), 1 if elastic_only else 0, _ptr(Ftr),
                                       _ptr(Fe), _ptr(tau), ct.byref(dg))
        return Fe.reshape(d, d), tau.reshape(d, d), int(cas), dg.value

    def sym_eig(self, A):
        A = _f64(A)
        d = A.shape[0]
        ev = np.empty(3)
        V = np.empty(d * d)
        self.L.orc_sym_eig(d, _ptr(A.reshape(-1)), _ptr(ev), _ptr(V))
        return ev[:d], V.reshape(d, d)

    def pressure(self, J):
        return float(self.L.orc_fluid_pressure(ct.byref(self.c), float(J)))

    def cone_alpha(self):
        return float(self.L.orc_cone_alpha(ct.byref(self.c)))

    # whole step ------------------------------------------------------------
    def step(self, st: State, dt, floor_mu=None, want_grid=False):
        """One step in place (sort, P2G, grid, G2P, constitutive).
        Returns (perm, key[, grid_m, grid_v])."""
        d = self.cfg.dim
        perm = np.empty(st.N, dtype=np.int32)
        key = np.empty(st.N, dtype=np.int32)
        gm = np.empty(self.NN) if want_grid else None
        gv = np.empty((d, self.NN)) if want_grid else None
        fm = None if floor_mu is None else _f64(floor_mu)
        rc = self.L.orc_step(ct.byref(self.c), st.N, dt, _ptr(fm), _ptr(st.x), _ptr(st.v),
                             _ptr(st.C), _ptr(st.F), _ptr(st.J), _ptr(st.S), _ptr(st.pid),
                             _ptr(perm), _ptr(key), _ptr(gm), _ptr(gv), _ptr(st.eps))
        if rc != 0:
            raise MemoryError("oracle step failed to allocate")
        if want_grid:
            return perm, key, gm, gv
        return perm, key

    def step_complex(self, st: State, dt, floor_mu=None):
        """One step of the complex-step build, in place: st's float fields
        hold complex128 arrays (a real state plus i h times a direction), as
        may floor_mu.  The real parts follow step() to rounding (the complex
        square root, logarithm, exponential and power round differently from
        the real ones); the imaginary parts divided by h are the step's
        directional derivative."""
        c128 = lambda a: np.ascontiguousarray(a, dtype=np.complex128)
        for k in ("x", "v", "C", "F", "J", "S", "eps"):
            setattr(st, k, c128(getattr(st, k)))
        perm = np.empty(st.N, dtype=np.int32)
        key = np.empty(st.N, dtype=np.int32)
        fm = None if floor_mu is None else c128(floor_mu)
        rc = cs_lib().orc_step(ct.byref(self.c), st.N, dt, _ptr(fm), _ptr(st.x), _ptr(st.v),
                               _ptr(st.C), _ptr(st.F), _ptr(st.J), _ptr(st.S), _ptr(st.pid),
                               _ptr(perm), _ptr(key), None, None, _ptr(st.eps))
        if rc != 0:
            raise MemoryError("oracle step failed to allocate")
        return perm, key

    def run(self, st: State, steps, dt, floor_mu=None):
        for _ in range(steps):
            self.step(st, dt, floor_mu)
        return st


# ---------------------------------------------------------------------------
# Observation operators, loss and its gradient (Sec. 3.2)
# ---------------------------------------------------------------------------

class Observations:
    """Masked least-squares supervision (eq:inverse_loss).

    frames      steps after which the state is observed (1-based, ascending)
    tracer_pid  particle ids tracked by the Lagrangian operator Q_l(z) = z_l
    lag_field   'x' or 'v'
    lag_target  (n_frames, dim, n_tracers); lag_mask (n_frames, n_tracers)
    box_lo/hi   (n_boxes, dim): Eulerian regions [lo, hi) (half-open)
    eul_field   'x' or 'v'; Q_l = mean over the particles inside the box
    eul_target  (n_frames, dim, n_boxes); eul_mask (n_frames, n_boxes)
    An empty box contributes nothing at that frame; membership is held fixed
    when differentiating.
    """

    def __init__(self, frames, tracer_pid=None, lag_field="x", lag_target=None, lag_mask=None,
                 box_lo=None, box_hi=None, eul_field="v", eul_target=None, eul_mask=None):
        self.frames = [int(f) for f in frames]
        self.tracer_pid = None if tracer_pid is None else np.asarray(tracer_pid, dtype=np.int64)
        self.lag_field = lag_field
        self.lag_target = None if lag_target is None else np.asarray(lag_target, dtype=np.float64)
        self.lag_mask = None if lag_mask is None else np.asarray(lag_mask, dtype=np.float64)
        self.box_lo = None if box_lo is None else np.asarray(box_lo, dtype=np.float64)
        self.box_hi = None if box_hi is None else np.asarray(box_hi, dtype=np.float64)
        self.eul_field = eul_field
        self.eul_target = None if eul_target is None else np.asarray(eul_target, dtype=np.float64)
        self.eul_mask = None if eul_mask is None else np.asarray(eul_mask, dtype=np.float64)


def observe(st, obs, fi):
    """Q values at frame index fi: (lagrangian (dim, n_tr) or None, eulerian
    (dim, n_box) or None, eulerian counts)."""
    lag = eul = cnt = None
    if obs.tracer_pid is not None:
        slot = np.empty(st.N, dtype=np.int64)
        slot[st.pid] = np.arange(st.N)
        z = getattr(st, obs.lag_field)
        lag = z[:, slot[obs.tracer_pid]]
    if obs.box_lo is not None:
        z = getattr(st, obs.eul_field)
        nb = obs.box_lo.shape[0]
        eul = np.zeros((z.shape[0], nb), dtype=z.dtype)
        cnt = np.zeros(nb, dtype=np.int64)
        xr = np.real(st.x)   # membership from the positions (their real part in a complex step)
        for b in range(nb):
            inside = np.all((xr >= obs.box_lo[b][:, None]) & (xr < obs.box_hi[b][:, None]), axis=0)
            cnt[b] = inside.sum()
            if cnt[b] > 0:
                eul[:, b] = z[:, inside].mean(axis=1)
    return lag, eul, cnt


def frame_loss_and_seed(st, obs, fi):
    """Loss of frame fi and its gradient with respect to st's x and v (arrays
    in st's memory order)."""
    loss = 0.0
    gx = np.zeros_like(st.x)
    gv = np.zeros_like(st.v)
    lag, eul, cnt = observe(st, obs, fi)
    if lag is not None:
        m = np.ones(lag.shape[1]) if obs.lag_mask is None else obs.lag_mask[fi]
        r = lag - obs.lag_target[fi]
        loss += float((m * (r * r).sum(axis=0)).sum())
        slot = np.empty(st.N, dtype=np.int64)
        slot[st.pid] = np.arange(st.N)
        g = gx if obs.lag_field == "x" else gv
        np.add.at(g.T, slot[obs.tracer_pid], (2.0 * m * r).T)
    if eul is not None:
        nb = eul.shape[1]
        m = np.ones(nb) if obs.eul_mask is None else obs.eul_mask[fi]
        g = gx if obs.eul_field == "x" else gv
        for b in range(nb):
            if cnt[b] == 0 or m[b] == 0:
                continue
            r = eul[:, b] - obs.eul_target[fi][:, b]
            loss += float(m[b] * (r * r).sum())
            inside = np.all((st.x >= obs.box_lo[b][:, None]) & (st.x < obs.box_hi[b][:, None]), axis=0)
            g[:, inside] += (2.0 * m[b] * r / cnt[b])[:, None]
    return loss, gx, gv


def rollout(cfg, x0, v0, steps, dt, floor_mu=None, obs=None, keep_states=False, state0=None):
    """Forward rollout; returns (loss, states S^0..S^steps if kept, observed Q per frame).
    state0, when given, is the starting state (x0 and v0 are then ignored)."""
    o = Oracle(cfg)
    st = State(cfg, x0, v=v0) if state0 is None else state0.copy()
    states = [st.copy()] if keep_states else None
    loss = 0.0
    frames = {} if obs is None else {f: i for i, f in enumerate(obs.frames)}
    qs = []
    for t in range(steps):
        o.step(st, dt, floor_mu)
        if keep_states:
            states.append(st.copy())
        if (t + 1) in frames:
            fi = frames[t + 1]
            qs.append(observe(st, obs, fi))
            loss += frame_loss_and_seed(st, obs, fi)[0]
    return loss, (states if keep_states else st), qs


def adjoint_step(cfg, st_in, adj_out, dt, floor_mu=None, amu=None):
    """Vector-Jacobian product of one step.  st_in: the step's input state;
    adj_out: dict of adjoints of the step's outputs (x, v, C, F or J, S), in
    the output memory order.  Returns the input adjoints (input order)."""
    L = lib()
    c = make_config(cfg)
    d, N = cfg.dim, st_in.N
    z = lambda *shape: np.zeros(shape)
    out = {"x": z(d, N), "v": z(d, N), "C": z(d * d, N), "F": z(d * d, N), "J": z(N), "S": z(d * d, N)}
    a = {k: np.ascontiguousarray(adj_out.get(k, out[k] * 0), dtype=np.float64) for k in out}
    fm = None if floor_mu is None else _f64(floor_mu)
    rc = L.orc_adjoint_step(ct.byref(c), N, dt, _ptr(fm),
                            _ptr(st_in.x), _ptr(st_in.v), _ptr(st_in.C), _ptr(st_in.F), _ptr(st_in.J),
                            _ptr(st_in.S),
                            _ptr(a["x"]), _ptr(a["v"]), _ptr(a["C"]), _ptr(a["F"]), _ptr(a["J"]), _ptr(a["S"]),
                            _ptr(out["x"]), _ptr(out["v"]), _ptr(out["C"]), _ptr(out["F"]), _ptr(out["J"]),
                            _ptr(out["S"]), _ptr(amu))
    if rc == -2:
        raise NotImplementedError("the oracle's reverse step refused the configuration")
    if rc != 0:
        raise MemoryError("oracle adjoint failed to allocate")
    return out


def rollout_grad(cfg, x0, v0, steps, dt, floor_mu=None, obs=None, state0=None):
    """Loss and its gradient with respect to the initial velocity (pid order)
    and the per-node floor friction, by a reverse sweep over the stored
    states (Sec. 3.1, eq:dzda)."""
    loss, states, _ = rollout(cfg, x0, v0, steps, dt, floor_mu, obs, keep_states=True, state0=state0)
    frames = {} if obs is None else {f: i for i, f in enumerate(obs.frames)}
    d = cfg.dim
    N = states[0].N
    adj = {"x": np.zeros((d, N)), "v": np.zeros((d, N)), "C": np.zeros((d * d, N)),
           "F": np.zeros((d * d, N)), "J": np.zeros(N), "S": np.zeros((d * d, N))}
    amu = None if floor_mu is None else np.zeros_like(np.asarray(floor_mu, dtype=np.float64))
    for t in range(steps - 1, -1, -1):
        if (t + 1) in frames:
            _, gx, gv = frame_loss_and_seed(states[t + 1], obs, frames[t + 1])
            adj["x"] = adj["x"] + gx
            adj["v"] = adj["v"] + gv
        adj = adjoint_step(cfg, states[t], adj, dt, floor_mu, amu)
    # S^0 is in pid order (fresh state)
    gv0 = np.empty_like(adj["v"])
    gv0[:, states[0].pid] = adj["v"]
    return loss, gv0, amu

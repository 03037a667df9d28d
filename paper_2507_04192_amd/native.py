"""ctypes binding of libmpm.so (the C-ABI declared in include/mpm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (the workspace and I/O tensors) and the
stream.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_OK, MPM_EINVAL, MPM_ENOMEM, MPM_EHIP, MPM_ENONFINITE, MPM_EDOMAIN, MPM_ESTATE, MPM_ECONVERGE = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONFINITE", -5: "EDOMAIN",
                -6: "ESTATE", -7: "ECONVERGE"}
MPM_F32, MPM_F64 = 0, 1
MATERIAL = {"fluid": 0, "sand": 1, "elastic": 2, "dp_jaumann": 3}
TRANSFER = {"apic": 0, "pic": 1, "flip": 2, "tpic": 3}
MAX_OBSTACLES = 4
WALL = {"slip": 0, "stick": 1, "coulomb": 2}
FIELD = {"x": 0, "v": 1, "C": 2, "F": 3, "FmI": 4, "J": 5, "Jm1": 6, "stress": 7, "pid": 8, "eps_eq": 9}
ORDER = {"memory": 0, "pid": 1}
GRID = {"mass": 0, "vel": 1}


class MPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class MpmObs(ct.Structure):
    _fields_ = [
        ("n_frames", ct.c_int32), ("host_frames", ct.c_void_p),
        ("n_tracers", ct.c_int32), ("tracer_pid", ct.c_void_p), ("lag_field", ct.c_int32),
        ("lag_target", ct.c_void_p), ("lag_mask", ct.c_void_p),
        ("n_boxes", ct.c_int32), ("host_box_lo", ct.c_void_p), ("host_box_hi", ct.c_void_p),
        ("eul_field", ct.c_int32), ("eul_target", ct.c_void_p), ("eul_mask", ct.c_void_p),
    ]


class MpmMlp(ct.Structure):
    _fields_ = [
        ("n_layers", ct.c_int32), ("width", ct.c_int32 * 5), ("out_act", ct.c_int32), ("math", ct.c_int32),
        ("out_scale", ct.c_float), ("out_shift", ct.c_float),
        ("in_scale", ct.c_float * 4), ("in_shift", ct.c_float * 4), ("hidden_act", ct.c_int32),
    ]


class MpmConfig(ct.Structure):
    _fields_ = [
        ("dim", ct.c_int32), ("precision", ct.c_int32), ("n", ct.c_int32 * 3), ("ghost", ct.c_int32),
        ("tile", ct.c_int32), ("material", ct.c_int32), ("wall_mode", ct.c_int32 * 6),
        ("keep_grid", ct.c_int32),
        ("dx", ct.c_double), ("gravity", ct.c_double * 3), ("wall_mu", ct.c_double * 6),
        ("rho0", ct.c_double), ("bulk", ct.c_double), ("gamma", ct.c_double),
        ("youngs", ct.c_double), ("poisson", ct.c_double), ("phi_deg", ct.c_double),
        ("transfer", ct.c_int32), ("n_obstacles", ct.c_int32),
        ("flip_alpha", ct.c_double), ("viscosity", ct.c_double),
        ("psi_deg", ct.c_double), ("cohesion", ct.c_double), ("tension", ct.c_double),
        ("obst_lo", (ct.c_double * 3) * MAX_OBSTACLES), ("obst_hi", (ct.c_double * 3) * MAX_OBSTACLES),
        ("tape_segments", ct.c_int32), ("track_eps_eq", ct.c_int32),
    ]


_lib = None


def lib():
    """The loaded HIP library; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2507_04192_amd.build`")
        L = ct.CDLL(LIB_PATH)
        P, i32, i64 = ct.c_void_p, ct.c_int32, ct.c_int64
        sig = {
            "mpm_create": ([P, P, P], ct.c_int),
            "mpm_workspace_bytes": ([P, i64, i32, i32, P], ct.c_int),
            "mpm_bind_workspace": ([P, P, ct.c_size_t, i64, i32, i32], ct.c_int),
            "mpm_init_particles": ([P, i64, P, P, ct.c_double, ct.c_double], ct.c_int),
            "mpm_set_floor_mu": ([P, P, i64], ct.c_int),
            "mpm_step": ([P, i32, ct.c_double], ct.c_int),
            "mpm_sync_status": ([P, P], ct.c_int),
            "mpm_read_state": ([P, i32, i32, P], ct.c_int),
            "mpm_write_state": ([P, i32, i32, P], ct.c_int),
            "mpm_read_grid": ([P, i32, P], ct.c_int),
            "mpm_read_sort": ([P, P, P], ct.c_int),
            "mpm_num_particles": ([P], ct.c_int64),
            "mpm_profile_enable": ([P, ct.c_int], ct.c_int),
            "mpm_set_observations": ([P, P], ct.c_int),
            "mpm_forward_loss": ([P, i32, ct.c_double, P], ct.c_int),
            "mpm_backward": ([P, P, P], ct.c_int),
            "mpm_mlp_num_params": ([P], ct.c_int64),
            "mpm_mlp_cache_floats": ([P, i64], ct.c_int64),
            "mpm_mlp_forward": ([P, P, P, i64, P, P, P], ct.c_int),
            "mpm_mlp_backward": ([P, P, P, i64, P, P, P, P, P], ct.c_int),
            "mpm_mlp_backward_noalloc": ([P, P, P, i64, P, P, P, P], ct.c_int),
            "mpm_cell_field_gather": ([P, i32, i32, i32, P, P, i64, P, P, P], ct.c_int),
            "mpm_cell_field_scatter": ([P, i32, i32, i32, P, P, i64, P, P, P], ct.c_int),
            "mpm_extract": ([P, P, P], ct.c_int),
            "mpm_adam_step": ([P, i64, P, P, P, P, i32, ct.c_double, ct.c_double, ct.c_double, ct.c_double],
                              ct.c_int),
            "mpm_profile_read": ([P, P, P], ct.c_int),
            "mpm_last_error": ([P], ct.c_char_p),
            "mpm_destroy": ([P], ct.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return [n for n in _HEADER_NAMES if hasattr(lib(), n)]


_HEADER_NAMES = [
    "mpm_create", "mpm_workspace_bytes", "mpm_bind_workspace", "mpm_init_particles",
    "mpm_set_floor_mu", "mpm_step", "mpm_sync_status", "mpm_read_state", "mpm_write_state",
    "mpm_read_grid", "mpm_read_sort", "mpm_num_particles", "mpm_last_error", "mpm_destroy",
    "mpm_profile_enable", "mpm_profile_read", "mpm_set_observations", "mpm_forward_loss",
    "mpm_backward", "mpm_mlp_num_params", "mpm_mlp_cache_floats", "mpm_mlp_forward", "mpm_mlp_backward",
    "mpm_mlp_backward_noalloc",
    "mpm_adam_step", "mpm_cell_field_gather", "mpm_cell_field_scatter", "mpm_extract",
]
PROF_CLASSES = ["scan", "bucket", "p2g", "grid", "g2p", "g2p_adj", "grid_adj", "p2g_adj"]


def make_config(cfg, precision: str = "f64", keep_grid: bool = False, tape_segments: int = 0,
                track_eps_eq: bool = False) -> MpmConfig:
    """mpm_config from a workloads.SimConfig (tape_segments: trailing
    segments of a forward-plus-adjoint rollout kept on the tape)."""
    c = MpmConfig()
    c.tape_segments = int(tape_segments)
    c.track_eps_eq = 1 if track_eps_eq else 0
    c.dim = cfg.dim
    c.precision = MPM_F64 if precision == "f64" else MPM_F32
    for a in range(3):
        c.n[a] = int(cfg.n[a])
        c.gravity[a] = float(cfg.gravity[a])
    c.ghost = cfg.ghost
    c.tile = cfg.tile
    c.material = MATERIAL[cfg.material]
    for f in range(6):
        c.wall_mode[f] = WALL[cfg.wall_mode[f]]
        c.wall_mu[f] = float(cfg.wall_mu[f])
    c.keep_grid = 1 if keep_grid else 0
    c.dx = float(cfg.dx)
    c.rho0, c.bulk, c.gamma = float(cfg.rho0), float(cfg.bulk), float(cfg.gamma)
    c.youngs, c.poisson, c.phi_deg = float(cfg.youngs), float(cfg.poisson), float(cfg.phi_deg)
    c.transfer = TRANSFER[cfg.transfer]
    c.flip_alpha = float(cfg.flip_alpha)
    c.viscosity = float(cfg.viscosity)
    c.psi_deg, c.cohesion, c.tension = float(cfg.psi_deg), float(cfg.cohesion), float(cfg.tension)
    obs = list(cfg.obstacles)
    if len(obs) > MAX_OBSTACLES:
        raise ValueError(f"at most {MAX_OBSTACLES} obstacles")
    c.n_obstacles = len(obs)
    for o, (lo, hi) in enumerate(obs):
        for a in range(3):
            c.obst_lo[o][a] = float(lo[a]) if a < len(lo) else 0.0
            c.obst_hi[o][a] = float(hi[a]) if a < len(hi) else 0.0
    return c


def max_tape_segments(cfg, precision, n, steps, ckpt_every, budget):
    """The most trailing segments of a steps-long rollout, checkpointed
    every ckpt_every steps, that can stay on the tape with the workspace of
    n particles within budget bytes (mpm_workspace_bytes; at least one)."""
    L = lib()
    nb = ct.c_size_t()
    nseg = (steps + ckpt_every - 1) // ckpt_every
    best = 1
    for ns in range(1, nseg + 1):
        c = make_config(cfg, precision, tape_segments=ns)
        if L.mpm_workspace_bytes(ct.byref(c), int(n), int(steps), int(ckpt_every), ct.byref(nb)) != MPM_OK \
                or nb.value > budget:
            break
        best = ns
    return best


def _check(ctx, rc):
    if rc != MPM_OK:
        msg = lib().mpm_last_error(ctx)
        raise MPMError(rc, msg.decode() if msg else "")


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One solver context with its workspace (a torch uint8 tensor)."""

    def __init__(self, cfg, precision: str = "f64", capacity: Optional[int] = None,
                 tape_steps: int = 0, ckpt_every: int = 0, keep_grid: bool = False, stream=None,
                 tape_segments: int = 0, track_eps_eq: bool = False):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.np_dtype = np.float64 if precision == "f64" else np.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._c = make_config(cfg, precision, keep_grid, tape_segments, track_eps_eq)
        self.L = lib()
        ctx = ct.c_void_p()
        rc = self.L.mpm_create(ct.byref(self._c), ct.c_void_p(self.stream.cuda_stream), ct.byref(ctx))
        _check(None, rc)
        self.ctx = ctx
        self.capacity = capacity
        self.tape_steps, self.ckpt_every = tape_steps, ckpt_every
        self.ws = None
        self._floor_mu = None
        if capacity is not None:
            self.bind(capacity, tape_steps, ckpt_every)

    # -- C-ABI calls ---------------------------------------------------------
    def mpm_workspace_bytes(self, n_particles, tape_steps=0, ckpt_every=0):
        b = ct.c_size_t()
        _check(None, self.L.mpm_workspace_bytes(ct.byref(self._c), n_particles, tape_steps, ckpt_every,
                                                ct.byref(b)))
        return b.value

    def bind(self, capacity, tape_steps=0, ckpt_every=0):
        nbytes = self.mpm_workspace_bytes(capacity, tape_steps, ckpt_every)
        self.ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        _check(self.ctx, self.L.mpm_bind_workspace(self.ctx, ct.c_void_p(aligned), nbytes, capacity,
                                                   tape_steps, ckpt_every))
        self.capacity = capacity
        self.tape_steps, self.ckpt_every = tape_steps, ckpt_every

    def mpm_init_particles(self, x, v=None):
        """x, v: arrays of shape (dim, N) (numpy or torch)."""
        torch = self.torch
        xt = self._dev(x)
        N = xt.shape[1]
        vt = torch.zeros_like(xt) if v is None else self._dev(v)
        if self.ws is None:
            self.bind(N, self.tape_steps, self.ckpt_every)
        _check(self.ctx, self.L.mpm_init_particles(self.ctx, N, _ptr(xt), _ptr(vt), float(self.cfg.vol0),
                                                   float(self.cfg.mass)))
        self._keep = (xt, vt)

    def mpm_set_floor_mu(self, mu):
        if mu is None:
            self._floor_mu = None
            _check(self.ctx, self.L.mpm_set_floor_mu(self.ctx, None, 0))
            return
        t = self._dev(mu).reshape(-1)
        self._floor_mu = t
        _check(self.ctx, self.L.mpm_set_floor_mu(self.ctx, _ptr(t), t.numel()))

    def mpm_step(self, n=1, dt=None):
        dt = self.cfg.dt if dt is None else dt
        _check(self.ctx, self.L.mpm_step(self.ctx, int(n), float(dt)))

    def mpm_sync_status(self):
        bad = ct.c_int64(-1)
        rc = self.L.mpm_sync_status(self.ctx, ct.byref(bad))
        return rc, bad.value

    def num_particles(self):
        return int(self.L.mpm_num_particles(self.ctx))

    def mpm_read_state(self, field, order="memory"):
        torch = self.torch
        N = self.num_particles()
        d = self.cfg.dim
        ncomp = {"x": d, "v": d, "C": d * d, "F": d * d, "FmI": d * d, "J": 1, "Jm1": 1,
                 "stress": d * d, "pid": 1, "eps_eq": 1}[field]
        dt = torch.int32 if field == "pid" else self.dtype
        out = torch.empty((ncomp, N), dtype=dt, device=self.device)
        _check(self.ctx, self.L.mpm_read_state(self.ctx, FIELD[field], ORDER[order], _ptr(out)))
        return out

    def mpm_write_state(self, field, src, order="memory"):
        t = self._dev(src)
        _check(self.ctx, self.L.mpm_write_state(self.ctx, FIELD[field], ORDER[order], _ptr(t)))
        self._keep_w = t

    def mpm_read_grid(self, which):
        torch = self.torch
        nd = self.cfg.node_dims()
        nbox = nd[0] * nd[1] * nd[2]
        ncomp = 1 if which == "mass" else self.cfg.dim
        out = torch.empty((ncomp, nbox), dtype=self.dtype, device=self.device)
        _check(self.ctx, self.L.mpm_read_grid(self.ctx, GRID[which], _ptr(out)))
        return out

    def mpm_read_sort(self):
        torch = self.torch
        N = self.num_particles()
        perm = torch.empty(N, dtype=torch.int32, device=self.device)
        key = torch.empty(N, dtype=torch.int32, device=self.device)
        _check(self.ctx, self.L.mpm_read_sort(self.ctx, _ptr(perm), _ptr(key)))
        return perm, key

    def read_keys(self):
        torch = self.torch
        N = self.num_particles()
        key = torch.empty(N, dtype=torch.int32, device=self.device)
        _check(self.ctx, self.L.mpm_read_sort(self.ctx, None, _ptr(key)))
        return key

    def mpm_set_observations(self, frames, tracer_pid=None, lag_field="x", lag_target=None, lag_mask=None,
                             box_lo=None, box_hi=None, eul_field="v", eul_target=None, eul_mask=None):
        """Observation operators of the loss (see include/mpm.h, mpm_obs)."""
        torch = self.torch
        o = MpmObs()
        fr = np.ascontiguousarray(frames, dtype=np.int32)
        keep = [fr]
        o.n_frames = fr.shape[0]
        o.host_frames = fr.ctypes.data
        if tracer_pid is not None:
            tp = torch.as_tensor(np.asarray(tracer_pid), dtype=torch.int32).to(self.device).contiguous()
            tg = self._dev(lag_target)
            keep += [tp, tg]
            o.n_tracers = tp.numel()
            o.tracer_pid = tp.data_ptr()
            o.lag_field = FIELD[lag_field]
            o.lag_target = tg.data_ptr()
            if lag_mask is not None:
                mk = self._dev(lag_mask)
                keep.append(mk)
                o.lag_mask = mk.data_ptr()
        if box_lo is not None:
            lo = np.ascontiguousarray(box_lo, dtype=np.float64)
            hi = np.ascontiguousarray(box_hi, dtype=np.float64)
            tg = self._dev(eul_target)
            keep += [lo, hi, tg]
            o.n_boxes = lo.shape[0]
            o.host_box_lo = lo.ctypes.data
            o.host_box_hi = hi.ctypes.data
            o.eul_field = FIELD[eul_field]
            o.eul_target = tg.data_ptr()
            if eul_mask is not None:
                mk = self._dev(eul_mask)
                keep.append(mk)
                o.eul_mask = mk.data_ptr()
        _check(self.ctx, self.L.mpm_set_observations(self.ctx, ct.byref(o)))
        self._obs_keep = keep
        self._obs_counts = (o.n_tracers, o.n_boxes)

    def mpm_extract(self):
        """(tracer values [dim, n_tracers], box means [dim, n_boxes]) of the
        current state for the set observations."""
        torch = self.torch
        d = self.cfg.dim
        keep = getattr(self, "_obs_keep", None)
        ntr = nbox = 0
        if keep is not None:
            ntr = int(self._obs_counts[0])
            nbox = int(self._obs_counts[1])
        lq = torch.empty((d, ntr), dtype=self.dtype, device=self.device) if ntr else None
        eq = torch.empty((d, nbox), dtype=self.dtype, device=self.device) if nbox else None
        _check(self.ctx, self.L.mpm_extract(self.ctx, _ptr(lq), _ptr(eq)))
        return lq, eq

    def mpm_forward_loss(self, n_steps, dt=None):
        dt = self.cfg.dt if dt is None else dt
        loss = ct.c_double()
        _check(self.ctx, self.L.mpm_forward_loss(self.ctx, int(n_steps), float(dt), ct.byref(loss)))
        return loss.value

    def mpm_backward(self, want_v0=True, want_mu=True):
        """(dL/dv0 [dim, N] in pid order, dL/dmu per floor node) as tensors."""
        torch = self.torch
        N = self.num_particles()
        gv = torch.empty((self.cfg.dim, N), dtype=self.dtype, device=self.device) if want_v0 else None
        gm = torch.empty(self.cfg.floor_nodes(), dtype=self.dtype, device=self.device) if want_mu else None
        _check(self.ctx, self.L.mpm_backward(self.ctx, _ptr(gv), _ptr(gm)))
        return gv, gm

    def mpm_profile_enable(self, on=True):
        _check(self.ctx, self.L.mpm_profile_enable(self.ctx, 1 if on else 0))

    def mpm_profile_read(self):
        """{class: (total_ms, launches)} since the last read (synchronizes)."""
        ms = (ct.c_double * 8)()
        n = (ct.c_int64 * 8)()
        _check(self.ctx, self.L.mpm_profile_read(self.ctx, ms, n))
        return {name: (ms[i], n[i]) for i, name in enumerate(PROF_CLASSES)}

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mpm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------
    def _dev(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=self.dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype).to(self.device).contiguous()

    def state_numpy(self, order="pid"):
        """All state fields as float64 numpy arrays (synchronizes)."""
        out = {}
        carries_j = self.cfg.material in ("fluid", "dp_jaumann")
        names = ["x", "v", "C", "stress"] + (["Jm1"] if carries_j else ["FmI"])
        for f in names:
            out[f] = self.mpm_read_state(f, order).cpu().numpy().astype(np.float64)
        if order == "memory":
            out["pid"] = self.mpm_read_state("pid", "memory").cpu().numpy()[0]
        return out


# ---------------------------------------------------------------------------
# Learned field: MLP on MFMA, Adam, and autograd glue
# ---------------------------------------------------------------------------

class MLP:
    """alpha(x) = N_theta(x) evaluated by the MFMA kernels (mpm_mlp_*).

    widths: [d_in, hidden..., d_out]; hidden 'tanh' or 'relu'; output 'none'
    or 'sigmoid' followed by out_shift + out_scale * act.  Inputs are mapped
    feature-wise to in_scale * x + in_shift inside the kernel.  math: 'bf16'
    or 'f32'."""

    def __init__(self, widths, out_act="none", out_scale=1.0, out_shift=0.0, in_scale=None, in_shift=None,
                 math="bf16", hidden_act="tanh"):
        import torch
        self.torch = torch
        d = MpmMlp()
        d.n_layers = len(widths) - 1
        for i, wv in enumerate(widths):
            d.width[i] = int(wv)
        d.out_act = {"none": 0, "sigmoid": 1}[out_act]
        d.hidden_act = {"tanh": 0, "relu": 1}[hidden_act]
        d.math = {"bf16": 0, "f32": 1}[math]
        d.out_scale, d.out_shift = float(out_scale), float(out_shift)
        for k in range(4):
            d.in_scale[k] = float(in_scale[k]) if in_scale is not None and k < len(in_scale) else 1.0
            d.in_shift[k] = float(in_shift[k]) if in_shift is not None and k < len(in_shift) else 0.0
        self.desc = d
        self.widths = list(widths)
        self.L = lib()
        self.n_params = int(self.L.mpm_mlp_num_params(ct.byref(d)))
        if self.n_params < 0:
            raise MPMError(MPM_EINVAL, "invalid network description")

    def _stream(self):
        return ct.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def cache_floats(self, n):
        return int(self.L.mpm_mlp_cache_floats(ct.byref(self.desc), n))

    def forward(self, params, x):
        """x: float32 cuda tensor [d_in, n]; returns (y [d_out, n], cache)."""
        torch = self.torch
        n = x.shape[1]
        y = torch.empty((self.widths[-1], n), dtype=torch.float32, device=x.device)
        cache = torch.empty(max(self.cache_floats(n), 1), dtype=torch.float32, device=x.device)
        rc = self.L.mpm_mlp_forward(ct.byref(self.desc), self._stream(), _ptr(params), n, _ptr(x), _ptr(y),
                                    _ptr(cache))
        _check(None, rc)
        return y, cache

    def backward(self, params, x, cache, dy):
        torch = self.torch
        n = x.shape[1]
        work = torch.empty_like(cache)
        dp = torch.empty_like(params)
        rc = self.L.mpm_mlp_backward(ct.byref(self.desc), self._stream(), _ptr(params), n, _ptr(x), _ptr(cache),
                                     _ptr(dy.contiguous()), _ptr(work), _ptr(dp))
        _check(None, rc)
        return dp

    def backward_noalloc_into(self, params, x, cache, dy, dparams):
        """The backward pass through mpm_mlp_backward_noalloc (the work buffer
        is the library's static device array; nothing is allocated by the
        call): writes the parameter gradient into the caller's dparams."""
        n = x.shape[1]
        rc = self.L.mpm_mlp_backward_noalloc(ct.byref(self.desc), self._stream(), _ptr(params), n, _ptr(x),
                                             _ptr(cache), _ptr(dy), _ptr(dparams))
        _check(None, rc)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update on float32 cuda tensors (mpm_adam_step)."""
    import torch
    L = lib()
    rc = L.mpm_adam_step(ct.c_void_p(torch.cuda.current_stream().cuda_stream), params.numel(), _ptr(params),
                         _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1), float(beta2), float(eps))
    _check(None, rc)


def _autograd():
    import torch

    class MLPFunction(torch.autograd.Function):
        """y = N_theta(x); gradient with respect to theta only."""

        @staticmethod
        def forward(ctx, params, x, net):
            y, cache = net.forward(params, x)
            ctx.save_for_backward(params, x, cache)
            ctx.net = net
            return y

        @staticmethod
        def backward(ctx, dy):
            params, x, cache = ctx.saved_tensors
            return ctx.net.backward(params, x, cache, dy.float()), None, None

    class MPMRollout(torch.autograd.Function):
        """loss = L(v0, mu): a checkpointed rollout of the solver from its
        initial positions (forward: mpm_forward_loss) and the hand-written
        reverse sweep (backward: mpm_backward)."""

        @staticmethod
        def forward(ctx, v0, mu, solver, x0, steps):
            solver.mpm_init_particles(x0, v0.to(solver.dtype))
            if mu is not None:
                solver.mpm_set_floor_mu(mu.to(solver.dtype))
            loss = solver.mpm_forward_loss(steps)
            ctx.solver = solver
            ctx.has_mu = mu is not None
            ctx.v0_dtype = v0.dtype
            ctx.mu_dtype = None if mu is None else mu.dtype
            return torch.tensor(loss, dtype=torch.float64, device=v0.device)

        @staticmethod
        def backward(ctx, gl):
            gv, gm = ctx.solver.mpm_backward(want_v0=True, want_mu=ctx.has_mu)
            gv = (gv * gl).to(ctx.v0_dtype)
            gm = None if gm is None else (gm * gl).to(ctx.mu_dtype)
            return gv, gm, None, None, None

    return MLPFunction, MPMRollout


_fns = None


def autograd_functions():
    """(MLPFunction, MPMRollout) torch.autograd.Function classes."""
    global _fns
    if _fns is None:
        _fns = _autograd()
    return _fns


class CellField:
    """Piecewise-constant parametric field (mpm_cell_field_gather/scatter):
    nc components on an nx x ny grid over [lo, hi) of the first two
    coordinates."""

    def __init__(self, nc, nx, ny, lo, hi):
        self.nc, self.nx, self.ny = int(nc), int(nx), int(ny)
        self.lo = np.ascontiguousarray(lo[:2], dtype=np.float64)
        self.hi = np.ascontiguousarray(hi[:2], dtype=np.float64)
        self.n_params = self.nc * self.nx * self.ny
        self.L = lib()

    def _s(self):
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)

    def gather(self, table, x):
        import torch
        n = x.shape[1]
        out = torch.empty((self.nc, n), dtype=torch.float32, device=x.device)
        _check(None, self.L.mpm_cell_field_gather(self._s(), self.nc, self.nx, self.ny, self.lo.ctypes.data,
                                                  self.hi.ctypes.data, n, _ptr(x), _ptr(table), _ptr(out)))
        return out

    def scatter(self, x, dout):
        import torch
        n = x.shape[1]
        dt = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        _check(None, self.L.mpm_cell_field_scatter(self._s(), self.nc, self.nx, self.ny, self.lo.ctypes.data,
                                                   self.hi.ctypes.data, n, _ptr(x), _ptr(dout.contiguous()),
                                                   _ptr(dt)))
        return dt


def cell_field_function():
    import torch

    class CellFieldFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, table, x, field):
            ctx.save_for_backward(x)
            ctx.field = field
            return field.gather(table, x)

        @staticmethod
        def backward(ctx, dout):
            (x,) = ctx.saved_tensors
            return ctx.field.scatter(x, dout.float()), None, None

    return CellFieldFunction

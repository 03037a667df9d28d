"""Seeded synthetic inputs and simulation settings.

This module is shared by the solver's tests, the benchmark and the oracle's
tests.  It holds configuration values and random draws only -- no step of the
method's arithmetic -- so that both the HIP solver and the oracle can be fed
the very same arrays.

Particle seeding: lattice points at (k + (j + 1/2)/m) h per axis, j < m for m
particles per cell per axis, kept when the *unjittered* point lies inside
the body, then jittered by a uniform draw in [-0.1 h, 0.1 h] per component.
All random numbers come from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

FLUID = "fluid"          # weakly compressible Tait fluid (optionally viscous)
SAND = "sand"            # Drucker-Prager sand, Hencky-strain return
ELASTIC = "elastic"      # Hencky elastic (no return), used by checks
DP_JAUMANN = "dp_jaumann"   # hypoelastic Drucker-Prager, Jaumann rate, tension cutoff

APIC, PIC, FLIP, TPIC = "apic", "pic", "flip", "tpic"   # grid-to-particle transfers

SLIP, STICK, COULOMB = "slip", "stick", "coulomb"


@dataclasses.dataclass
class SimConfig:
    dim: int
    n: Tuple[int, int, int]
    dx: float
    dt: float
    material: str
    ppc: int                         # particles per cell (total)
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    wall_mode: Tuple[str, ...] = (SLIP,) * 6   # x-, x+, y-, y+, z-, z+
    wall_mu: Tuple[float, ...] = (0.0,) * 6
    rho0: float = 1000.0
    bulk: float = 1.0e5
    gamma: float = 7.0
    youngs: float = 1.0e7
    poisson: float = 0.3
    phi_deg: float = 30.0
    ghost: int = 2
    tile: int = 0                    # 0: 4 in 3D, 8 in 2D
    transfer: str = APIC
    flip_alpha: float = 1.0          # FLIP share of the FLIP/PIC blend
    viscosity: float = 0.0           # fluid dynamic viscosity (Pa s)
    psi_deg: float = 0.0             # dilation angle (DP_JAUMANN)
    cohesion: float = 0.0            # c (DP_JAUMANN)
    tension: float = 0.0             # tensile cutoff sigma^t (DP_JAUMANN)
    obstacles: Tuple = ()            # resting rigid boxes: ((lo...), (hi...)) each

    def __post_init__(self):
        n = tuple(int(v) for v in self.n) + (1,) * (3 - len(self.n))
        self.n = n[:3]
        if self.tile == 0:
            self.tile = 4 if self.dim == 3 else 8

    @property
    def vol0(self) -> float:
        return self.dx ** self.dim / self.ppc

    @property
    def mass(self) -> float:
        return self.rho0 * self.vol0

    @property
    def extent(self) -> Tuple[float, ...]:
        return tuple(self.n[a] * self.dx for a in range(self.dim))

    def node_dims(self) -> Tuple[int, int, int]:
        """Nodes per axis of the dense padded grid (ghost layers included)."""
        return tuple(self.n[a] + 1 + 2 * self.ghost if a < self.dim else 1 for a in range(3))

    def floor_nodes(self) -> int:
        nd = self.node_dims()
        return nd[0] if self.dim == 2 else nd[0] * nd[1]

    def replace(self, **kw) -> "SimConfig":
        return dataclasses.replace(self, **kw)


def lattice_particles(cfg: SimConfig, inside: Callable[[np.ndarray], np.ndarray],
                      lo: Sequence[float], hi: Sequence[float], seed: int,
                      per_axis: int = 2, jitter: float = 0.1) -> np.ndarray:
    """Seeded particles, shape (dim, N), float64, component-major."""
    d, h = cfg.dim, cfg.dx
    axes = []
    for a in range(d):
        c0 = int(math.floor(lo[a] / h))
        c1 = int(math.ceil(hi[a] / h))
        cells = np.arange(c0, c1, dtype=np.float64)
        offs = (np.arange(per_axis, dtype=np.float64) + 0.5) / per_axis
        axes.append(((cells[:, None] + offs[None, :]) * h).reshape(-1))
    grids = np.meshgrid(*axes, indexing="ij")
    # x varies fastest in the particle order
    pts = np.stack([g.transpose(*range(d)[::-1]).reshape(-1) for g in grids], axis=0)
    keep = inside(pts)
    pts = pts[:, keep]
    rng = np.random.default_rng(seed)
    pts = pts + rng.uniform(-jitter * h, jitter * h, size=pts.shape)
    for a in range(d):
        np.clip(pts[a], 0.0, cfg.n[a] * h, out=pts[a])
    return np.ascontiguousarray(pts)


def box_inside(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)

    def f(p):
        ok = np.ones(p.shape[1], dtype=bool)
        for a in range(p.shape[0]):
            ok &= (p[a] >= lo[a]) & (p[a] < hi[a])
        return ok
    return f


def cylinder_inside(cx, cy, radius, height):
    def f(p):
        r2 = (p[0] - cx) ** 2 + (p[1] - cy) ** 2
        return (r2 < radius * radius) & (p[2] >= 0.0) & (p[2] < height)
    return f


# ---------------------------------------------------------------------------
# Workloads (sizes follow the benchmark definitions; see the design notes)
# ---------------------------------------------------------------------------

def dam_break_2d(scale: int = 1, seed: int = 0):
    """2-D dam-break: 2.0 x 1.0 m domain at 128 x 64 cells (scale 1),
    water column 0.5 x 1.0 m, 2 x 2 particles per cell, Tait K=1e5,
    rho=1000, gamma=7, gravity -9.81, slip walls, dt = 1e-4 s (the same dt
    at every scale)."""
    n = (128 * scale, 64 * scale, 1)
    dx = 1.0 / (64 * scale)
    cfg = SimConfig(dim=2, n=n, dx=dx, dt=1e-4, material=FLUID, ppc=4,
                    gravity=(0.0, -9.81, 0.0), rho0=1000.0, bulk=1.0e5, gamma=7.0)
    x = lattice_particles(cfg, box_inside((0.0, 0.0), (0.5, 1.0)), (0.0, 0.0), (0.5, 1.0), seed)
    return cfg, x


def cylinder_collapse_3d(scale_div: int = 1, seed: int = 0):
    """3-D granular cylinder collapse: 256 x 256 x 64 cells, dx = 0.005 m,
    cylinder of radius and height 48 cells at the domain centre, 2x2x2
    particles per cell, Drucker-Prager sand E=1e7, nu=0.3, phi=30 deg,
    rho=2000, floor Coulomb mu = 0.5, other walls slip, dt = 2e-5 s.
    scale_div > 1 shrinks every length (cells and cylinder) by that factor
    at the same dx."""
    s = scale_div
    n = (256 // s, 256 // s, 64 // s)
    dx = 0.005
    modes = (SLIP, SLIP, SLIP, SLIP, COULOMB, SLIP)
    mus = (0.0, 0.0, 0.0, 0.0, 0.5, 0.0)
    cfg = SimConfig(dim=3, n=n, dx=dx, dt=2e-5, material=SAND, ppc=8,
                    gravity=(0.0, 0.0, -9.81), wall_mode=modes, wall_mu=mus,
                    rho0=2000.0, youngs=1.0e7, poisson=0.3, phi_deg=30.0)
    R = 48 * dx / s
    cx, cy = n[0] * dx / 2, n[1] * dx / 2
    x = lattice_particles(cfg, cylinder_inside(cx, cy, R, R),
                          (cx - R, cy - R, 0.0), (cx + R, cy + R, R), seed)
    return cfg, x


def paper_granular_material(cfg: SimConfig, phi_deg: float) -> SimConfig:
    """The granular material of the paper's 3-D collapses (Sec. 4.1.2, kept
    in Sec. 4.2.2-4.2.3): the hypoelastic Drucker-Prager model of App. A
    with rho = 2650 kg/m^3, K = 0.7 MPa (E = 3K(1 - 2nu) = 0.84 MPa),
    nu = 0.3, c = 0, psi = 0 and the friction angle phi_deg; a no-slip
    base, slip walls elsewhere; dt = 1e-5 s."""
    return cfg.replace(material=DP_JAUMANN, rho0=2650.0, youngs=3 * 0.7e6 * (1 - 2 * 0.3), poisson=0.3,
                       phi_deg=float(phi_deg), psi_deg=0.0, cohesion=0.0, dt=1e-5,
                       wall_mode=(SLIP, SLIP, SLIP, SLIP, STICK, SLIP), wall_mu=(0.0,) * 6)


def cylinder_paper_grid(scale_div: int = 1, seed: int = 0):
    """The paper's timing case of the 3-D cylinder collapse (Sec. 4.2.3,
    Table tab:simulation_params): a 400 x 400 x 100 grid at dx = 1/400 m
    and a sand cylinder of radius and height 47.68 cells (0.1192 m) at the
    domain centre, 2x2x2 particles per cell: 2,713,580 particles, the
    table's 2,712,960 within 0.03% (the text gives neither dimension; this
    radius is the one whose lattice count comes closest), with the paper's
    granular material at phi = 20 deg (the first of the friction angles the
    section compares).  scale_div shrinks every length."""
    s = scale_div
    n = (400 // s, 400 // s, 100 // s)
    dx = 1.0 / 400.0
    cfg = paper_granular_material(SimConfig(dim=3, n=n, dx=dx, dt=1e-5, material=SAND, ppc=8,
                                            gravity=(0.0, 0.0, -9.81)), phi_deg=20.0)
    R = 47.68 * dx / s
    cx, cy = n[0] * dx / 2, n[1] * dx / 2
    x = lattice_particles(cfg, cylinder_inside(cx, cy, R, R), (cx - R, cy - R, 0.0), (cx + R, cy + R, R), seed)
    return cfg, x


def granular_column_paper(scale_div: int = 1, seed: int = 0):
    """The paper's timing case of the 3-D granular column (Sec. 4.2.2,
    Table tab:simulation_params): a 400 x 32 x 200 grid at dx = 1/400 m;
    the column of aspect ratio 3 fills the width: L0 = 56 cells (0.14 m),
    H0 = 168 cells (0.42 m), 32 cells wide, at 2x2x2 particles per cell
    (2,408,448 particles, the table's count), with the paper's granular
    material (phi = 19.8 deg, unchanged from Sec. 4.1.2).  scale_div
    shrinks the length and the height."""
    s = scale_div
    n = (400 // s, 32, 200 // s)
    dx = 1.0 / 400.0
    cfg = paper_granular_material(SimConfig(dim=3, n=n, dx=dx, dt=1e-5, material=SAND, ppc=8,
                                            gravity=(0.0, 0.0, -9.81)), phi_deg=19.8)
    hi = (56 * dx / s, 32 * dx, 168 * dx / s)
    x = lattice_particles(cfg, box_inside((0, 0, 0), hi), (0, 0, 0), hi, seed)
    return cfg, x


def friction_dam_break_2d(seed_mu: int = 2, seed_eval: int = 3, seed_tracers: int = 4,
                          scale: int = 2):
    """Dam-break at 256 x 128 cells with 32 floor segments of friction."""
    cfg, x = dam_break_2d(scale=scale, seed=0)
    modes = (SLIP, SLIP, COULOMB, SLIP, SLIP, SLIP)
    cfg = cfg.replace(wall_mode=modes)
    return cfg, x


def segment_mu(cfg: SimConfig, mu_seg: np.ndarray, seg_len: float = 0.0625) -> np.ndarray:
    """Expand per-segment floor friction to one value per floor node
    (node x = i*h, segment = clamp(floor(x / seg_len), 0, nseg-1))."""
    nd = cfg.node_dims()
    i = np.arange(nd[0]) - cfg.ghost
    xs = i * cfg.dx
    seg = np.clip(np.floor(xs / seg_len).astype(np.int64), 0, len(mu_seg) - 1)
    return np.ascontiguousarray(np.asarray(mu_seg, dtype=np.float64)[seg])


def uniform_mu_segments(seed: int, count: int = 32, lo: float = 0.1, hi: float = 0.6):
    return np.random.default_rng(seed).uniform(lo, hi, size=count)


def pick_tracers(n_particles: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_particles, size=count, replace=False)).astype(np.int32)


def random_state(cfg: SimConfig, n_particles: int, seed: int, vscale: float = 0.1,
                 cscale: float = 1.0, fscale: float = 1e-3, margin: float = 2.0):
    """Random particle state for kernel-level checks: positions uniform in
    the interior (margin cells from each wall), small random v, C, F - I."""
    rng = np.random.default_rng(seed)
    d = cfg.dim
    x = np.empty((d, n_particles))
    for a in range(d):
        lo = margin * cfg.dx
        hi = cfg.n[a] * cfg.dx - margin * cfg.dx
        x[a] = rng.uniform(lo, hi, size=n_particles)
    v = rng.normal(0.0, vscale, size=(d, n_particles))
    C = rng.normal(0.0, cscale, size=(d * d, n_particles))
    G = rng.normal(0.0, fscale, size=(d * d, n_particles))
    return x, v, C, G


# ---------------------------------------------------------------------------
# Inverse problems: seeded hidden fields and observation layouts
# ---------------------------------------------------------------------------

def granular_block_2d(seed: int = 0):
    """Learned initial velocity: a 0.4 x 0.2 m Drucker-Prager block (friction
    angle 35 deg, E = 1e7, nu = 0.3, rho = 2000) resting on the floor of a
    0.8 x 0.4 m domain at 256 x 128 cells (dx = 1/320 m), x in [0.2, 0.6],
    2 x 2 particles per cell (32,768 particles), floor Coulomb mu = 0.5,
    other walls slip, dt = 1e-5 s."""
    n = (256, 128, 1)
    dx = 1.0 / 320.0
    cfg = SimConfig(dim=2, n=n, dx=dx, dt=1e-5, material=SAND, ppc=4, gravity=(0.0, -9.81, 0.0),
                    wall_mode=(SLIP, SLIP, COULOMB, SLIP, SLIP, SLIP), wall_mu=(0.0, 0.0, 0.5, 0.0, 0.0, 0.0),
                    rho0=2000.0, youngs=1.0e7, poisson=0.3, phi_deg=35.0)
    lo, hi = (0.2, 0.0), (0.6, 0.2)
    x = lattice_particles(cfg, box_inside(lo, hi), lo, hi, seed)
    return cfg, x, np.array(lo), np.array(hi)


def gaussian_bumps(seed: int, lo, hi, count: int = 4):
    """Hidden velocity field: sum of `count` Gaussian bumps with centres
    uniform in the block, widths uniform in [0.02, 0.06] m, directions uniform
    and magnitudes uniform in [0.3, 1.0] m/s.  Returns the bump parameters."""
    rng = np.random.default_rng(seed)
    c = np.stack([rng.uniform(lo[a], hi[a], count) for a in range(2)], axis=1)
    sig = rng.uniform(0.02, 0.06, count)
    ang = rng.uniform(0.0, 2 * np.pi, count)
    mag = rng.uniform(0.3, 1.0, count)
    amp = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=1)
    return c, sig, amp


def eval_bumps(bumps, x):
    """v0(x) = sum_k a_k exp(-|x - c_k|^2 / (2 s_k^2)); x: (2, N)."""
    c, sig, amp = bumps
    v = np.zeros((2, x.shape[1]))
    for k in range(len(sig)):
        r2 = (x[0] - c[k, 0]) ** 2 + (x[1] - c[k, 1]) ** 2
        v += amp[k][:, None] * np.exp(-r2 / (2 * sig[k] ** 2))[None, :]
    return v


def block_boxes(lo, hi, nx: int = 4, ny: int = 2, half: float = 0.02):
    """Eulerian monitor boxes: squares of half-side `half` centred on the
    block's nx x ny sub-cells.  Returns (box_lo, box_hi), each (nx*ny, 2)."""
    cx = lo[0] + (np.arange(nx) + 0.5) * (hi[0] - lo[0]) / nx
    cy = lo[1] + (np.arange(ny) + 0.5) * (hi[1] - lo[1]) / ny
    C = np.array([[x, y] for y in cy for x in cx])
    return C - half, C + half


def dam_break_3d(scale_div: int = 1, seed: int = 0):
    """Learned base friction: 3-D dam-break on 192 x 96 x 64 cells
    (dx = 0.01 m), water column 0.6 x 0.96 x 0.4 m at 8 particles per cell
    (1,843,200 particles), Tait fluid as the 2-D dam-break, gravity -z,
    friction per floor node, dt = 5e-5 s.  scale_div shrinks every length
    by that factor at the same dx."""
    s = scale_div
    n = (192 // s, 96 // s, 64 // s)
    dx = 0.01
    cfg = SimConfig(dim=3, n=n, dx=dx, dt=5e-5, material=FLUID, ppc=8, gravity=(0.0, 0.0, -9.81),
                    wall_mode=(SLIP, SLIP, SLIP, SLIP, COULOMB, SLIP), rho0=1000.0, bulk=1.0e5, gamma=7.0)
    hi = (0.6 / s, 0.96 / s, 0.4 / s)
    x = lattice_particles(cfg, box_inside((0, 0, 0), hi), (0, 0, 0), hi, seed)
    return cfg, x


def dam_break_columns_3d(scale_div: int = 1, seed: int = 0):
    """3-D dam-break against two rigid square columns (Sec. 4.2.1):
    domain 1.0 x 0.5 x 0.4 m at dx = 0.005 m (200 x 100 x 80 cells), water
    column L0 x W0 x H0 = 0.3 x 0.5 x 0.2 m at 8 particles per cell
    (1,920,000 particles), weakly compressible Newtonian fluid with
    mu = 1.01e-3 Pa s and sound speed 35 m/s (Tait, gamma 7, K = rho c^2),
    gravity -z, slip walls, dt = 4e-5 s (0.28 of the acoustic limit dx/c).
    The columns have sides 0.04 and 0.06 m, stand on the floor through the
    domain's height, and are centred at (0.5, 0.3) and (0.6, 0.1) m.
    scale_div shrinks every length by that factor at the same dx."""
    s = scale_div
    n = (200 // s, 100 // s, 80 // s)
    dx = 0.005
    c = 35.0
    zt = n[2] * dx
    cols = []
    for (cx, cy), side in (((0.5, 0.3), 0.04), ((0.6, 0.1), 0.06)):
        r = 0.5 * side / s
        cols.append(((cx / s - r, cy / s - r, 0.0), (cx / s + r, cy / s + r, zt)))
    cfg = SimConfig(dim=3, n=n, dx=dx, dt=4e-5, material=FLUID, ppc=8, gravity=(0.0, 0.0, -9.81),
                    rho0=1000.0, bulk=1000.0 * c * c, gamma=7.0, viscosity=1.01e-3, obstacles=tuple(cols))
    hi = (0.3 / s, 0.5 / s, 0.2 / s)
    x = lattice_particles(cfg, box_inside((0, 0, 0), hi), (0, 0, 0), hi, seed)
    return cfg, x


def floor_node_coords(cfg: SimConfig) -> np.ndarray:
    """Positions (x, y) of the floor nodes in the order of the per-node
    friction array (x fastest), shape (2, n_floor)."""
    nd = cfg.node_dims()
    xs = (np.arange(nd[0]) - cfg.ghost) * cfg.dx
    ys = (np.arange(nd[1]) - cfg.ghost) * cfg.dx
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X.reshape(-1), Y.reshape(-1)])


def sinusoid_friction(cfg: SimConfig, seed: int) -> np.ndarray:
    """Hidden base friction mu(x, y) = 0.3 + 0.2 sin(2 pi x / L) cos(2 pi y / W)
    plus N(0, 0.02^2) per floor node, clipped to [0, 1]."""
    L, Wd = cfg.n[0] * cfg.dx, cfg.n[1] * cfg.dx
    xy = floor_node_coords(cfg)
    mu = 0.3 + 0.2 * np.sin(2 * np.pi * xy[0] / L) * np.cos(2 * np.pi * xy[1] / Wd)
    mu = mu + np.random.default_rng(seed).normal(0.0, 0.02, size=mu.shape)
    return np.clip(mu, 0.0, 1.0)


def mlp_init_params(widths, seed: int) -> np.ndarray:
    """Seeded starting parameters of a dense network in the library's layout
    (per layer: W row-major [out][in], then b), each uniform in
    +-1/sqrt(fan_in).  FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(widths[:-1], widths[1:]):
        r = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-r, r, size=o * i))
        parts.append(rng.uniform(-r, r, size=o))
    return np.concatenate(parts).astype(np.float32)



# ---------------------------------------------------------------------------
# The paper's own inverse experiments (Sec. 5), synthetic reproductions
# ---------------------------------------------------------------------------

def inverse_dam_break_2d(seed: int = 0, fine: bool = False):
    """Dam-break of the initial-velocity inverse problems (Sec. 5.1, 5.2):
    water column H0 = L0 = 0.5 m at 2 x 2 particles per cell, inviscid
    fluid with the numerical sound speed c0 = 50 m/s (the linear EOS:
    gamma = 1, K = rho0 c0^2), dt = 3e-5 s, slip walls, in the domain of the
    paper's table, 1.5 x 0.6 m: 150 x 60 cells at dx = 0.01 m (10,000
    particles), or with fine=True 300 x 120 cells at dx = 0.005 m (40,000
    particles, the table's second size).  With the ground-truth initial
    velocity of Sec. 5.1 (alpha = 2) the front is at 1.37 m at t = 0.3 s,
    short of the far wall.  Returns (cfg, x, H0)."""
    c0, rho0 = 50.0, 1000.0
    n, dx = ((300, 120, 1), 0.005) if fine else ((150, 60, 1), 0.01)
    cfg = SimConfig(dim=2, n=n, dx=dx, dt=3e-5, material=FLUID, ppc=4,
                    gravity=(0.0, -9.8, 0.0), rho0=rho0, bulk=rho0 * c0 * c0, gamma=1.0)
    H0 = L0 = 0.5
    x = lattice_particles(cfg, box_inside((0.0, 0.0), (L0, H0)), (0.0, 0.0), (L0, H0), seed)
    return cfg, x, H0


def velocity_monitors_2d(half: float = 0.01):
    """The nine Eulerian monitors of Sec. 5.1: squares of half-side 0.01 m
    centred on {0.2, 0.3, 0.4} x {0.1, 0.2, 0.3} m.  Returns (lo, hi)."""
    C = np.array([[cx, cy] for cy in (0.1, 0.2, 0.3) for cx in (0.2, 0.3, 0.4)])
    return C - half, C + half


def velocity_profile(y, H0: float = 0.5):
    """The hidden initial horizontal velocity of Sec. 5.2:
    v_x(y) = 2 (1 - (y/H0)^2) + 0.2 sin(4 pi y / H0)."""
    y = np.asarray(y, dtype=np.float64)
    return 2.0 * (1.0 - (y / H0) ** 2) + 0.2 * np.sin(4.0 * np.pi * y / H0)


def friction_segments_2d(seed: int = 0):
    """Dam-break of the segmented-friction inverse problem (Sec. 5.3):
    domain L = 1.6 m x H = 0.4 m at dx = 0.01 m (160 x 40 cells), water
    column L0 = 0.5 m x H0 = 0.3 m at 2 x 2 particles per cell (6,000
    particles, the count of the paper's table), dt = 4e-5 s, the floor in
    four equal Coulomb segments, the other walls slip.  The sound speed is
    not given for this problem; it takes the 50 m/s of Sec. 5.1.  Returns
    (cfg, x, segment length)."""
    c0, rho0 = 50.0, 1000.0
    cfg = SimConfig(dim=2, n=(160, 40, 1), dx=0.01, dt=4e-5, material=FLUID, ppc=4,
                    gravity=(0.0, -9.8, 0.0), rho0=rho0, bulk=rho0 * c0 * c0, gamma=1.0,
                    wall_mode=(SLIP, SLIP, COULOMB, SLIP, SLIP, SLIP))
    x = lattice_particles(cfg, box_inside((0.0, 0.0), (0.5, 0.3)), (0.0, 0.0), (0.5, 0.3), seed)
    return cfg, x, 0.4


FRICTION_SEGMENTS_TRUE = (0.0, 0.5, 0.1, 0.2)     # Sec. 5.3 ground truth

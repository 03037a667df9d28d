"""Parity of the step's other forms against the oracle, through the C-ABI:
the PIC, TPIC, FLIP and blended FLIP/PIC transfers (Sec. 2.2 G2P; App. B),
the viscous fluid (Sec. 2.3 eq:stress_strain), the hypoelastic
Drucker-Prager material with the Jaumann rate and tension cutoff (Sec. 2.3
eq:dp_stress; App. A) and resting rigid obstacles (Sec. 4.2.1).

Bounds as for the APIC step: relative L2 <= 1e-10 (binary64) and <= 1e-4
(binary32 against the binary64 oracle on the same rounded inputs) on
positions (as displacements) and velocities after 10 steps; the other
state fields to 1e-8 / 5e-3.
"""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W
from tests.helpers import displacement_error, gpu_fields, gpu_solver, oracle_fields, oracle_state, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}
TOLF = {"f64": 1e-8, "f32": 5e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _moving_velocity(cfg, x, frac=0.05, div=0.0):
    """A smooth sheared and rotating field moving about `frac` of a cell per
    step, so that ten steps move particles far beyond binary32 rounding;
    div > 0 adds a stretching part along x (expansion where cos(4 pi x/L) >
    0, compression elsewhere)."""
    a = frac * cfg.dx / cfg.dt
    L = cfg.n[0] * cfg.dx
    v = np.empty_like(x)
    v[0] = a * (0.8 + 0.4 * np.sin(2 * np.pi * x[1] / L) + div * np.sin(4 * np.pi * x[0] / L))
    v[1] = a * 0.5 * np.cos(2 * np.pi * x[0] / L)
    if x.shape[0] == 3:
        v[2] = a * 0.3 * np.sin(2 * np.pi * (x[0] + x[1]) / L)
    return v


def _rounded(precision, *arrays):
    if precision != "f32":
        return arrays
    return tuple(None if a is None else np.asarray(a).astype(np.float32).astype(np.float64) for a in arrays)


def _run_pair(orc, cfg, precision, x, v, steps=10, fields=("C", "stress"), floor_mu=None):
    """Runs the oracle and the GPU for `steps` steps from the same rounded
    inputs and checks positions, displacements, velocities and `fields`."""
    x, v = _rounded(precision, x, v)
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v)
    s = gpu_solver(cfg, precision, x, v=v, floor_mu=floor_mu)
    o.run(st, steps, cfg.dt, floor_mu)
    s.mpm_step(steps)
    rc, bad = s.mpm_sync_status()
    assert rc == 0, (rc, bad)
    g = gpu_fields(s)
    r = oracle_fields(cfg, st)
    s.close()
    ex, ev = rel_l2(g["x"], r["x"]), rel_l2(g["v"], r["v"])
    ed, tol_d = displacement_error(g["x"], r["x"], x, steps, precision)
    print(f"  rel L2 x={ex:.3e} v={ev:.3e} displacement={ed:.3e} (bound {tol_d:.2e})", flush=True)
    assert ex <= TOL[precision] and ev <= TOL[precision] and ed <= tol_d
    extra = list(fields) + ["Jm1" if "Jm1" in r else "FmI"]
    for f in extra:
        e = rel_l2(g[f], r[f])
        print(f"  rel L2 {f}={e:.3e}", flush=True)
        assert e <= TOLF[precision], f
    return g, r, st


# ---------------------------------------------------------------------------
# Transfers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("transfer,alpha", [("pic", 1.0), ("tpic", 1.0), ("flip", 1.0), ("flip", 0.95)])
def test_transfer_dam_break(orc, precision, transfer, alpha):
    cfg, x = W.dam_break_2d()
    cfg = cfg.replace(transfer=transfer, flip_alpha=alpha)
    print(f"[case] {transfer} alpha={alpha} dam-break {precision} N={x.shape[1]}", flush=True)
    g, r, _ = _run_pair(orc, cfg, precision, x, _moving_velocity(cfg, x))
    if transfer in ("pic", "flip"):
        assert not g["C"].any()          # no affine part is carried


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("transfer,alpha", [("tpic", 1.0), ("flip", 1.0), ("flip", 0.9)])
def test_transfer_sand_3d(orc, precision, transfer, alpha):
    cfg, x = W.cylinder_collapse_3d(scale_div=8, seed=0)
    cfg = cfg.replace(transfer=transfer, flip_alpha=alpha)
    print(f"[case] {transfer} alpha={alpha} small cylinder {precision} N={x.shape[1]}", flush=True)
    _run_pair(orc, cfg, precision, x, _moving_velocity(cfg, x))


def test_flip_keeps_particle_velocities_without_forces(orc):
    """FLIP with no gravity and no stress gradient (a uniform translation
    of a fluid at rest density): each particle keeps its own velocity, also
    where the grid velocity is a smoothed average of different ones (the
    grid increment is zero); PIC returns the smoothed value."""
    cfg, x = W.dam_break_2d()
    cfg = cfg.replace(gravity=(0.0, 0.0, 0.0), transfer="flip", flip_alpha=1.0)
    rng = np.random.default_rng(41)
    v = 0.5 + rng.normal(0.0, 0.05, size=x.shape)
    s = gpu_solver(cfg, "f64", x, v=v)
    s.mpm_step(1)
    assert s.mpm_sync_status()[0] == 0
    vg = s.mpm_read_state("v", "pid").cpu().numpy()
    s.close()
    # pressure stays zero (J = 1 + O(dt div v)); the particles away from the
    # walls keep v to the size of one step's force
    inner = (x[0] > 0.05) & (x[0] < 0.45) & (x[1] > 0.05) & (x[1] < 0.95)
    assert np.abs(vg[:, inner] - v[:, inner]).max() < 5e-3
    cfg_p = cfg.replace(transfer="pic")
    s = gpu_solver(cfg_p, "f64", x, v=v)
    s.mpm_step(1)
    vp = s.mpm_read_state("v", "pid").cpu().numpy()
    s.close()
    assert np.abs(vp[:, inner] - v[:, inner]).max() > 2e-2     # PIC smooths the noise away


# ---------------------------------------------------------------------------
# Viscous fluid
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_fluid(orc, precision, dim):
    """A viscosity large enough that the viscous stress is of the size of
    the pressure (50 Pa s against a sheared flow of ~100 1/s)."""
    if dim == 2:
        cfg, x = W.dam_break_2d()
    else:
        cfg, x = W.dam_break_3d(scale_div=8, seed=0)
    cfg = cfg.replace(viscosity=50.0)
    print(f"[case] viscous fluid {dim}-D {precision} N={x.shape[1]}", flush=True)
    g, r, _ = _run_pair(orc, cfg, precision, x, _moving_velocity(cfg, x))
    # the viscous shear stress is there, of the size V0 2 mu gdot_xy with the
    # field's shear-rate amplitude gdot_xy = a (2 pi / L)(0.4 + 0.5) / 2
    d = cfg.dim
    S = g["stress"].reshape(d, d, -1)
    a = 0.05 * cfg.dx / cfg.dt
    gdot = a * (2 * np.pi / (cfg.n[0] * cfg.dx)) * 0.45
    expect = cfg.vol0 * 2 * cfg.viscosity * gdot
    off = np.abs(S[0, 1]).max()
    print(f"  largest shear stress {off:.3e} (V0 2 mu gdot = {expect:.3e})", flush=True)
    assert 0.3 * expect < off < 3 * expect


# ---------------------------------------------------------------------------
# Hypoelastic Drucker-Prager (Jaumann rate, tension cutoff)
# ---------------------------------------------------------------------------

def _zone_counts(orc, cfg, st, dt):
    """Zones of App. A that the oracle's next stress update takes, per
    particle (the velocity gradient from the oracle's own P2G/grid/G2P)."""
    o = orc.Oracle(cfg)
    s2 = st.copy()
    gm, gp = o.p2g(s2, dt)
    gv = o.grid_update(gm, gp, dt)
    L = o.g2p(s2, gv, dt)
    d = cfg.dim
    counts = np.zeros(4, dtype=np.int64)
    for p in range(s2.N):
        sig = s2.S[:, p].reshape(d, d) / (cfg.vol0 * s2.J[p])
        _, zone, _ = o.dp_jaumann(L[:, p].reshape(d, d), sig, dt)
        counts[zone] += 1
    return counts


DIV = {"block2d": 1.0, "cylinder3d": 1.0}


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["block2d", "cylinder3d"])
def test_dp_jaumann_moving(orc, precision, case):
    """A sheared, rotating and partly diverging start velocity: the 10 steps
    take every zone of App. A (elastic, shear return, tension cutoff)."""
    if case == "block2d":
        cfg, x, _, _ = W.granular_block_2d(seed=0)
    else:
        cfg, x = W.cylinder_collapse_3d(scale_div=8, seed=0)
    cfg = cfg.replace(material=W.DP_JAUMANN, psi_deg=5.0)
    print(f"[case] dp_jaumann {case} {precision} N={x.shape[1]}", flush=True)
    v = _moving_velocity(cfg, x, frac=0.02, div=DIV[case])
    zones = _zone_counts(orc, cfg, oracle_state(orc, cfg, *_rounded(precision, x, v)), cfg.dt)
    g, r, st = _run_pair(orc, cfg, precision, x, v)
    zones += _zone_counts(orc, cfg, st, cfg.dt)
    print(f"  zones of the first and the next update (I, II, III): {zones[1:]}", flush=True)
    assert (zones[1:] > 0).all()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dp_jaumann_random_stress_one_step(orc, precision):
    """Random prestress over the three zones (mean stress of either sign,
    deviators below and above the cone), random velocities and affine
    matrices, with cohesion and a negative cutoff: one step."""
    cfg = W.SimConfig(dim=3, n=(20, 16, 12), dx=0.01, dt=1e-5, material=W.DP_JAUMANN, ppc=8,
                      gravity=(0, 0, -9.81), youngs=1e6, rho0=1500.0, phi_deg=30.0, psi_deg=10.0,
                      cohesion=200.0, tension=-50.0,
                      wall_mode=(W.SLIP, W.STICK, W.SLIP, W.SLIP, W.COULOMB, W.SLIP),
                      wall_mu=(0, 0, 0, 0, 0.4, 0))
    N = 5003
    x, v, C, _ = W.random_state(cfg, N, 32, vscale=0.5, cscale=5.0, margin=0.0)
    rng = np.random.default_rng(35)
    sig = rng.normal(0, 1, size=(3, 3, N))
    sig = 0.5 * (sig + sig.transpose(1, 0, 2)) * rng.uniform(0, 3e3, size=N)
    sig += np.eye(3)[:, :, None] * rng.uniform(-3e3, 1e3, size=N)
    Jm1 = rng.normal(0, 1e-3, size=N)
    S = (sig * (cfg.vol0 * (1.0 + Jm1))).reshape(9, N)
    x, v, C, S, Jm1 = _rounded(precision, x, v, C, S, Jm1)
    print(f"[case] dp_jaumann random prestress {precision} N={N}", flush=True)
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v, C=C, S=S, Jm1=Jm1)
    zones = _zone_counts(orc, cfg, st, cfg.dt)
    print(f"  zones (I, II, III): {zones[1:]}", flush=True)
    assert (zones[1:] > 50).all()
    s = gpu_solver(cfg, precision, x, v=v, C=C, S=S, Jm1=Jm1)
    o.step(st, cfg.dt)
    s.mpm_step(1)
    assert s.mpm_sync_status()[0] == 0
    g = gpu_fields(s)
    r = oracle_fields(cfg, st)
    s.close()
    tol = 1e-12 if precision == "f64" else 2e-5
    for f in g:
        e = rel_l2(g[f], r[f])
        print(f"  {f}: {e:.3e}", flush=True)
        assert e <= (tol if f in ("x", "v", "C") else tol * 100), f


# ---------------------------------------------------------------------------
# Resting rigid obstacles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_obstacle_dam_break_2d(orc, precision):
    """A box standing on the floor just downstream of the water column, the
    column pushed into it.  The box faces sit between node planes (no
    position ties between the precisions)."""
    cfg, x = W.dam_break_2d()
    h = cfg.dx
    cfg = cfg.replace(obstacles=(((32.37 * h, 0.0), (40.41 * h, 20.29 * h)),))
    print(f"[case] obstacle dam-break {precision}", flush=True)
    v = _moving_velocity(cfg, x)
    g, r, _ = _run_pair(orc, cfg, precision, x, v)
    # the obstacle holds the water back: no particle got more than a cell inside
    lo, hi = cfg.obstacles[0]
    inside = (g["x"][0] > lo[0] + h) & (g["x"][1] < hi[1] - h)
    assert not inside.any()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_obstacles_dam_break_3d(orc, precision):
    """The 3-D dam-break with two rigid columns downstream (Sec. 4.2.1), at
    1/8 scale, the water pushed towards them."""
    cfg, x = W.dam_break_3d(scale_div=8, seed=0)
    h = cfg.dx
    zt = cfg.n[2] * h
    cols = (((8.53 * h, 2.47 * h, 0.0), (10.47 * h, 4.53 * h, zt)),
            ((8.53 * h, 7.47 * h, 0.0), (10.47 * h, 9.53 * h, zt)))
    cfg = cfg.replace(obstacles=cols)
    print(f"[case] two columns, 3-D dam-break {precision} N={x.shape[1]}", flush=True)
    v = _moving_velocity(cfg, x, frac=0.05)
    v[0] = np.abs(v[0]) + 0.05 * cfg.dx / cfg.dt
    _run_pair(orc, cfg, precision, x, v, steps=20)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dam_break_columns_paper_geometry(orc, precision):
    """The paper's 3-D dam-break against two square columns (Sec. 4.2.1)
    with its viscous fluid, at 1/4 scale (30,000 particles), the water
    pushed towards the columns at a quarter cell per step so that its front
    (9 cells away) meets them: 50 steps against the oracle, and no particle
    more than a cell inside the wider column (3 cells across at this scale;
    the oracle puts 39 particles there without the obstacles)."""
    cfg, x = W.dam_break_columns_3d(scale_div=4, seed=0)
    h = cfg.dx
    print(f"[case] paper's columns, 3-D dam-break / 4, viscous, {precision} N={x.shape[1]}", flush=True)
    v = _moving_velocity(cfg, x, frac=0.05)
    v[0] = np.abs(v[0]) + 0.25 * h / cfg.dt
    g, _, _ = _run_pair(orc, cfg, precision, x, v, steps=50)
    assert g["x"][0].max() > cfg.obstacles[0][0][0]       # the front has reached the first column
    lo, hi = cfg.obstacles[1]
    deep = np.ones(g["x"].shape[1], dtype=bool)
    for a in range(2):
        deep &= (g["x"][a] > lo[a] + h) & (g["x"][a] < hi[a] - h)
    assert not deep.any()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["cylinder", "column"])
def test_paper_granular_timing_cases(orc, precision, case):
    """The paper's two granular timing cases (Sec. 4.2.2-4.2.3: hypoelastic
    Drucker-Prager sand on a no-slip base, dt = 1e-5 s) at 1/8 scale: the
    cylinder on 50 x 50 x 12 cells and the column of aspect ratio 3 on
    50 x 32 x 25, from a sheared, rotating and partly diverging velocity so
    that the 10 steps leave the elastic zone and reach the base."""
    if case == "cylinder":
        cfg, x = W.cylinder_paper_grid(scale_div=8, seed=0)
    else:
        cfg, x = W.granular_column_paper(scale_div=8, seed=0)
    assert cfg.material == W.DP_JAUMANN and cfg.wall_mode[4] == W.STICK
    print(f"[case] paper's {case} / 8, dp_jaumann, {precision} N={x.shape[1]}", flush=True)
    v = _moving_velocity(cfg, x, frac=0.02, div=1.0)
    zones = _zone_counts(orc, cfg, oracle_state(orc, cfg, *_rounded(precision, x, v)), cfg.dt)
    _run_pair(orc, cfg, precision, x, v)
    print(f"  zones of the first update (I, II, III): {zones[1:]}", flush=True)
    assert zones[2] > 0

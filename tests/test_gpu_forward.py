"""Forward-step parity: the HIP solver against the oracle on identical seeded
inputs, through the C-ABI.

Integers (cell keys, sort permutation) must match bit for bit; floating
point must meet the stated bounds: relative L2 <= 1e-10 (binary64) and
<= 1e-4 (binary32 against the binary64 oracle) on positions and velocities
after 10 steps.
"""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W
from tests.helpers import displacement_error, gpu_fields, gpu_solver, oracle_fields, oracle_state, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _np(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[gpu] {torch.cuda.get_device_name(0)}", flush=True)


def _small_3d(scale_div=8):
    return W.cylinder_collapse_3d(scale_div=scale_div, seed=0)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["dam2d", "sand3d"])
def test_keys_and_sort_bit_exact(orc, precision, case):
    cfg, x = W.dam_break_2d() if case == "dam2d" else _small_3d()
    print(f"[case] keys/sort {case} {precision} N={x.shape[1]}", flush=True)
    o = orc.Oracle(cfg, key_f32=(precision == "f32"))
    s = gpu_solver(cfg, precision, x)
    xg = _np(s.mpm_read_state("x")).astype(np.float64)       # positions as the GPU holds them
    key0 = _np(s.read_keys())
    assert np.array_equal(key0, o.keys(xg))
    for step in range(3):
        xb = _np(s.mpm_read_state("x")).astype(np.float64)
        kb = _np(s.read_keys())
        assert np.array_equal(kb, o.keys(xb)), f"keys differ before step {step}"
        s.mpm_step(1)
        perm, _ = s.mpm_read_sort()
        assert np.array_equal(_np(perm), o.sort_perm(kb)), f"perm differs at step {step}"
    rc, _ = s.mpm_sync_status()
    assert rc == 0


def _moving_velocity(cfg, x):
    """A smooth sheared and rotating field whose speed is about 5 % of a cell
    per step (7 m/s in the dam-break, 12 m/s in the small cylinder), so that
    ten steps move particles by ~0.5 cells: the displacement is then far
    above the rounding of binary32 positions."""
    a = 0.05 * cfg.dx / cfg.dt
    L = cfg.n[0] * cfg.dx
    v = np.empty_like(x)
    v[0] = a * (0.8 + 0.4 * np.sin(2 * np.pi * x[1] / L))
    v[1] = a * 0.5 * np.cos(2 * np.pi * x[0] / L)
    if x.shape[0] == 3:
        v[2] = a * 0.3 * np.sin(2 * np.pi * (x[0] + x[1]) / L)
    return v


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["dam2d", "sand3d", "dam2d_moving", "sand3d_moving"])
def test_ten_steps_match_oracle(orc, precision, case):
    cfg, x = W.dam_break_2d() if case.startswith("dam2d") else _small_3d()
    print(f"[case] 10 steps {case} {precision} N={x.shape[1]}", flush=True)
    o = orc.Oracle(cfg)
    xin = x.astype(np.float32).astype(np.float64) if precision == "f32" else x
    v0 = None
    if case.endswith("moving"):
        v0 = _moving_velocity(cfg, xin)
        if precision == "f32":
            v0 = v0.astype(np.float32).astype(np.float64)
    st = oracle_state(orc, cfg, xin, v=v0)
    s = gpu_solver(cfg, precision, xin, v=v0)
    o.run(st, 10, cfg.dt)
    s.mpm_step(10)
    rc, bad = s.mpm_sync_status()
    assert rc == 0, bad
    g = gpu_fields(s)
    r = oracle_fields(cfg, st)
    ex, ev = rel_l2(g["x"], r["x"]), rel_l2(g["v"], r["v"])
    ed, tol_d = displacement_error(g["x"], r["x"], xin, 10, precision)
    print(f"  rel L2 x={ex:.3e} v={ev:.3e} displacement={ed:.3e} (bound {tol_d:.2e})", flush=True)
    assert ex <= TOL[precision]
    assert ev <= TOL[precision]
    assert ed <= tol_d
    if case.endswith("moving"):
        assert tol_d < 3 * TOL[precision]      # the rounding floor is small here
    # the other state fields to the same order of accuracy
    tolf = 1e-8 if precision == "f64" else 5e-3
    for f in ("C", "stress", "Jm1" if cfg.material == W.FLUID else "FmI"):
        e = rel_l2(g[f], r[f])
        print(f"  rel L2 {f}={e:.3e}", flush=True)
        assert e <= tolf, f
    if precision == "f64":
        # memory order matches too: both sides sort the same way every step
        assert np.array_equal(_np(s.mpm_read_state("pid"))[0], st.pid)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_grid_fields_after_one_step(orc, precision):
    cfg, x = W.dam_break_2d()
    print(f"[case] grid fields {precision}", flush=True)
    rng = np.random.default_rng(31)
    v = rng.normal(0, 0.3, size=x.shape)
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v)
    _, _, gm, gv = o.step(st, cfg.dt, want_grid=True)
    s = gpu_solver(cfg, precision, x, v=v, keep_grid=True)
    s.mpm_step(1)
    m_gpu = _np(s.mpm_read_grid("mass"))[0].astype(np.float64)
    v_gpu = _np(s.mpm_read_grid("vel")).astype(np.float64)
    tol = 1e-12 if precision == "f64" else 1e-6
    assert rel_l2(m_gpu, gm) <= tol
    assert rel_l2(v_gpu, gv) <= (1e-11 if precision == "f64" else 1e-5)
    # nodes the particles never reach stay exactly empty on both sides
    assert np.array_equal(m_gpu == 0, gm == 0)


def test_grid_read_after_many_steps(orc):
    """The grid read back after 60 steps of the dam-break (the column has
    collapsed, so tiles that held particles earlier are empty now): nodal
    mass and velocity equal the oracle's, and nodes without mass read as
    exactly empty on both sides (the grid kernel writes only the active
    tiles' nodes; the read masks the rest)."""
    cfg, x = W.dam_break_2d()
    print("[case] grid read after 60 steps", flush=True)
    rng = np.random.default_rng(37)
    v = np.stack([rng.uniform(2.0, 3.0, x.shape[1]), rng.uniform(-0.5, 0.5, x.shape[1])])
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v)
    o.run(st, 59, cfg.dt)
    _, _, gm, gv = o.step(st, cfg.dt, want_grid=True)
    s = gpu_solver(cfg, "f64", x, v=v, keep_grid=True)
    s.mpm_step(60)
    assert s.mpm_sync_status()[0] == 0
    m_gpu = _np(s.mpm_read_grid("mass"))[0]
    v_gpu = _np(s.mpm_read_grid("vel"))
    assert rel_l2(m_gpu, gm) <= 1e-10
    assert rel_l2(v_gpu, gv) <= 1e-10
    assert np.array_equal(m_gpu == 0, gm == 0)
    assert not v_gpu[:, m_gpu == 0].any()
    # the run moved the column: nodes it covered at the start are empty now
    m0 = np.zeros_like(gm)
    o0 = orc.Oracle(cfg)
    _, _, m0, _ = o0.step(oracle_state(orc, cfg, x, v=v), cfg.dt, want_grid=True)
    assert ((m0 > 0) & (gm == 0)).sum() > 50


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("material", [W.SAND, W.ELASTIC, W.FLUID])
@pytest.mark.parametrize("fscale", [2e-3, 3e-2])
def test_random_state_one_step(orc, precision, material, fscale):
    """Random x, v, C, F and stress cache: one step exercises every branch of
    the return mapping (apex, elastic, cone) and every stencil position.  At
    the small strain scale the kernel's series form of the Hencky return
    serves most particles; at the large one the eigen-decomposition does."""
    if material == W.FLUID and fscale != 2e-3:
        pytest.skip("the fluid carries no deformation gradient")
    cfg = W.SimConfig(dim=3, n=(20, 16, 12), dx=0.01, dt=1e-5, material=material, ppc=8,
                      gravity=(0, 0, -9.81), youngs=1e6, rho0=1500.0,
                      wall_mode=(W.SLIP, W.STICK, W.SLIP, W.SLIP, W.COULOMB, W.SLIP),
                      wall_mu=(0, 0, 0, 0, 0.4, 0))
    N = 5003       # ragged: not a multiple of the workgroup size
    print(f"[case] random state {material} {precision} N={N} fscale={fscale}", flush=True)
    x, v, C, G = W.random_state(cfg, N, 32, vscale=0.5, cscale=5.0, fscale=fscale, margin=0.0)
    rng = np.random.default_rng(33)
    S = rng.normal(0, 1e-3, size=(3, 3, N))
    S = (S + S.transpose(1, 0, 2)).reshape(9, N)
    if material == W.FLUID:
        S = np.repeat(np.eye(3).reshape(9, 1), N, axis=1) * rng.normal(0, 1e-3, size=N)
        Jm1 = rng.normal(0, 1e-3, size=N)
        G = None
    else:
        Jm1 = None
    if precision == "f32":
        x, v, C, S = (a.astype(np.float32).astype(np.float64) for a in (x, v, C, S))
        G = None if G is None else G.astype(np.float32).astype(np.float64)
        Jm1 = None if Jm1 is None else Jm1.astype(np.float32).astype(np.float64)
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v, C=C, G=G, S=S, Jm1=Jm1)
    s = gpu_solver(cfg, precision, x, v=v, C=C, G=G, S=S, Jm1=Jm1)
    o.step(st, cfg.dt)
    s.mpm_step(1)
    assert s.mpm_sync_status()[0] == 0
    g = gpu_fields(s)
    r = oracle_fields(cfg, st)
    tol = 1e-12 if precision == "f64" else 2e-5
    for f in g:
        e = rel_l2(g[f], r[f])
        print(f"  {f}: {e:.3e}", flush=True)
        assert e <= (tol if f in ("x", "v", "C") else tol * 100), f


def test_floor_friction_field(orc):
    cfg, x = W.friction_dam_break_2d(scale=1)
    print("[case] per-node floor friction", flush=True)
    mu = W.segment_mu(cfg, W.uniform_mu_segments(2))
    rng = np.random.default_rng(34)
    v = np.stack([rng.uniform(0.5, 1.5, x.shape[1]), rng.uniform(-1.0, 0.0, x.shape[1])])
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v)
    s = gpu_solver(cfg, "f64", x, v=v, floor_mu=mu)
    o.run(st, 5, cfg.dt, floor_mu=mu)
    s.mpm_step(5)
    g, r = gpu_fields(s), oracle_fields(cfg, st)
    assert rel_l2(g["v"], r["v"]) <= 1e-10
    assert rel_l2(g["x"], r["x"]) <= 1e-10


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,cells", [(3000, 8), (900, 2)])
def test_crowded_tile_uses_global_sort(orc, N, cells, precision):
    """One tile holding more particles than the in-LDS sort takes (1024:
    the sort runs in global memory), or fewer but with more than 64 per
    cell (ranks past the 64-entry rank table)."""
    cfg = W.SimConfig(dim=2, n=(32, 32, 1), dx=0.01, dt=1e-5, material=W.FLUID, ppc=4,
                      gravity=(0, -9.81, 0))
    rng = np.random.default_rng(35)
    # inside cells [10, 10 + cells) of the tile whose base + ghost is in [8, 16)
    lo = (8 - 2 + 0.5) * cfg.dx + 1e-6
    hi = (8 + cells - 2 + 0.5) * cfg.dx - 1e-6
    x = rng.uniform(lo, hi, size=(2, N))
    if precision == "f32":
        x = x.astype(np.float32).astype(np.float64)
    print(f"[case] crowded tile N={N} over {cells}x{cells} cells {precision}", flush=True)
    o = orc.Oracle(cfg, key_f32=(precision == "f32"))
    st = oracle_state(orc, cfg, x)
    s = gpu_solver(cfg, precision, x)
    kb = _np(s.read_keys())
    assert len(np.unique(kb >> 6)) == 1
    o.step(st, cfg.dt)
    s.mpm_step(1)
    assert s.mpm_sync_status()[0] == 0
    perm, _ = s.mpm_read_sort()
    assert np.array_equal(_np(perm), o.sort_perm(kb))
    g, r = gpu_fields(s), oracle_fields(cfg, st)
    assert rel_l2(g["x"], r["x"]) <= (1e-12 if precision == "f64" else 2e-5)
    assert rel_l2(g["v"], r["v"]) <= (1e-10 if precision == "f64" else 1e-4)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N", [1023, 1024, 1025])
def test_tile_at_sort_capacity(orc, precision, N):
    """A tile with one particle fewer than, exactly as many as, and one more
    than the in-LDS sort takes (1024: 16 entries per lane of the one-wave
    sort; above it the sort runs in global memory), 16 particles per cell
    over the 64 cells of a 2-D tile: the GPU's order must equal the oracle's
    ordering of the GPU's own keys, and the step must match the oracle."""
    cfg = W.SimConfig(dim=2, n=(32, 32, 1), dx=0.01, dt=1e-5, material=W.FLUID, ppc=4,
                      gravity=(0, -9.81, 0))
    rng = np.random.default_rng(36 + N)
    lo = (8 - 2 + 0.5) * cfg.dx + 1e-6
    hi = (8 + 8 - 2 + 0.5) * cfg.dx - 1e-6
    x = rng.uniform(lo, hi, size=(2, N))
    if precision == "f32":
        x = x.astype(np.float32).astype(np.float64)
    print(f"[case] tile at sort capacity N={N} {precision}", flush=True)
    o = orc.Oracle(cfg, key_f32=(precision == "f32"))
    s = gpu_solver(cfg, precision, x)
    kb = _np(s.read_keys())
    assert len(np.unique(kb >> 6)) == 1
    assert np.array_equal(kb, o.keys(_np(s.mpm_read_state("x")).astype(np.float64)))
    st = oracle_state(orc, cfg, x)
    o.step(st, cfg.dt)
    s.mpm_step(1)
    assert s.mpm_sync_status()[0] == 0
    perm, _ = s.mpm_read_sort()
    assert np.array_equal(_np(perm), o.sort_perm(kb))
    g, r = gpu_fields(s), oracle_fields(cfg, st)
    tol = 1e-12 if precision == "f64" else 2e-5
    assert rel_l2(g["x"], r["x"]) <= tol
    assert rel_l2(g["v"], r["v"]) <= (1e-10 if precision == "f64" else 1e-4)


def test_walls_and_clamping(orc):
    """Particles on the walls and moving out of the box are clamped the same
    way on both sides."""
    cfg = W.SimConfig(dim=2, n=(24, 24, 1), dx=0.01, dt=2e-4, material=W.FLUID, ppc=4,
                      gravity=(0, -9.81, 0),
                      wall_mode=(W.SLIP, W.STICK, W.COULOMB, W.SLIP, W.SLIP, W.SLIP),
                      wall_mu=(0, 0, 0.3, 0, 0, 0))
    rng = np.random.default_rng(36)
    N = 777
    x = rng.uniform(0, 0.24, size=(2, N))
    x[:, :40] = 0.0
    x[0, 40:80] = 0.24
    v = rng.normal(0, 2.0, size=(2, N))
    print("[case] walls and clamping", flush=True)
    o = orc.Oracle(cfg)
    st = oracle_state(orc, cfg, x, v=v)
    s = gpu_solver(cfg, "f64", x, v=v)
    o.run(st, 4, cfg.dt)
    s.mpm_step(4)
    assert s.mpm_sync_status()[0] == 0
    g, r = gpu_fields(s), oracle_fields(cfg, st)
    assert np.isfinite(r["x"]).all()
    # some particles were pushed against the walls and held there
    ext = cfg.n[0] * cfg.dx
    assert (g["x"] == 0.0).any() and (g["x"][0] == ext).any()
    assert rel_l2(g["x"], r["x"]) <= 1e-10
    assert rel_l2(g["v"], r["v"]) <= 1e-10
    assert g["x"].min() >= 0.0 and g["x"].max() <= ext


def test_empty_and_nan(orc):
    import torch
    cfg, x = W.dam_break_2d()
    s = gpu_solver(cfg, "f64", x[:, :0], capacity=16)
    s.mpm_step(3)
    assert s.mpm_sync_status()[0] == 0
    # non-finite state is latched and reported with the particle id
    s = gpu_solver(cfg, "f64", x)
    v = s.mpm_read_state("v", "pid")
    v[0, 123] = float("nan")
    s.mpm_write_state("v", v, "pid")
    s.mpm_step(1)
    rc, bad = s.mpm_sync_status()
    assert rc == -4
    # the NaN spreads through the grid to the particles sharing its nodes;
    # the latch reports the smallest of their ids
    vn = _np(s.mpm_read_state("v", "pid"))
    nan_ids = np.where(~np.isfinite(vn).all(axis=0))[0]
    assert 123 in nan_ids and bad == nan_ids.min()
    assert s.mpm_sync_status()[0] == 0      # latch cleared


def test_cfl_violation_is_reported():
    """A step in which particles move more than one cell is latched as
    EDOMAIN with the smallest such particle id; a normal step is not."""
    cfg, x = W.dam_break_2d()
    s = gpu_solver(cfg, "f64", x)
    s.mpm_step(2)
    assert s.mpm_sync_status()[0] == 0
    v = s.mpm_read_state("v", "pid")
    v[0, :] = 2.5 * cfg.dx / cfg.dt
    s.mpm_write_state("v", v, "pid")
    s.mpm_step(1)
    rc, bad = s.mpm_sync_status()
    assert rc == -5
    vn = _np(s.mpm_read_state("v", "pid"))
    fast = np.where((np.abs(vn) * cfg.dt > cfg.dx).any(axis=0))[0]
    assert len(fast) > 0 and bad == fast.min()
    assert s.mpm_sync_status()[0] == 0      # latch cleared


def test_read_write_round_trip(orc):
    cfg, x = _small_3d()
    s = gpu_solver(cfg, "f64", x)
    s.mpm_step(2)
    pid = _np(s.mpm_read_state("pid"))[0]
    xm = _np(s.mpm_read_state("x", "memory"))
    xp = _np(s.mpm_read_state("x", "pid"))
    assert np.array_equal(xp[:, pid], xm)
    F = _np(s.mpm_read_state("F", "pid"))
    G = _np(s.mpm_read_state("FmI", "pid"))
    eye = np.eye(3).reshape(9, 1)
    assert np.allclose(F, G + eye, atol=1e-15)
    s.mpm_write_state("FmI", G * 2, "pid")
    assert np.array_equal(_np(s.mpm_read_state("FmI", "pid")), G * 2)
    with pytest.raises(Exception):
        s.mpm_read_state("J")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_step_is_deterministic(orc, precision):
    """No floating-point atomics anywhere in the step: two runs from the same
    input agree bit for bit."""
    cfg, x = _small_3d()
    out = []
    for _ in range(2):
        s = gpu_solver(cfg, precision, x)
        s.mpm_step(5)
        out.append({f: _np(s.mpm_read_state(f, "memory")) for f in ("x", "v", "C", "FmI", "stress", "pid")})
    for f in out[0]:
        assert np.array_equal(out[0][f], out[1][f]), f


@pytest.mark.parametrize("case", ["cylinder", "dambreak3d", "cylinder_jaumann", "columns", "paper_cylinder",
                                  "paper_column"])
def test_full_size_steps_match_oracle(orc, case):
    """Full-size workloads in the launch configuration the bench times: the
    3-D cylinder collapse (2,780,928 particles, Drucker-Prager sand with the
    Hencky return, and with the hypoelastic material of App. A), the 3-D
    dam-break of the friction problem (1,843,200 particles, fluid) and the
    3-D dam-break against two columns (1,920,000 particles, viscous fluid,
    Sec. 4.2.1), and the paper's two granular timing cases on its own grids
    (Sec. 4.2.2-4.2.3: the cylinder on 400 x 400 x 100, 2,713,580
    particles; the column on 400 x 32 x 200, 2,408,448).  Ten steps in
    binary64 and binary32 against one oracle run from the same
    binary32-rounded input, whole arrays compared (positions,
    displacements, velocities)."""
    from paper_2507_04192_amd.native import Solver
    if case == "paper_cylinder":
        cfg, x = W.cylinder_paper_grid()
    elif case == "paper_column":
        cfg, x = W.granular_column_paper()
    elif case.startswith("cylinder"):
        cfg, x = W.cylinder_collapse_3d(scale_div=1, seed=0)
        if case == "cylinder_jaumann":
            cfg = cfg.replace(material=W.DP_JAUMANN)
    else:
        cfg, x = W.dam_break_3d() if case == "dambreak3d" else W.dam_break_columns_3d()
    x = x.astype(np.float32).astype(np.float64)
    N = x.shape[1]
    steps = 10
    print(f"[case] full size {case} N={N}, {steps} steps (oracle first)", flush=True)
    o = orc.Oracle(cfg)
    st = orc.State(cfg, x)
    o.run(st, steps, cfg.dt)
    xr, vr = st.by_pid("x"), st.by_pid("v")
    for precision in ("f64", "f32"):
        s = Solver(cfg, precision, capacity=N)
        s.mpm_init_particles(x)
        s.mpm_step(steps)
        rc, bad = s.mpm_sync_status()
        assert rc == 0, bad
        xg = s.mpm_read_state("x", "pid").cpu().numpy()
        vg = s.mpm_read_state("v", "pid").cpu().numpy()
        s.close()
        ex, ev = rel_l2(xg, xr), rel_l2(vg, vr)
        ed, tol_d = displacement_error(xg, xr, x, steps, precision)
        print(f"  {precision}: rel L2 x={ex:.3e} v={ev:.3e} displacement={ed:.3e} (bound {tol_d:.2e})", flush=True)
        assert ex <= TOL[precision] and ev <= TOL[precision]
        assert ed <= tol_d

"""Pins of the oracle's grid-to-particle transfers (Sec. 2.2 G2P; App. B)
against what the transfers fix independently of the oracle's code:

- FLIP adds only the grid's velocity increment, so without forces it
  returns every particle's own velocity, however rough the field; PIC
  replaces it by the interpolated grid velocity; the blend is the weighted
  sum of the two (Zhu & Bridson's blend, cited in Sec. 2.2);
- in free fall every transfer gives v = g t and x = x0 + g dt^2 n(n+1)/2;
- with internal stress and no walls or gravity every transfer conserves
  linear momentum (internal forces sum to zero);
- the quadratic B-spline quasi-interpolant differentiates quadratic
  fields exactly (sum_i f(x_i) grad phi_i = grad f for f of degree 2) and
  shifts their values by the second moment h^2/4, so TPIC's affine matrix
  equals the field's gradient and every transfer's velocity equals
  f + (h^2/8) lap f;
- one particle alone: APIC and TPIC keep its affine matrix (D_p^{-1} D_p
  = I; sum_i d_i grad phi_i^T = I), PIC and FLIP drop it.

Each test names the mistake it catches.
"""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W


def _block_cfg(transfer, alpha=1.0, dim=2, g=0.0, bulk=1e-12):
    n = (32, 32, 1) if dim == 2 else (16, 16, 16)
    grav = (0.0, g, 0.0) if dim == 2 else (0.0, 0.0, g)
    return W.SimConfig(dim=dim, n=n, dx=1.0 / n[0], dt=1e-3, material=W.FLUID, ppc=4 if dim == 2 else 8,
                       gravity=grav, bulk=bulk, rho0=1000.0, gamma=1.0, transfer=transfer, flip_alpha=alpha)


def _block(cfg, seed=3):
    lo = tuple(0.3 for _ in range(cfg.dim))
    hi = tuple(0.7 for _ in range(cfg.dim))
    return W.lattice_particles(cfg, W.box_inside(lo, hi), lo, hi, seed=seed)


def _rough_velocity(x, seed, amp=1e-3):
    return np.random.default_rng(seed).uniform(-amp, amp, size=x.shape)


@pytest.mark.parametrize("dim", [2, 3])
def test_flip_without_forces_keeps_particle_velocity(orc, dim):
    """No stress (bulk modulus 1e-12), no gravity, walls out of reach, a
    rough particle velocity field: FLIP (alpha = 1) returns each particle's
    velocity to rounding, PIC smooths it away, and the blend with alpha =
    0.3 is 0.3 v + 0.7 v_PIC.  Catches: a wrong sign of the increment, the
    increment formed from the momentum with the force or with v^n taken
    after the update, the blend weight ignored or swapped."""
    res = {}
    for xf, a in (("flip", 1.0), ("pic", 1.0), ("flip", 0.3)):
        cfg = _block_cfg(xf, a, dim=dim)
        x = _block(cfg)
        v0 = _rough_velocity(x, 5)
        st = orc.State(cfg, x, v=v0)
        orc.Oracle(cfg).step(st, cfg.dt)
        res[(xf, a)] = st.by_pid("v")
        if xf in ("flip", "pic"):
            assert np.abs(st.C).max() == 0.0        # no affine part carried
    v_flip, v_pic, v_blend = res[("flip", 1.0)], res[("pic", 1.0)], res[("flip", 0.3)]
    assert np.abs(v_flip - v0).max() <= 1e-15 * 1e3 * np.abs(v0).max()
    assert np.linalg.norm(v_pic - v0) > 0.3 * np.linalg.norm(v0)       # PIC dissipates the noise
    assert np.abs(v_blend - (0.3 * v0 + 0.7 * v_pic)).max() <= 1e-12 * np.abs(v0).max()


@pytest.mark.parametrize("transfer", ["pic", "flip", "tpic", "apic"])
def test_free_fall_every_transfer(orc, transfer):
    """Gravity only: v^n = n dt g exactly and x^n = x0 + g dt^2 n(n+1)/2.
    Catches: FLIP's increment missing the gravity of the step (v^n formed
    after gravity), a transfer that moves particles with the old velocity."""
    cfg = _block_cfg(transfer, dim=2, g=-9.81)
    x = _block(cfg)
    st = orc.State(cfg, x)
    o = orc.Oracle(cfg)
    n = 12
    for _ in range(n):
        o.step(st, cfg.dt)
    v, xn = st.by_pid("v"), st.by_pid("x")
    assert np.abs(v[0]).max() < 1e-14
    assert np.abs(v[1] - n * cfg.dt * -9.81).max() < 1e-13
    want = x[1] + -9.81 * cfg.dt ** 2 * n * (n + 1) / 2
    assert np.abs(xn[1] - want).max() < 1e-13


@pytest.mark.parametrize("transfer", ["pic", "flip", "tpic", "apic"])
def test_internal_forces_keep_linear_momentum(orc, transfer):
    """Random symmetric particle stresses and velocities, no gravity, walls
    out of reach: the total momentum sum m_p v_p is unchanged by a step of
    each transfer.  Catches: FLIP's grid increment taken without the force
    on one side only, a force that leaks into v^n."""
    cfg = _block_cfg(transfer, dim=3, bulk=1e3)
    x = _block(cfg, seed=8)
    N = x.shape[1]
    rng = np.random.default_rng(9)
    v0 = rng.normal(0.0, 0.01, size=(3, N))
    A = rng.normal(0.0, 1.0, size=(3, 3, N))
    S = (A + A.transpose(1, 0, 2)).reshape(9, N) * 1e-6
    st = orc.State(cfg, x, v=v0, S=S)
    p0 = (cfg.mass * v0).sum(axis=1)
    orc.Oracle(cfg).step(st, cfg.dt)
    p1 = (cfg.mass * st.v).sum(axis=1)
    scale = cfg.mass * np.abs(v0).sum()
    assert np.abs(p1 - p0).max() <= 1e-13 * scale
    # the forces did act on individual particles
    st2 = orc.State(cfg, x, v=v0)
    orc.Oracle(cfg).step(st2, cfg.dt)
    assert np.abs(st.by_pid("v") - st2.by_pid("v")).max() > 1e-9


def _node_xy(cfg, o):
    """Coordinates of every node of the dense padded grid, (dim, NN)."""
    dims = o.dims
    idx = np.arange(o.NN)
    I = [idx % dims[0], (idx // dims[0]) % dims[1], idx // (dims[0] * dims[1])]
    return np.stack([(I[a] - cfg.ghost) * cfg.dx for a in range(cfg.dim)])


@pytest.mark.parametrize("transfer", ["tpic", "apic", "pic"])
def test_quadratic_grid_field_is_differentiated_exactly(orc, transfer):
    """G2P from the grid field v_x = 0.3 y^2 + 0.2 x y, v_y = -0.1 x^2 + 0.5 y:
    every transfer's particle velocity is f + (h^2/8) lap f (the
    quasi-interpolant's second-moment shift), TPIC's affine matrix is the
    exact gradient [[0.2 y, 0.6 y + 0.2 x], [-0.2 x, 0.5]], PIC's is zero and
    APIC's differs from the gradient (its third-moment term).  Catches:
    TPIC storing the APIC moment (or the transpose of the gradient), PIC
    keeping an affine part."""
    cfg = _block_cfg(transfer, dim=2)
    o = orc.Oracle(cfg)
    xy = _node_xy(cfg, o)
    X, Y = xy
    gv = np.stack([0.3 * Y ** 2 + 0.2 * X * Y, -0.1 * X ** 2 + 0.5 * Y])
    rng = np.random.default_rng(21)
    xp = rng.uniform(0.2, 0.8, size=(2, 200))
    st = orc.State(cfg, xp)
    o.g2p(st, gv, 0.0)
    px, py = xp
    h2 = cfg.dx ** 2
    vx = 0.3 * (py ** 2 + h2 / 4) + 0.2 * px * py
    vy = -0.1 * (px ** 2 + h2 / 4) + 0.5 * py
    assert np.abs(st.v[0] - vx).max() < 1e-14 and np.abs(st.v[1] - vy).max() < 1e-14
    grad = np.stack([0.2 * py, 0.6 * py + 0.2 * px, -0.2 * px, 0.5 * np.ones_like(px)])
    if transfer == "tpic":
        assert np.abs(st.C - grad).max() < 1e-12
    elif transfer == "pic":
        assert np.abs(st.C).max() == 0.0
    else:
        assert np.abs(st.C - grad).max() > 1e-6


@pytest.mark.parametrize("transfer,keeps", [("apic", True), ("tpic", True), ("pic", False), ("flip", False)])
def test_single_particle_affine_matrix(orc, transfer, keeps):
    """One particle with v and an affine matrix C, no forces: the grid field
    it makes is v + C (x_i - x_p) on its stencil; G2P gives back v, and C
    for APIC (D^{-1} D = I) and TPIC (sum_i d_i grad phi_i^T = I), zero for
    PIC and FLIP.  Catches: a wrong D^{-1}, the affine term dropped from
    P2G, FLIP or PIC keeping C."""
    cfg = _block_cfg(transfer, dim=3)
    xp = np.array([[0.4312], [0.5077], [0.4861]])
    v = np.array([[0.01], [-0.02], [0.005]])
    C = np.array([[0.3, -0.1, 0.2, 0.05, -0.4, 0.1, 0.0, 0.2, -0.3]]).T
    st = orc.State(cfg, xp, v=v, C=C)
    orc.Oracle(cfg).step(st, cfg.dt)
    assert np.abs(st.v - v).max() < 1e-15
    if keeps:
        assert np.abs(st.C - C).max() < 1e-13
    else:
        assert np.abs(st.C).max() == 0.0

"""Pins of the oracle's kinematics, fluid stress and observation operators
against what the mechanics fixes independently of the oracle's code:

- an affine velocity field moves every particle by one map M, so the
  deformation gradient must compose with it (F_n = M F_0) and the volume
  ratio must be its determinant (J_n = det M J_0) -- M is fitted from the
  positions alone (Sec. 2.2 G2P; Sec. 2.3 density update read as
  J' = J det(I + dt grad v));
- a fluid held at a uniform pre-compression J0 carries sound at
  c^2 = dp/drho = K J0^(1-gamma)/rho0, so the fundamental mode of a closed
  box has period 2L/c (textbook acoustics) -- this fixes the Kirchhoff
  stress tau = -J p I (dropping J changes c by 15 % at J0 = 0.8);
- the Lagrangian and Eulerian operators and the masked loss of
  eq:inverse_loss (Sec. 3.2) in states whose values are known in closed
  form: free fall, and uniform translation.

Each test names the mistake it catches.
"""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W


def _fit_affine(x0, xn):
    """Least-squares M, c with xn = M x0 + c (columns are particles)."""
    d, N = x0.shape
    A = np.vstack([x0, np.ones((1, N))]).T
    sol, *_ = np.linalg.lstsq(A, xn.T, rcond=None)
    M = sol[:d].T
    c = sol[d]
    res = np.abs(A @ sol - xn.T).max()
    return M, c, res


@pytest.mark.parametrize("material", [W.ELASTIC, W.FLUID])
def test_affine_flow_deformation_follows_motion(orc, material):
    """v = A x + b with C = A imposed at each step (APIC then carries the
    affine field to the grid and back exactly) and a negligible stiffness:
    after n steps the particles' positions are an
    affine image x_n = M x_0 + c of the start, and F_n = M F_0 (elastic) or
    J_n = det(M) J_0 (fluid) for every particle.  A is a shear plus a spin
    and F_0 a stretch that does not commute with it.  Catches: F (I + dt L)
    in place of (I + dt L) F, L transposed, a linearised or otherwise wrong
    J update (1 + tr in place of det)."""
    cfg = W.SimConfig(dim=3, n=(24, 24, 24), dx=1.0 / 24, dt=2e-3, material=material, ppc=8,
                      gravity=(0.0, 0.0, 0.0), youngs=1e-9, bulk=1e-9, rho0=1000.0)
    lo, hi = (0.3, 0.3, 0.3), (0.7, 0.7, 0.7)
    x0 = W.lattice_particles(cfg, W.box_inside(lo, hi), lo, hi, seed=11)
    N = x0.shape[1]
    A = np.array([[0.3, 0.8, 0.0], [-0.5, 0.1, 0.4], [0.2, -0.3, -0.2]])
    b = np.array([0.05, -0.02, 0.01])
    v = A @ x0 + b[:, None]
    C = np.repeat(A.reshape(9, 1), N, axis=1)
    rng = np.random.default_rng(12)
    F0 = np.array([[1.2, 0.1, 0.0], [0.1, 0.9, 0.05], [0.0, 0.05, 1.1]])
    J0 = 1.0 + rng.uniform(-0.05, 0.05, size=N)
    st = orc.State(cfg, x0, v=v, C=C, F=np.repeat(F0.reshape(9, 1), N, axis=1), J=J0)
    o = orc.Oracle(cfg)
    steps = 25
    for _ in range(steps):
        # the prescribed motion: the affine field is imposed at the start of
        # every step (APIC stores v at the old position, so a free affine
        # field does not stay exactly affine near the body's edge)
        st.v[:] = A @ st.x + b[:, None]
        st.C[:] = A.reshape(9, 1)
        o.step(st, cfg.dt)
    xn = st.by_pid("x")
    M, _, res = _fit_affine(x0, xn)
    assert res < 1e-12
    # the map is the flow of the field: (I + dt A)^n, not I
    assert np.abs(M - np.linalg.matrix_power(np.eye(3) + cfg.dt * A, steps)).max() < 1e-12
    assert np.abs(M - np.eye(3)).max() > 0.01
    if material == W.ELASTIC:
        Fn = st.by_pid("F").reshape(3, 3, N)
        want = M @ F0
        err = np.abs(Fn - want[:, :, None]).max()
        assert err < 1e-11, err
        # the two orders differ by far more than the tolerance
        assert np.abs(F0 @ M - want).max() > 1e-3
    else:
        Jn = st.by_pid("J")
        err = np.abs(Jn - np.linalg.det(M) * J0).max()
        assert err < 1e-12, err
        lin = np.prod([1 + cfg.dt * np.trace(A)] * steps)
        assert abs(lin - np.linalg.det(M)) > 1e-6


def _acoustic_box(orc, J0, gamma=7.0, K=1e5, L=1.0, ncell=64, wide=4, v0=0.01):
    """A closed box [0, L] x [0, wide h] filled with fluid at the uniform
    compression J0 (current particle volume h^2/4, so V0 = h^2/(4 J0)), its
    static pressure balanced by the slip walls, and the fundamental
    standing wave v_x = v0 sin(pi x/L) superposed.  Returns the measured
    period of the mode amplitude and the textbook one 2L/c with
    c^2 = dp/drho at rho0/J0 = K J0^(1-gamma)/rho0."""
    h = L / ncell
    cfg = W.SimConfig(dim=2, n=(ncell, wide, 1), dx=h, dt=1e-4, material=W.FLUID, ppc=4,
                      gravity=(0.0, 0.0, 0.0), rho0=1000.0, bulk=K, gamma=gamma)
    x = W.lattice_particles(cfg, W.box_inside((0, 0), (L, wide * h)), (0, 0), (L, wide * h), seed=0, jitter=0.0)
    N = x.shape[1]
    o = orc.Oracle(cfg)
    vol0 = h * h / 4 / J0
    o.c.vol0 = vol0
    o.c.mass = cfg.rho0 * vol0
    p0 = (K / gamma) * (J0 ** -gamma - 1.0)
    S = np.zeros((4, N))
    S[0] = S[3] = -vol0 * J0 * p0          # the static state: tau = -J p I
    v = np.zeros((2, N))
    v[0] = v0 * np.sin(np.pi * x[0] / L)
    st = orc.State(cfg, x, v=v, J=np.full(N, J0), S=S)
    c = np.sqrt(K * J0 ** (1.0 - gamma) / cfg.rho0)
    T = 2.0 * L / c
    steps = int(1.2 * T / cfg.dt)
    amp = np.empty(steps)
    for n in range(steps):
        o.step(st, cfg.dt)
        w = np.sin(np.pi * st.x[0] / L)
        amp[n] = (st.v[0] * w).sum() / (w * w).sum()
    t = (np.arange(steps) + 1) * cfg.dt
    zc = [t[i - 1] + cfg.dt * amp[i - 1] / (amp[i - 1] - amp[i])
          for i in range(1, steps) if (amp[i - 1] > 0) != (amp[i] > 0)]
    return 2.0 * (zc[1] - zc[0]), T, amp


@pytest.mark.parametrize("J0", [0.8, 1.0])
def test_precompressed_fluid_sound_speed(orc, J0):
    """Period of the fundamental mode of a closed box within 2 % of 2L/c,
    c^2 = K J0^(1-gamma)/rho0.  At J0 = 0.8 a Kirchhoff stress without the
    factor J (tau = -p I) gives c^2 = (K J0^-gamma + p)/rho0, a 15 % shorter
    period; the EOS derivative itself is pinned in test_eos_closed_form."""
    per, T, amp = _acoustic_box(orc, J0)
    assert abs(per / T - 1.0) < 0.02, (per, T)
    # small amplitude, no growth
    assert np.abs(amp).max() < 0.0102


# ---------------------------------------------------------------------------
# Observation operators and the loss (Sec. 3.2, eq:inverse_loss)
# ---------------------------------------------------------------------------

def _free_fall_cfg():
    return W.SimConfig(dim=2, n=(32, 64, 1), dx=1.0 / 64, dt=1e-3, material=W.FLUID, ppc=4,
                       gravity=(0.0, -9.81, 0.0), bulk=1e-6)


def test_lagrangian_operator_free_fall(orc):
    """Tracers in free fall, observed after several sorted steps (memory order
    is no longer pid order): Q_l is the closed form x0 + g dt^2 n(n+1)/2 of
    particle tracer_pid[l], and the loss against targets offset by known
    vectors d_l is sum m_l |d_l|^2, with seed -2 m_l d_l on that particle.
    Catches: tracers read by slot instead of pid, a dropped mask, a wrong
    sign or factor in the seed."""
    cfg = _free_fall_cfg()
    x0 = W.lattice_particles(cfg, W.box_inside((0.1, 0.6), (0.4, 0.9)), (0.1, 0.6), (0.4, 0.9), seed=13)
    N = x0.shape[1]
    tr = W.pick_tracers(N, 37, 14)
    rng = np.random.default_rng(15)
    frames = [3, 7, 10]
    off = rng.normal(0, 0.01, size=(len(frames), 2, len(tr)))
    mask = (rng.uniform(size=(len(frames), len(tr))) < 0.7).astype(float)
    g = np.array(cfg.gravity[:2])
    closed = [x0[:, tr] + g[:, None] * cfg.dt ** 2 * f * (f + 1) / 2 for f in frames]
    tgt = np.stack([closed[i] - off[i] for i in range(len(frames))])
    obs = orc.Observations(frames, tr, "x", tgt, lag_mask=mask)
    o = orc.Oracle(cfg)
    st = orc.State(cfg, x0)
    done = 0
    for fi, f in enumerate(frames):
        o.run(st, f - done, cfg.dt)
        done = f
        assert not np.array_equal(st.pid, np.arange(N))
        lag, eul, _ = orc.observe(st, obs, fi)
        assert eul is None
        assert np.abs(lag - closed[fi]).max() < 1e-12
        loss, gx, gv = orc.frame_loss_and_seed(st, obs, fi)
        assert abs(loss - (mask[fi] * (off[fi] ** 2).sum(axis=0)).sum()) < 1e-12
        assert not gv.any()
        want = np.zeros((2, N))
        want[:, tr] = 2.0 * mask[fi] * off[fi]
        gx_pid = np.empty_like(gx)
        gx_pid[:, st.pid] = gx
        assert np.abs(gx_pid - want).max() < 1e-12


def test_eulerian_operator_uniform_translation(orc):
    """Uniform translation v = u (no gravity, negligible pressure): every box
    mean of v is u exactly, every box count is the number of lattice points
    x0 + u t inside [lo, hi) (brute force), and an empty box contributes
    nothing.  The seed of box l is 2 m_l (Q_l - z_l)/|P_l| on each member.
    Catches: a closed box [lo, hi], a sum in place of a mean, a count that
    includes the wrong particles."""
    cfg = W.SimConfig(dim=2, n=(64, 32, 1), dx=1.0 / 64, dt=1e-3, material=W.FLUID, ppc=4,
                      gravity=(0.0, 0.0, 0.0), bulk=1e-9)
    lo, hi = (0.2, 0.1), (0.6, 0.3)
    x0 = W.lattice_particles(cfg, W.box_inside(lo, hi), lo, hi, seed=16)
    N = x0.shape[1]
    u = np.array([0.7, -0.2])
    v = np.repeat(u[:, None], N, axis=1)
    box_lo = np.array([[0.25, 0.12], [0.4, 0.2], [0.55, 0.25], [0.9, 0.4]])
    box_hi = box_lo + np.array([[0.05, 0.05], [0.08, 0.03], [0.1, 0.1], [0.02, 0.02]])
    frames = [4, 9]
    tgt = np.random.default_rng(17).normal(0, 0.1, size=(2, 2, 4))
    obs = orc.Observations(frames, box_lo=box_lo, box_hi=box_hi, eul_field="v", eul_target=tgt)
    o = orc.Oracle(cfg)
    st = orc.State(cfg, x0, v=v, C=np.zeros((4, N)))
    done = 0
    for fi, f in enumerate(frames):
        o.run(st, f - done, cfg.dt)
        done = f
        xs = x0 + u[:, None] * cfg.dt * f
        assert np.abs(st.by_pid("x") - xs).max() < 1e-12
        _, eul, cnt = orc.observe(st, obs, fi)
        for b in range(4):
            inside = np.all((xs >= box_lo[b][:, None]) & (xs < box_hi[b][:, None]), axis=0)
            assert cnt[b] == inside.sum()
            if cnt[b]:
                assert np.abs(eul[:, b] - u).max() < 1e-12
            else:
                assert not eul[:, b].any()
        assert cnt[3] == 0 and cnt[:3].min() > 0
        loss, gx, gv = orc.frame_loss_and_seed(st, obs, fi)
        r = u[:, None] - tgt[fi][:, :3]
        assert abs(loss - (r ** 2).sum()) < 1e-12
        assert not gx.any()
        want = np.zeros((2, N))
        xs_mem = st.x
        for b in range(3):
            inside = np.all((xs_mem >= box_lo[b][:, None]) & (xs_mem < box_hi[b][:, None]), axis=0)
            want[:, inside] += (2.0 * r[:, b] / cnt[b])[:, None]
        assert np.abs(gv - want).max() < 1e-12

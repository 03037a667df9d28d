"""Gradient parity: the HIP forward-plus-adjoint rollout (checkpoints,
recomputation, hand-written reverse kernels) against the oracle's reverse
sweep on identical seeded inputs, and against central differences of the
HIP forward pass.  Bounds: binary64 relative L2 <= 1e-8, binary32 <= 5e-3
against the binary64 oracle."""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W
from tests.helpers import oracle_state, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _np(t):
    return t.cpu().numpy().astype(np.float64)


def friction_case(scale_steps=60):
    """Small dam-break over a Coulomb floor with 8 friction segments."""
    cfg = W.SimConfig(dim=2, n=(48, 24, 1), dx=1 / 64, dt=1e-4, material=W.FLUID, ppc=4,
                      gravity=(0, -9.81, 0), rho0=1000.0, bulk=1e5, gamma=7.0,
                      wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP))
    x0 = W.lattice_particles(cfg, W.box_inside((0, 0), (0.25, 0.3)), (0, 0), (0.25, 0.3), seed=80)
    N = x0.shape[1]
    rng = np.random.default_rng(81)
    v0 = np.stack([rng.uniform(0.5, 1.0, N), rng.uniform(-0.1, 0.1, N)])
    seg = W.uniform_mu_segments(82, count=8)
    mu = W.segment_mu(cfg, seg, seg_len=0.1)
    tr = W.pick_tracers(N, 32, 83)
    frames = list(range(scale_steps // 4, scale_steps + 1, scale_steps // 4))
    tgt = np.stack([x0[:, tr] + rng.normal(0, 0.01, size=(2, 32)) for _ in frames])
    return cfg, x0, v0, mu, tr, frames, tgt, scale_steps


def run_gpu(cfg, precision, x0, v0, mu, steps, k, obs, tape_segments=0):
    from paper_2507_04192_amd.native import Solver
    s = Solver(cfg, precision, capacity=x0.shape[1], tape_steps=steps, ckpt_every=k, tape_segments=tape_segments)
    s.mpm_init_particles(x0, v0)
    if mu is not None:
        s.mpm_set_floor_mu(mu)
    s.mpm_set_observations(**obs)
    loss = s.mpm_forward_loss(steps)
    gv, gm = s.mpm_backward()
    assert s.mpm_sync_status()[0] == 0
    return loss, _np(gv), (_np(gm) if mu is not None else None), s


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_friction_gradient_matches_oracle(orc, precision):
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case()
    print(f"[case] friction gradient {precision} N={x0.shape[1]} steps={steps}", flush=True)
    if precision == "f32":
        x0 = x0.astype(np.float32).astype(np.float64)
        v0 = v0.astype(np.float32).astype(np.float64)
        mu = mu.astype(np.float32).astype(np.float64)
        tgt = tgt.astype(np.float32).astype(np.float64)
    obs_o = orc.Observations(frames, tr, "x", tgt)
    loss_o, gv_o, gmu_o = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, mu, obs_o)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    loss, gv, gmu, _ = run_gpu(cfg, precision, x0, v0, mu, steps, 16, obs)
    el, ev, em = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o), rel_l2(gmu, gmu_o)
    print(f"  loss {loss:.6e} vs {loss_o:.6e} ({el:.2e}); dL/dv0 {ev:.2e}; dL/dmu {em:.2e}", flush=True)
    tol = 1e-8 if precision == "f64" else 5e-3
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    assert ev <= tol and em <= tol
    assert np.abs(gmu_o).max() > 0
    # nodes no particle reached get an exact zero on both sides
    assert np.array_equal(gmu == 0, gmu_o == 0) if precision == "f64" else True


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_sand_3d_velocity_gradient_matches_oracle(orc, precision):
    cfg, x0 = W.cylinder_collapse_3d(scale_div=8, seed=0)
    N = x0.shape[1]
    rng = np.random.default_rng(84)
    v0 = rng.normal(0, 0.2, size=(3, N))
    if precision == "f32":
        x0 = x0.astype(np.float32).astype(np.float64)
        v0 = v0.astype(np.float32).astype(np.float64)
    steps, k = 12, 5
    tr = W.pick_tracers(N, 40, 85)
    frames = [4, 8, 12]
    tgt = rng.normal(0, 0.1, size=(3, 3, 40)).astype(np.float32).astype(np.float64)
    print(f"[case] 3D sand velocity gradient {precision} N={N}", flush=True)
    obs_o = orc.Observations(frames, tr, "v", tgt)
    loss_o, gv_o, _ = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, None, obs_o)
    loss, gv, _, _ = run_gpu(cfg, precision, x0, v0, None, steps, k,
                             dict(frames=frames, tracer_pid=tr, lag_field="v", lag_target=tgt))
    ev = rel_l2(gv, gv_o)
    print(f"  loss {abs(loss - loss_o) / loss_o:.2e}; dL/dv0 {ev:.2e}", flush=True)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eulerian_boxes_gradient_matches_oracle(orc, precision):
    cfg = W.SimConfig(dim=2, n=(64, 32, 1), dx=1 / 160, dt=1e-5, material=W.SAND, ppc=4,
                      gravity=(0, -9.81, 0), rho0=2000.0, youngs=1e7, poisson=0.3, phi_deg=35.0,
                      wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP),
                      wall_mu=(0, 0, 0.5, 0, 0, 0))
    x0 = W.lattice_particles(cfg, W.box_inside((0.1, 0), (0.3, 0.1)), (0.1, 0), (0.3, 0.1), seed=86)
    N = x0.shape[1]
    rng = np.random.default_rng(87)
    v0 = rng.normal(0, 0.5, size=(2, N))
    if precision == "f32":
        x0 = x0.astype(np.float32).astype(np.float64)
        v0 = v0.astype(np.float32).astype(np.float64)
    lo = np.array([[0.12, 0.0], [0.18, 0.03], [0.24, 0.05], [0.28, 0.0]])
    hi = lo + 0.04
    frames = [5, 10, 15, 20]
    tgt = rng.normal(0, 0.2, size=(4, 2, 4)).astype(np.float32).astype(np.float64)
    tr = W.pick_tracers(N, 20, 88)
    ttg = (x0[:, tr][None] + rng.normal(0, 1e-3, size=(4, 2, 20))).astype(np.float32).astype(np.float64)
    print(f"[case] eulerian boxes {precision} N={N}", flush=True)
    obs_o = orc.Observations(frames, tr, "x", ttg, box_lo=lo, box_hi=hi, eul_field="v", eul_target=tgt)
    loss_o, gv_o, _ = orc.rollout_grad(cfg, x0, v0, 20, cfg.dt, None, obs_o)
    loss, gv, _, _ = run_gpu(cfg, precision, x0, v0, None, 20, 6,
                             dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=ttg,
                                  box_lo=lo, box_hi=hi, eul_field="v", eul_target=tgt))
    el, ev = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o)
    print(f"  loss {el:.2e}; dL/dv0 {ev:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)


def test_checkpoint_interval_does_not_change_gradient(orc):
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case(40)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    ref = None
    for k in (1, 7, 40):
        loss, gv, gmu, _ = run_gpu(cfg, "f64", x0, v0, mu, steps, k, obs)
        if ref is None:
            ref = (loss, gv, gmu)
        else:
            assert loss == ref[0]
            assert rel_l2(gv, ref[1]) <= 1e-12 and rel_l2(gmu, ref[2]) <= 1e-12


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_taped_segments_do_not_change_gradient(orc, precision):
    """Trailing segments kept on the tape (1, 2, 3 of 6, all 6, more than
    there are) instead of recomputed: the same loss bit for bit (the forward
    step is deterministic) and the same gradient up to the order of the
    reverse step's LDS atomics; a second backward recomputes every segment."""
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case(40)
    if precision == "f32":
        x0, v0, mu, tgt = (a.astype(np.float32).astype(np.float64) for a in (x0, v0, mu, tgt))
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    tol = 1e-12 if precision == "f64" else 1e-5
    ref = None
    for ns in (1, 2, 3, 6, 9):
        loss, gv, gmu, s = run_gpu(cfg, precision, x0, v0, mu, steps, 7, obs, tape_segments=ns)
        gv2, gmu2 = s.mpm_backward()
        assert s.mpm_sync_status()[0] == 0
        s.close()
        assert rel_l2(_np(gv2), gv) <= tol and rel_l2(_np(gmu2), gmu) <= tol
        if ref is None:
            ref = (loss, gv, gmu)
        else:
            assert loss == ref[0], ns
            assert rel_l2(gv, ref[1]) <= tol and rel_l2(gmu, ref[2]) <= tol, ns


def test_second_backward_recomputes_every_segment():
    """The forward rollout leaves its last segment on the tape for the first
    backward sweep; a second sweep recomputes it from its checkpoint and
    must give the same gradient, and the state and sort after the rollout
    must be bit for bit those of plain steps."""
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case(40)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    loss, gv, gmu, s = run_gpu(cfg, "f64", x0, v0, mu, steps, 7, obs)
    gv2, gm2 = s.mpm_backward()
    # the reverse kernels sum node adjoints with atomics: equal up to rounding
    assert rel_l2(_np(gv2), gv) <= 1e-12 and rel_l2(_np(gm2), gmu) <= 1e-12
    from paper_2507_04192_amd.native import Solver
    p = Solver(cfg, "f64", capacity=x0.shape[1])
    p.mpm_init_particles(x0, v0)
    p.mpm_set_floor_mu(mu)
    p.mpm_step(steps)
    for f in ("x", "v", "C"):
        assert np.array_equal(_np(s.mpm_read_state(f, "pid")), _np(p.mpm_read_state(f, "pid"))), f
    pa, ka = s.mpm_read_sort()
    pb, kb = p.mpm_read_sort()
    assert np.array_equal(_np(pa), _np(pb)) and np.array_equal(_np(ka), _np(kb))


def test_gradient_against_gpu_finite_differences():
    """Segment friction: dL/dmu_seg from the adjoint against central
    differences of the HIP forward loss (binary64, h = 1e-6)."""
    from paper_2507_04192_amd.native import Solver
    cfg, x0, v0, _, tr, frames, tgt, steps = friction_case(80)
    seg = W.uniform_mu_segments(89, count=8)
    seg_len = 0.1
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    s = Solver(cfg, "f64", capacity=x0.shape[1], tape_steps=steps, ckpt_every=20)

    def loss_at(sv, grad=False):
        s.mpm_init_particles(x0, v0)
        s.mpm_set_floor_mu(W.segment_mu(cfg, sv, seg_len))
        s.mpm_set_observations(**obs)
        L = s.mpm_forward_loss(steps)
        if not grad:
            return L
        return L, _np(s.mpm_backward()[1])

    L0, gnode = loss_at(seg, True)
    nd = cfg.node_dims()
    idx = np.clip(np.floor((np.arange(nd[0]) - cfg.ghost) * cfg.dx / seg_len).astype(int), 0, 7)
    gseg = np.bincount(idx, weights=gnode, minlength=8)
    h = 1e-6
    for kk in range(8):
        e = np.zeros(8)
        e[kk] = h
        fd = (loss_at(seg + e) - loss_at(seg - e)) / (2 * h)
        print(f"  seg {kk}: adjoint {gseg[kk]: .6e}  fd {fd: .6e}", flush=True)
        # central differences carry rounding noise of about eps * L / h
        noise = 100 * np.finfo(float).eps * abs(L0) / h
        assert abs(fd - gseg[kk]) <= 1e-5 * abs(fd) + 1e-6 * np.abs(gseg).max() + noise


def test_backward_needs_forward():
    from paper_2507_04192_amd.native import MPMError, Solver
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case(20)
    s = Solver(cfg, "f64", capacity=x0.shape[1], tape_steps=20, ckpt_every=5)
    s.mpm_init_particles(x0, v0)
    with pytest.raises(MPMError):
        s.mpm_backward()
    s2 = Solver(cfg, "f64", capacity=x0.shape[1])
    s2.mpm_init_particles(x0, v0)
    with pytest.raises(MPMError):
        s2.mpm_forward_loss(10)
    # a plain step after a rollout and its gradient still matches the oracle
    s.mpm_set_floor_mu(mu)
    s.mpm_set_observations(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    s.mpm_forward_loss(steps)
    s.mpm_backward()
    s.mpm_step(3)
    assert s.mpm_sync_status()[0] == 0


def _c2_setup():
    """Friction inverse at full size: dam-break on 256 x 128 cells (32,768
    particles), 32 floor segments of friction drawn from seed 2 (truth) and 3
    (evaluation point), 64 tracers (seed 4) observed every 50 steps."""
    cfg, x0 = W.friction_dam_break_2d(scale=2)
    N = x0.shape[1]
    tr = W.pick_tracers(N, 64, 4)
    mu_true = W.segment_mu(cfg, W.uniform_mu_segments(2))
    mu_eval = W.segment_mu(cfg, W.uniform_mu_segments(3))
    return cfg, x0, tr, mu_true, mu_eval


def _seg_grad(cfg, gnode, nseg=32, seg_len=0.0625):
    nd = cfg.node_dims()
    idx = np.clip(np.floor((np.arange(nd[0]) - cfg.ghost) * cfg.dx / seg_len).astype(int), 0, nseg - 1)
    return np.bincount(idx, weights=gnode, minlength=nseg)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_friction_inverse_full_size_vs_oracle(orc, precision):
    """Full particle count, 100 steps (checkpoint every 50): HIP gradient
    against the oracle's binary64 reverse sweep (binary64 to 1e-8, binary32
    to 5e-3, both from the same rounded inputs).  The column starts sliding
    at 0.5 m/s so that the floor friction acts from the first step."""
    from paper_2507_04192_amd.native import Solver
    cfg, x0, tr, mu_true, mu_eval = _c2_setup()
    steps, frames = 100, [50, 100]
    v0 = np.zeros_like(x0)
    v0[0] = 0.5
    if precision == "f32":
        x0, mu_true, mu_eval = (a.astype(np.float32).astype(np.float64) for a in (x0, mu_true, mu_eval))
    print(f"[case] friction inverse full size {precision} N={x0.shape[1]} steps={steps}", flush=True)
    _, _, qs = orc.rollout(cfg, x0, v0, steps, cfg.dt, mu_true,
                           orc.Observations(frames, tr, "x", np.zeros((2, 2, 64))))
    rng = np.random.default_rng(90)
    tgt = np.stack([q[0] for q in qs]) + rng.normal(0, 1e-3, size=(2, 2, 64))
    if precision == "f32":
        tgt = tgt.astype(np.float32).astype(np.float64)
    obs_o = orc.Observations(frames, tr, "x", tgt)
    loss_o, gv_o, gmu_o = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, mu_eval, obs_o)
    s = Solver(cfg, precision, capacity=x0.shape[1], tape_steps=steps, ckpt_every=50)
    s.mpm_init_particles(x0, v0)
    s.mpm_set_floor_mu(mu_eval)
    s.mpm_set_observations(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    loss = s.mpm_forward_loss(steps)
    gv, gmu = s.mpm_backward()
    gv, gmu = _np(gv), _np(gmu)
    print(f"  loss {loss:.4e}: {abs(loss - loss_o) / loss_o:.2e}; dL/dv0 {rel_l2(gv, gv_o):.2e}; "
          f"dL/dmu {rel_l2(gmu, gmu_o):.2e}", flush=True)
    tol = 1e-8 if precision == "f64" else 5e-3
    assert abs(loss - loss_o) <= (1e-10 if precision == "f64" else 1e-4) * loss_o
    assert rel_l2(gv, gv_o) <= tol
    assert rel_l2(gmu, gmu_o) <= tol
    assert np.abs(gmu_o).max() > 0
    # the flow has not reached the far segments: their gradient is exactly 0
    assert _seg_grad(cfg, gmu)[-1] == 0.0 and _seg_grad(cfg, gmu_o)[-1] == 0.0


def test_friction_inverse_full_size_finite_differences():
    """The benchmark's friction inverse as specified: 500 steps, checkpoint
    every 50, 10 frames; every segment's gradient against central
    differences of the HIP forward loss (binary64, h = 1e-6)."""
    from paper_2507_04192_amd.native import Solver
    cfg, x0, tr, mu_true, mu_eval = _c2_setup()
    steps, frames = 500, list(range(50, 501, 50))
    seg_eval = W.uniform_mu_segments(3)
    print(f"[case] friction inverse FD N={x0.shape[1]} steps={steps}", flush=True)
    s = Solver(cfg, "f64", capacity=x0.shape[1], tape_steps=steps, ckpt_every=50)
    # targets: the same solver run with the true friction
    s.mpm_init_particles(x0)
    s.mpm_set_floor_mu(mu_true)
    tgt = []
    for f in range(len(frames)):
        s.mpm_step(50)
        tgt.append(_np(s.mpm_read_state("x", "pid"))[:, tr])
    tgt = np.stack(tgt)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)

    def loss_at(seg, grad=False):
        s.mpm_init_particles(x0)
        s.mpm_set_floor_mu(W.segment_mu(cfg, seg))
        s.mpm_set_observations(**obs)
        L = s.mpm_forward_loss(steps)
        return (L, _np(s.mpm_backward()[1])) if grad else L

    L0, gnode = loss_at(seg_eval, True)
    gs = _seg_grad(cfg, gnode)
    h = 1e-6
    noise = 100 * np.finfo(float).eps * abs(L0) / h
    fds = np.zeros(32)
    for k in range(32):
        e = np.zeros(32)
        e[k] = h
        fds[k] = (loss_at(seg_eval + e) - loss_at(seg_eval - e)) / (2 * h)
    gmax = np.abs(gs).max()
    err = rel_l2(gs, fds)
    print(f"  loss {L0:.4e}; |g|max {gmax:.3e}; rel L2 adjoint vs FD over 32 segments {err:.2e}", flush=True)
    assert gmax > 0
    assert err <= 1e-5
    # per segment; components far below the gradient's scale sit where
    # stick/slip switches make the difference quotient unreliable
    for k in range(32):
        assert abs(fds[k] - gs[k]) <= 1e-5 * abs(fds[k]) + 1e-6 * gmax + noise, (k, fds[k], gs[k])


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("material,fscale", [(W.SAND, 2e-3), (W.SAND, 3e-2), (W.ELASTIC, 2e-3),
                                             (W.ELASTIC, 3e-2), (W.FLUID, 0.0)])
def test_return_mapping_gradient_from_random_state(orc, precision, material, fscale):
    """Three steps from a random state (F or J, C and stress random): for
    sand the gradient flows through every case of the return (apex,
    elastic, cone), for the elastic material through the plain Hencky
    stress, for the fluid through the equation of state.  At the small
    strain scale the kernels take the series form of the return and of its
    reverse, at the large one the eigen form."""
    from paper_2507_04192_amd.native import Solver
    cfg = W.SimConfig(dim=3, n=(20, 16, 12), dx=0.01, dt=1e-5, material=material, ppc=8,
                      gravity=(0, 0, -9.81), youngs=1e6, rho0=1500.0,
                      wall_mode=(W.SLIP, W.STICK, W.SLIP, W.SLIP, W.COULOMB, W.SLIP),
                      wall_mu=(0, 0, 0, 0, 0.4, 0))
    N = 3001
    x, v, C, G = W.random_state(cfg, N, 52, vscale=0.5, cscale=5.0, fscale=max(fscale, 1e-3), margin=2.0)
    rng = np.random.default_rng(53)
    S = rng.normal(0, 1e-3, size=(3, 3, N))
    S = (S + S.transpose(1, 0, 2)).reshape(9, N)
    Jm1 = None
    if material == W.FLUID:
        S = np.repeat(np.eye(3).reshape(9, 1), N, axis=1) * rng.normal(0, 1e-3, size=N)
        Jm1 = rng.normal(0, 1e-3, size=N)
        G = None
    if precision == "f32":
        x, v, C, S = (a.astype(np.float32).astype(np.float64) for a in (x, v, C, S))
        G = None if G is None else G.astype(np.float32).astype(np.float64)
        Jm1 = None if Jm1 is None else Jm1.astype(np.float32).astype(np.float64)
    steps, frames = 3, [1, 2, 3]
    tr = W.pick_tracers(N, 300, 54)
    tgt = rng.normal(0, 0.3, size=(3, 3, 300)).astype(np.float32).astype(np.float64)
    print(f"[case] return-mapping gradient {material} {precision} fscale={fscale} N={N}", flush=True)
    st0 = oracle_state(orc, cfg, x, v=v, C=C, G=G, S=S, Jm1=Jm1)
    obs_o = orc.Observations(frames, tr, "v", tgt)
    loss_o, gv_o, _ = orc.rollout_grad(cfg, x, v, steps, cfg.dt, None, obs_o, state0=st0)
    s = Solver(cfg, precision, capacity=N, tape_steps=steps, ckpt_every=2)
    s.mpm_init_particles(x, v)
    s.mpm_write_state("C", C, "pid")
    if G is not None:
        s.mpm_write_state("FmI", G, "pid")
    if Jm1 is not None:
        s.mpm_write_state("Jm1", np.asarray(Jm1).reshape(1, -1), "pid")
    s.mpm_write_state("stress", S, "pid")
    s.mpm_set_observations(frames=frames, tracer_pid=tr, lag_field="v", lag_target=tgt)
    loss = s.mpm_forward_loss(steps)
    gv, _ = s.mpm_backward(True, False)
    assert s.mpm_sync_status()[0] == 0
    el, ev = abs(loss - loss_o) / loss_o, rel_l2(_np(gv), gv_o)
    print(f"  loss {el:.2e}; dL/dv0 {ev:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)



@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gradient_from_rest(orc, precision):
    """A sand block released from rest (v0 = 0).  Away from the floor the
    first steps leave the strain at rounding level, where the return is not
    differentiable (the apex); below a Hencky strain of 1e-6 both sides take
    the elastic case, so the branch, and with it the gradient, is the same on
    both sides.  Element-wise parity at the usual bounds; no overflow in the
    reverse of the return (it has terms like tr E / |dev E|^2)."""
    cfg = W.SimConfig(dim=2, n=(48, 24, 1), dx=1 / 80, dt=2e-5, material=W.SAND, ppc=4,
                      gravity=(0, -9.81, 0), rho0=2000.0, youngs=1e7, poisson=0.3, phi_deg=35.0,
                      wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP),
                      wall_mu=(0, 0, 0.5, 0, 0, 0))
    x0 = W.lattice_particles(cfg, W.box_inside((0.1, 0), (0.4, 0.1)), (0.1, 0), (0.4, 0.1), seed=120)
    x0 = x0.astype(np.float32).astype(np.float64)
    N = x0.shape[1]
    v0 = np.zeros((2, N))
    steps, frames = 20, [5, 10, 15, 20]
    tr = W.pick_tracers(N, 40, 121)
    tgt = np.random.default_rng(122).normal(0, 0.05, size=(4, 2, 40)).astype(np.float32).astype(np.float64)
    print(f"[case] gradient from rest {precision} N={N}", flush=True)
    obs_o = orc.Observations(frames, tr, "v", tgt)
    loss_o, gv_o, _ = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, None, obs_o)
    loss, gv, _, _ = run_gpu(cfg, precision, x0, v0, None, steps, 8,
                             dict(frames=frames, tracer_pid=tr, lag_field="v", lag_target=tgt))
    assert np.all(np.isfinite(gv))
    el, ev = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o)
    print(f"  loss {el:.2e}; dL/dv0 {ev:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)


_REST = {}


def _cylinder_from_rest_oracle(orc):
    """The oracle's loss and gradients for the benchmark's forward+adjoint
    leg at 1/8 scale (computed once for both precisions)."""
    if "res" not in _REST:
        cfg, x0 = W.cylinder_collapse_3d(scale_div=8, seed=0)
        x0 = x0.astype(np.float32).astype(np.float64)
        N = x0.shape[1]
        steps, k = 200, 50
        tr = W.pick_tracers(N, 500, 7)
        frames = list(range(20, steps + 1, 20))
        tgt = np.repeat(x0[:, tr][None], len(frames), axis=0)
        mu = np.full(cfg.floor_nodes(), cfg.wall_mu[4])
        obs_o = orc.Observations(frames, tr, "x", tgt)
        loss_o, gv_o, gmu_o = orc.rollout_grad(cfg, x0, np.zeros_like(x0), steps, cfg.dt, mu, obs_o)
        _REST["res"] = (cfg, x0, steps, k, tr, frames, tgt, mu, loss_o, gv_o, gmu_o)
    return _REST["res"]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cylinder_from_rest_gradient(orc, precision):
    """The benchmark's forward+adjoint leg (cylinder released from rest,
    tracer positions against their starting positions every 20 steps,
    gradients with respect to v0 and the per-node floor friction, checkpoint
    and recomputation) at 1/8 scale (5,376 particles, 200 steps, checkpoint
    every 50): loss and both gradients element-wise against the oracle's
    reverse sweep."""
    print(f"[case] cylinder from rest gradient {precision} (oracle first)", flush=True)
    cfg, x0, steps, k, tr, frames, tgt, mu, loss_o, gv_o, gmu_o = _cylinder_from_rest_oracle(orc)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    loss, gv, gmu, _ = run_gpu(cfg, precision, x0, np.zeros_like(x0), mu, steps, k, obs)
    assert np.all(np.isfinite(gv)) and np.all(np.isfinite(gmu))
    el, ev, em = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o), rel_l2(gmu, gmu_o)
    print(f"  loss {loss:.4e} vs {loss_o:.4e} ({el:.2e}); dL/dv0 {ev:.2e}; dL/dmu {em:.2e} "
          f"(|dL/dmu|max {np.abs(gmu_o).max():.2e})", flush=True)
    # binary32: the loss is a sum of squared displacements of ~8e-5 m (200
    # steps of free settling) read from positions stored to half an ulp of
    # 0.64 m (3e-8 m), so each term carries ~4e-4 relative rounding; the
    # stated binary32 adjoint tolerance (5e-3) covers loss and gradients
    assert el <= (1e-10 if precision == "f64" else 2e-3)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)
    assert em <= (1e-8 if precision == "f64" else 5e-3)


# ---------------------------------------------------------------------------
# Hypoelastic Drucker-Prager (Sec. 2.3 eq:dp_stress; App. A) in the reverse sweep
# ---------------------------------------------------------------------------

def _jaumann_velocity(cfg, x, frac=0.02, div=1.0):
    """Sheared, rotating and stretched start velocity (about `frac` of a
    cell per step): the rollout takes every zone of App. A."""
    a = frac * cfg.dx / cfg.dt
    L = cfg.n[0] * cfg.dx
    v = np.empty_like(x)
    v[0] = a * (0.8 + 0.4 * np.sin(2 * np.pi * x[1] / L) + div * np.sin(4 * np.pi * x[0] / L))
    v[1] = a * 0.5 * np.cos(2 * np.pi * x[0] / L)
    if x.shape[0] == 3:
        v[2] = a * 0.3 * np.sin(2 * np.pi * (x[0] + x[1]) / L)
    return v


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dp_jaumann_block_gradient_matches_oracle(orc, precision):
    """2-D granular block of the hypoelastic material on a Coulomb floor,
    moving start: tracer positions at four frames over 24 steps; gradients
    with respect to v0 and the per-node floor friction."""
    cfg = W.SimConfig(dim=2, n=(64, 32, 1), dx=1 / 160, dt=1e-5, material=W.DP_JAUMANN, ppc=4,
                      gravity=(0, -9.81, 0), rho0=2000.0, youngs=1e7, poisson=0.3, phi_deg=35.0, psi_deg=5.0,
                      wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP),
                      wall_mu=(0, 0, 0.5, 0, 0, 0))
    x0 = W.lattice_particles(cfg, W.box_inside((0.1, 0), (0.3, 0.1)), (0.1, 0), (0.3, 0.1), seed=90)
    N = x0.shape[1]
    rng = np.random.default_rng(91)
    v0 = _jaumann_velocity(cfg, x0)
    mu = rng.uniform(0.3, 0.6, cfg.floor_nodes())
    tr = W.pick_tracers(N, 48, 92)
    steps, k = 24, 7
    frames = [6, 12, 18, 24]
    tgt = np.stack([x0[:, tr] + rng.normal(0, 2e-4, size=(2, 48)) for _ in frames])
    if precision == "f32":
        x0, v0, mu, tgt = (a.astype(np.float32).astype(np.float64) for a in (x0, v0, mu, tgt))
    print(f"[case] dp_jaumann block gradient {precision} N={N}", flush=True)
    obs_o = orc.Observations(frames, tr, "x", tgt)
    loss_o, gv_o, gmu_o = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, mu, obs_o)
    loss, gv, gmu, _ = run_gpu(cfg, precision, x0, v0, mu, steps, k,
                               dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt))
    el, ev, em = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o), rel_l2(gmu, gmu_o)
    print(f"  loss {loss:.6e} vs {loss_o:.6e} ({el:.2e}); dL/dv0 {ev:.2e}; dL/dmu {em:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    tol = 1e-8 if precision == "f64" else 5e-3
    assert ev <= tol and em <= tol
    assert np.abs(gmu_o).max() > 0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dp_jaumann_prestressed_3d_gradient_matches_oracle(orc, precision):
    """3-D cube of the hypoelastic material with cohesion, a negative
    cutoff and a random prestress spread over the three zones, random
    velocities: tracer velocities at three frames over 6 steps, gradient
    with respect to v0 (the prestress enters through the recorded state)."""
    cfg = W.SimConfig(dim=3, n=(20, 16, 12), dx=0.01, dt=1e-5, material=W.DP_JAUMANN, ppc=8,
                      gravity=(0, 0, -9.81), youngs=1e6, rho0=1500.0, phi_deg=30.0, psi_deg=10.0,
                      cohesion=200.0, tension=-50.0,
                      wall_mode=(W.SLIP, W.STICK, W.SLIP, W.SLIP, W.COULOMB, W.SLIP),
                      wall_mu=(0, 0, 0, 0, 0.4, 0))
    N = 2003
    x0, v0, C0, _ = W.random_state(cfg, N, 93, vscale=0.5, cscale=5.0, margin=2.0)
    rng = np.random.default_rng(94)
    sig = rng.normal(0, 1, size=(3, 3, N))
    sig = 0.5 * (sig + sig.transpose(1, 0, 2)) * rng.uniform(0, 3e3, size=N)
    sig += np.eye(3)[:, :, None] * rng.uniform(-3e3, 1e3, size=N)
    S0 = (sig * cfg.vol0).reshape(9, N)
    tr = W.pick_tracers(N, 40, 95)
    steps, k = 6, 4
    frames = [2, 4, 6]
    tgt = rng.normal(0, 0.1, size=(3, 3, 40))
    if precision == "f32":
        x0, v0, C0, S0, tgt = (a.astype(np.float32).astype(np.float64) for a in (x0, v0, C0, S0, tgt))
    print(f"[case] dp_jaumann prestressed 3-D gradient {precision} N={N}", flush=True)
    st0 = oracle_state(orc, cfg, x0, v=v0, C=C0, S=S0)
    obs_o = orc.Observations(frames, tr, "v", tgt)
    loss_o, gv_o, _ = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, None, obs_o, state0=st0)
    from paper_2507_04192_amd.native import Solver
    s = Solver(cfg, precision, capacity=N, tape_steps=steps, ckpt_every=k)
    s.mpm_init_particles(x0, v0)
    s.mpm_write_state("C", C0, "pid")
    s.mpm_write_state("stress", S0, "pid")
    s.mpm_set_observations(frames=frames, tracer_pid=tr, lag_field="v", lag_target=tgt)
    loss = s.mpm_forward_loss(steps)
    gv, _ = s.mpm_backward(True, False)
    assert s.mpm_sync_status()[0] == 0
    s.close()
    el, ev = abs(loss - loss_o) / loss_o, rel_l2(_np(gv), gv_o)
    print(f"  loss {loss:.6e} vs {loss_o:.6e} ({el:.2e}); dL/dv0 {ev:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    assert ev <= (1e-8 if precision == "f64" else 5e-3)


def _other_form_case(form):
    """Small 2-D cases of the step's other forms: the granular block with
    the PIC, TPIC or FLIP/PIC (alpha = 0.9) transfer, the dam-break of the friction case with a
    viscous fluid, or with a resting box just ahead of its front."""
    if form in ("pic", "tpic", "flip"):
        cfg = W.SimConfig(dim=2, n=(64, 32, 1), dx=1 / 160, dt=1e-5, material=W.SAND, ppc=4,
                          gravity=(0, -9.81, 0), rho0=2000.0, youngs=1e7, poisson=0.3, phi_deg=35.0,
                          wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP),
                          wall_mu=(0, 0, 0.5, 0, 0, 0), transfer={"pic": W.PIC, "tpic": W.TPIC, "flip": W.FLIP}[form],
                          flip_alpha=0.9)
        x0 = W.lattice_particles(cfg, W.box_inside((0.1, 0), (0.3, 0.1)), (0.1, 0), (0.3, 0.1), seed=100)
        v0 = _jaumann_velocity(cfg, x0, frac=0.02, div=0.5)
        rng = np.random.default_rng(101)
        mu = rng.uniform(0.3, 0.6, cfg.floor_nodes())
        N = x0.shape[1]
        tr = W.pick_tracers(N, 48, 102)
        steps, k, frames = 24, 7, [6, 12, 18, 24]
        tgt = np.stack([x0[:, tr] + rng.normal(0, 2e-4, size=(2, 48)) for _ in frames])
        return cfg, x0, v0, mu, tr, frames, tgt, steps, k
    cfg, x0, v0, mu, tr, frames, tgt, steps = friction_case()
    if form == "viscous":
        cfg = cfg.replace(viscosity=2.0)
    else:
        h = cfg.dx
        cfg = cfg.replace(obstacles=(((0.25 + 0.35 * h, 0.0), (0.25 + 3.3 * h, 0.2)),))
    return cfg, x0, v0, mu, tr, frames, tgt, steps, 13


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("form", ["pic", "tpic", "flip", "viscous", "obstacle"])
def test_other_forms_gradient_matches_oracle(orc, precision, form):
    """Gradients through the reverse sweep of the step's other forms (PIC,
    TPIC and the FLIP/PIC blend, Sec. 2.2 and App. B; the Newtonian viscous fluid, Sec.
    2.3 eq:stress_strain; a resting obstacle, Sec. 4.2.1) with respect to v0
    and the per-node floor friction, against the oracle's reverse sweep."""
    cfg, x0, v0, mu, tr, frames, tgt, steps, k = _other_form_case(form)
    if precision == "f32":
        x0, v0, mu, tgt = (a.astype(np.float32).astype(np.float64) for a in (x0, v0, mu, tgt))
    N = x0.shape[1]
    print(f"[case] {form} gradient {precision} N={N}", flush=True)
    obs = dict(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)
    obs_o = orc.Observations(frames, tr, "x", tgt)
    loss_o, gv_o, gmu_o = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, mu, obs_o)
    loss, gv, gmu, _ = run_gpu(cfg, precision, x0, v0, mu, steps, k, obs)
    el, ev, em = abs(loss - loss_o) / loss_o, rel_l2(gv, gv_o), rel_l2(gmu, gmu_o)
    print(f"  loss {loss:.6e} vs {loss_o:.6e} ({el:.2e}); dL/dv0 {ev:.2e}; dL/dmu {em:.2e}", flush=True)
    assert el <= (1e-10 if precision == "f64" else 1e-4)
    tol = 1e-8 if precision == "f64" else 5e-3
    assert ev <= tol and em <= tol
    assert np.abs(gmu_o).max() > 0
    if form in ("viscous", "obstacle") and precision == "f64":
        # the form changes the gradient: the same rollout without it differs
        base = cfg.replace(viscosity=0.0, obstacles=())
        _, gv_b, _ = orc.rollout_grad(base, x0, v0, steps, cfg.dt, mu, obs_o)
        assert rel_l2(gv_b, gv_o) > 1e-3

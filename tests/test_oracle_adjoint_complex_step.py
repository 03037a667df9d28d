"""The oracle's hand-written adjoint against the complex-step derivative of
its own forward step (the dot-product test <grad L, delta> = dL/de along
delta, Sec. 3.1 eq:dzda).

The forward step is compiled a second time with complex binary64 data: a
state a + i h delta, stepped with every branch taken on the real part,
gives Im L / h = dL/de (a + e delta) with no cancellation, so the
derivative is exact to rounding (h = 1e-20 leaves an O(h^2) error far below
it).  Finite differences pin the adjoint to about 1e-6; this pins it to
about 1e-15, for every input field and the floor friction at once, in every
material, transfer and boundary form, and over a rollout with the
Lagrangian and Eulerian losses.  A dropped term anywhere in the reverse
sweep, however small its contribution, fails here.

The complex functions (csqrt, clog, cexp, cpow) round differently from the
real ones, so the real part of the complex step matches the real step to
rounding, not bit for bit; that it matches within 1e-12 also shows that
both took the same branches.
"""
import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W
from tests.test_oracle_adjoint import _cfg, _other_form, _outputs, _state

H = 1e-20
TOL_DOT = 1e-12
TOL_REAL = 1e-12


def _jaumann_state(orc, cfg, N, seed):
    """Prestresses spread over the three zones of App. A (elastic, shear
    failure, tension cutoff)."""
    d = cfg.dim
    rng = np.random.default_rng(seed)
    x, v, C, _ = W.random_state(cfg, N, seed + 1, vscale=0.3, cscale=3.0, margin=0.3)
    sig = rng.normal(0, 1, size=(d, d, N))
    sig = 0.5 * (sig + sig.transpose(1, 0, 2)) * rng.uniform(0, 150, size=N)
    sig += np.eye(d)[:, :, None] * rng.uniform(-300, 200, size=N)
    J = 1.0 + rng.normal(0, 1e-3, size=N)
    S = (sig * (cfg.vol0 * J)).reshape(d * d, N)
    return orc.State(cfg, x, v=v, C=C, J=J, S=S)


def _form(dim, form):
    if form in ("fluid", "sand", "elastic"):
        return _cfg(dim, {"fluid": W.FLUID, "sand": W.SAND, "elastic": W.ELASTIC}[form])
    if form == "jaumann":
        return _cfg(dim, W.DP_JAUMANN, phi_deg=30.0, psi_deg=10.0, cohesion=40.0, tension=-10.0)
    if form == "flip1":
        return _cfg(dim, W.SAND, transfer=W.FLIP, flip_alpha=1.0)
    return _other_form(dim, form)


FORMS = ["fluid", "viscous", "sand", "elastic", "jaumann", "pic", "tpic", "flip", "flip1", "obstacle"]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("form", FORMS)
def test_adjoint_step_matches_complex_step(orc, dim, form):
    """One step with a per-node Coulomb floor friction: the adjoint's inner
    product with a random direction in every input field (x, v, C, S, F or
    J) and in the floor friction, against Im L / h of the complex step."""
    cfg = _form(dim, form)
    o = orc.Oracle(cfg)
    N = 300 if dim == 3 else 400
    st0 = _jaumann_state(orc, cfg, N, 40 + dim) if form == "jaumann" else _state(orc, cfg, N, 30 + dim)
    rng = np.random.default_rng(20 + dim)
    mu = rng.uniform(0.2, 0.4, cfg.floor_nodes())
    st1 = st0.copy()
    o.step(st1, cfg.dt, mu)
    w = {k: rng.normal(size=v.shape) for k, v in _outputs(cfg, st1).items()}
    amu = np.zeros_like(mu)
    g = orc.adjoint_step(cfg, st0, w, cfg.dt, mu, amu)

    fields = ["x", "v", "C", "S"] + (["J"] if cfg.material in (W.FLUID, W.DP_JAUMANN) else ["F"])
    scale = {"x": cfg.dx, "v": 1.0, "C": 10.0, "S": np.abs(st0.S).max(), "J": 1e-3, "F": 1e-3}
    delta = {f: rng.normal(size=getattr(st0, f).shape) * scale[f] for f in fields}
    dmu = rng.normal(size=mu.shape) * 0.1
    sc = st0.copy()
    for f in fields:
        setattr(sc, f, getattr(st0, f) + 1j * H * delta[f])
    o.step_complex(sc, cfg.dt, mu + 1j * H * dmu)

    for k in w:
        real = np.real(getattr(sc, k))
        ref = getattr(st1, k)
        assert np.abs(real - ref).max() <= TOL_REAL * max(np.abs(ref).max(), 1e-30), k
    cs = sum(complex((w[k] * getattr(sc, k)).sum()) for k in w).imag / H
    ad = sum(float((g[f] * delta[f]).sum()) for f in fields) + float((amu * dmu).sum())
    assert abs(cs - ad) <= TOL_DOT * abs(cs), (cs, ad)
    if form == "obstacle":
        # the box is in the way: without it the step differs
        s_free = st0.copy()
        orc.Oracle(cfg.replace(obstacles=())).step(s_free, cfg.dt, mu)
        assert np.abs(s_free.v - st1.v).max() > 1e-3
    if cfg.wall_mode[2 * (dim - 1)] == W.COULOMB:
        assert np.abs(amu).max() > 0          # the floor friction is in play


def _complex_loss(orc, st, obs, fi):
    """eq:inverse_loss of one frame on a complex state: the masked sum of
    squared residuals, squared without conjugation so that it stays analytic."""
    lag, eul, cnt = orc.observe(st, obs, fi)
    loss = 0.0 + 0.0j
    if lag is not None:
        m = np.ones(lag.shape[1]) if obs.lag_mask is None else obs.lag_mask[fi]
        r = lag - obs.lag_target[fi]
        loss += (m * (r * r).sum(axis=0)).sum()
    if eul is not None:
        m = np.ones(eul.shape[1]) if obs.eul_mask is None else obs.eul_mask[fi]
        for b in range(eul.shape[1]):
            if cnt[b] > 0 and m[b] != 0:
                r = eul[:, b] - obs.eul_target[fi][:, b]
                loss += m[b] * (r * r).sum()
    return loss


@pytest.mark.parametrize("material", [W.FLUID, W.SAND])
def test_rollout_gradient_matches_complex_step(orc, material):
    """A 2-D block sheared over a Coulomb floor with per-node friction for 40
    steps, observed by 16 tracer positions and the mean velocity in four
    boxes every 10 steps: the reverse sweep's gradients with respect to the
    initial velocity and the floor friction against the complex step of the
    whole rollout."""
    cfg = W.SimConfig(dim=2, n=(24, 12, 1), dx=1 / 32, dt=2e-4, material=material, ppc=4,
                      gravity=(0, -9.81, 0), rho0=1000.0, bulk=2e4, gamma=7.0, youngs=2e5,
                      wall_mode=(W.SLIP, W.SLIP, W.COULOMB, W.SLIP, W.SLIP, W.SLIP))
    x0 = W.lattice_particles(cfg, W.box_inside((0.05, 0), (0.3, 0.2)), (0.05, 0), (0.3, 0.2), seed=61)
    N = x0.shape[1]
    rng = np.random.default_rng(62)
    # sheared and stretched, so that the strain is never at rest
    v0 = np.stack([0.4 + 2.0 * x0[1] + 0.3 * np.sin(9 * x0[0]), -0.3 * x0[1] + 0.1 * np.cos(7 * x0[0])])
    mu = rng.uniform(0.1, 0.6, cfg.floor_nodes())
    steps, frames = 40, [10, 20, 30, 40]
    tr = W.pick_tracers(N, 16, 63)
    lo = np.array([[0.05, 0.0], [0.15, 0.0], [0.05, 0.1], [0.2, 0.05]])
    hi = lo + np.array([0.1, 0.08])
    probe = orc.Observations(frames, tr, "x", np.zeros((4, 2, 16)), box_lo=lo, box_hi=hi, eul_field="v",
                             eul_target=np.zeros((4, 2, 4)))
    _, _, qs = orc.rollout(cfg, x0, v0 * 0.8, steps, cfg.dt, mu * 1.3, probe)
    obs = orc.Observations(frames, tr, "x", np.stack([q[0] for q in qs]), box_lo=lo, box_hi=hi,
                           eul_field="v", eul_target=np.stack([q[1] for q in qs]))
    loss, gv0, amu = orc.rollout_grad(cfg, x0, v0, steps, cfg.dt, mu, obs)
    assert loss > 0 and np.abs(amu).max() > 0

    dv = rng.normal(size=v0.shape)
    dmu = rng.normal(size=mu.shape) * 0.1
    o = orc.Oracle(cfg)
    st = orc.State(cfg, x0, v=v0)
    st.v = st.v + 1j * H * dv
    muc = mu + 1j * H * dmu
    fidx = {f: i for i, f in enumerate(frames)}
    lc = 0.0 + 0.0j
    for t in range(steps):
        o.step_complex(st, cfg.dt, muc)
        if t + 1 in fidx:
            lc += _complex_loss(orc, st, obs, fidx[t + 1])
    assert abs(lc.real - loss) <= 1e-12 * loss
    cs = lc.imag / H
    ad = float((gv0 * dv).sum()) + float((amu * dmu).sum())
    assert abs(cs - ad) <= 1e-11 * abs(cs), (cs, ad)


def test_planted_mistake_below_finite_differences_is_caught(orc, tmp_path, monkeypatch):
    """A mistake of relative size 1e-7 planted in a copy of the oracle's
    reverse step (the APIC factor D^-1 = 4/h^2 of App. B in the adjoint of
    the affine transfer) passes the central-difference check of one step at
    its 2e-6 bound but not the complex-step dot test."""
    import ctypes as ct
    import os
    import shutil
    import subprocess
    src = os.path.dirname(orc.__file__)
    for f in ("mpm_oracle.c", "mpm_oracle_adjoint.c", "mpm_oracle.h"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    p = tmp_path / "mpm_oracle_adjoint.c"
    text = p.read_text()
    line = "double Dinv = 4.0 / (c->dx * c->dx);"
    assert text.count(line) == 1
    p.write_text(text.replace(line, "double Dinv = 4.0000004 / (c->dx * c->dx);"))
    so = str(tmp_path / "liborc_planted.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                    str(tmp_path / "mpm_oracle.c"), str(p), "-o", so, "-lm"], check=True)
    planted = ct.CDLL(so)
    orc._declare(planted)

    cfg = _form(3, "sand")
    o = orc.Oracle(cfg)
    st0 = _state(orc, cfg, 300, 33)
    rng = np.random.default_rng(23)
    st1 = st0.copy()
    o.step(st1, cfg.dt)
    w = {k: rng.normal(size=v.shape) for k, v in _outputs(cfg, st1).items()}
    dC = rng.normal(size=st0.C.shape) * 10.0

    def grad(lib):
        monkeypatch.setattr(orc, "_lib", lib)
        return orc.adjoint_step(cfg, st0, w, cfg.dt)["C"]

    g_true, g_planted = grad(orc.lib()), grad(planted)
    monkeypatch.undo()
    sc = st0.copy()
    sc.C = st0.C + 1j * H * dC
    o.step_complex(sc, cfg.dt)
    cs = sum(complex((w[k] * getattr(sc, k)).sum()) for k in w).imag / H

    def loss(st):
        s = st.copy()
        o.step(s, cfg.dt)
        return sum(float((w[k] * v).sum()) for k, v in _outputs(cfg, s).items())

    eps = 1e-2
    sp, sm = st0.copy(), st0.copy()
    sp.C, sm.C = st0.C + eps * 1e-3 * dC, st0.C - eps * 1e-3 * dC
    fd = (loss(sp) - loss(sm)) / (2 * eps * 1e-3)
    ad_true = float((g_true * dC).sum())
    ad_planted = float((g_planted * dC).sum())
    assert abs(cs - ad_true) <= TOL_DOT * abs(cs)                   # the oracle as it is
    assert abs(fd - ad_planted) <= 2e-6 * abs(fd)                   # finite differences miss the mistake
    print(f"  complex step {cs:.15e}, adjoint {ad_true:.15e} (rel {abs(cs - ad_true) / abs(cs):.1e}), planted "
          f"{ad_planted:.15e} (rel {abs(cs - ad_planted) / abs(cs):.1e}); central differences {fd:.15e} "
          f"(rel {abs(fd - ad_planted) / abs(fd):.1e} to the planted adjoint)", flush=True)
    assert abs(cs - ad_planted) > 1e3 * TOL_DOT * abs(cs)           # the complex step does not

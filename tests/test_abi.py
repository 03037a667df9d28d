"""The C-ABI library loads and exports every symbol that include/mpm.h
declares; configuration errors come back as status codes (no GPU needed)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "mpm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_calls():
    syms = header_symbols()
    for s in ("mpm_create", "mpm_step", "mpm_read_state", "mpm_destroy"):
        assert s in syms


def test_library_exports_header_symbols():
    from paper_2507_04192_amd import native
    L = native.lib()
    missing = [s for s in header_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_config_validation_without_gpu():
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    cfg, _ = W.dam_break_2d()
    L = native.lib()
    c = native.make_config(cfg, "f64")
    nb = ct.c_size_t()
    assert L.mpm_workspace_bytes(ct.byref(c), 8192, 0, 0, ct.byref(nb)) == 0
    assert nb.value > 8192 * 8
    bad = native.make_config(cfg, "f64")
    bad.dim = 4
    assert L.mpm_workspace_bytes(ct.byref(bad), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert b"dim" in L.mpm_last_error(None)
    bad = native.make_config(cfg, "f64")
    bad.tile = 5
    assert L.mpm_workspace_bytes(ct.byref(bad), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    bad = native.make_config(cfg, "f64")
    bad.dx = -1.0
    assert L.mpm_workspace_bytes(ct.byref(bad), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    bad = native.make_config(cfg, "f64")
    bad.wall_mode[2] = 7
    assert L.mpm_workspace_bytes(ct.byref(bad), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert L.mpm_workspace_bytes(ct.byref(c), -5, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    # a null context is rejected, not dereferenced
    assert L.mpm_step(None, 1, 1e-4) == native.MPM_EINVAL
    assert L.mpm_destroy(None) == 0


def test_grid_beyond_int32_keys_is_rejected():
    """Cell keys are int32 (tile * 64 + cell): a grid whose tile count times
    64 reaches 2^31 is an EINVAL from both mpm_workspace_bytes and
    mpm_create, computed without overflow; the largest grid below the
    limit is accepted."""
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    L = native.lib()
    nb = ct.c_size_t()
    cfg = W.SimConfig(dim=3, n=(8192, 8192, 8192), dx=1e-3, dt=1e-5, material=W.SAND, ppc=8)
    c = native.make_config(cfg, "f32")
    assert L.mpm_workspace_bytes(ct.byref(c), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert b"32-bit cell keys" in L.mpm_last_error(None)
    ctx = ct.c_void_p()
    assert L.mpm_create(ct.byref(c), None, ct.byref(ctx)) == native.MPM_EINVAL
    # 2^31 / 64 = 2^25 tiles.  With 4^3-cell tiles, 8192 x 8192 cells take
    # ceil(8197 / 4)^2 = 2050^2 tile columns: 7 tiles deep (n_z = 23) is
    # below the limit, 8 (n_z = 24) above it
    below = W.SimConfig(dim=3, n=(8192, 8192, 23), dx=1e-3, dt=1e-5, material=W.SAND, ppc=8)
    above = below.replace(n=(8192, 8192, 24))
    assert L.mpm_workspace_bytes(ct.byref(native.make_config(below, "f32")), 10, 0, 0, ct.byref(nb)) == 0
    assert L.mpm_workspace_bytes(ct.byref(native.make_config(above, "f32")), 10, 0, 0, ct.byref(nb)) == native.MPM_EINVAL


def test_added_physics_validation_without_gpu():
    """Transfers, obstacles, viscosity and the hypoelastic Drucker-Prager
    parameters are checked by mpm_workspace_bytes (no GPU needed); a FLIP
    workspace is larger (its P2G blocks and grid carry the velocity before
    the update)."""
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    L = native.lib()
    nb = ct.c_size_t()
    cfg, _ = W.dam_break_2d()

    def rc(c):
        return L.mpm_workspace_bytes(ct.byref(native.make_config(c, "f32")), 100, 0, 0, ct.byref(nb))

    assert rc(cfg) == 0
    base = nb.value
    assert rc(cfg.replace(transfer=W.FLIP, flip_alpha=0.97)) == 0 and nb.value > base
    for good in (cfg.replace(transfer=W.PIC), cfg.replace(transfer=W.TPIC), cfg.replace(viscosity=1.01e-3),
                 cfg.replace(obstacles=(((0.6, 0.0), (0.7, 0.3)),))):
        assert rc(good) == 0
    bad = native.make_config(cfg, "f32")
    bad.transfer = 7
    assert L.mpm_workspace_bytes(ct.byref(bad), 100, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert b"transfer" in L.mpm_last_error(None)
    assert rc(cfg.replace(transfer=W.FLIP, flip_alpha=1.5)) == native.MPM_EINVAL
    assert rc(cfg.replace(obstacles=(((0.7, 0.0), (0.6, 0.3)),))) == native.MPM_EINVAL
    bad = native.make_config(cfg, "f32")
    bad.n_obstacles = 5
    assert L.mpm_workspace_bytes(ct.byref(bad), 100, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert rc(cfg.replace(viscosity=-1.0)) == native.MPM_EINVAL
    sand, _ = W.cylinder_collapse_3d(scale_div=8)
    assert rc(sand.replace(viscosity=1.0)) == native.MPM_EINVAL            # viscosity is the fluid's
    dp = sand.replace(material=W.DP_JAUMANN, psi_deg=5.0)
    assert rc(dp) == 0
    assert rc(dp.replace(psi_deg=40.0)) == native.MPM_EINVAL               # psi above phi
    assert rc(dp.replace(tension=10.0)) == native.MPM_EINVAL               # above the apex (c = 0)
    assert rc(dp.replace(cohesion=1000.0, tension=10.0)) == 0              # below it with cohesion
    assert rc(dp.replace(cohesion=-1.0)) == native.MPM_EINVAL


def test_tape_segments_workspace_without_gpu():
    """Each taped segment adds ckpt_every + 1 states and ckpt_every grid
    records to the workspace; the count is clamped to the rollout's segments
    and validated."""
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    cfg, _ = W.dam_break_2d()
    L = native.lib()
    nb = ct.c_size_t()
    sizes = []
    for ns in (0, 1, 2, 3, 10, 11):
        c = native.make_config(cfg, "f64", tape_segments=ns)
        assert L.mpm_workspace_bytes(ct.byref(c), 8192, 100, 10, ct.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[0] == sizes[1]                          # 0 and 1: the last segment only
    per = sizes[2] - sizes[1]
    assert per > 11 * 8192 * 8 and sizes[3] - sizes[2] == per
    assert sizes[4] == sizes[1] + 9 * per and sizes[5] == sizes[4]   # at most the 10 segments
    for bad in (-1, 65):
        c = native.make_config(cfg, "f64", tape_segments=bad)
        assert L.mpm_workspace_bytes(ct.byref(c), 8192, 100, 10, ct.byref(nb)) == native.MPM_EINVAL
        assert b"tape_segments" in L.mpm_last_error(None)


def test_max_tape_segments_within_budget():
    """The binding's choice of taped segments: every segment within a large
    budget, one within a tiny one, and in between the most whose workspace
    fits."""
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    cfg, _ = W.dam_break_2d()
    L = native.lib()
    nb = ct.c_size_t()

    def ws(ns):
        c = native.make_config(cfg, "f64", tape_segments=ns)
        assert L.mpm_workspace_bytes(ct.byref(c), 8192, 100, 10, ct.byref(nb)) == 0
        return nb.value

    assert native.max_tape_segments(cfg, "f64", 8192, 100, 10, 1 << 40) == 10
    assert native.max_tape_segments(cfg, "f64", 8192, 100, 10, 1) == 1
    assert native.max_tape_segments(cfg, "f64", 8192, 100, 10, ws(4)) == 4
    assert native.max_tape_segments(cfg, "f64", 8192, 100, 10, ws(5) - 1) == 4


def test_track_eps_eq_workspace_without_gpu():
    """Carrying the equivalent plastic strain adds two scalars per particle
    of workspace; any value other than 0 or 1 is refused."""
    from paper_2507_04192_amd import native
    from paper_2507_04192_amd import workloads as W
    cfg, _ = W.cylinder_collapse_3d(scale_div=8)
    L = native.lib()
    nb = ct.c_size_t()
    sizes = {}
    for prec, elem in (("f32", 4), ("f64", 8)):
        for t in (0, 1):
            c = native.make_config(cfg, prec, track_eps_eq=t)
            assert L.mpm_workspace_bytes(ct.byref(c), 100000, 0, 0, ct.byref(nb)) == 0
            sizes[prec, t] = nb.value
        extra = sizes[prec, 1] - sizes[prec, 0]
        assert 2 * 100000 * elem <= extra <= 2 * 100000 * elem + 512
    c = native.make_config(cfg, "f32")
    c.track_eps_eq = 2
    assert L.mpm_workspace_bytes(ct.byref(c), 100, 0, 0, ct.byref(nb)) == native.MPM_EINVAL
    assert b"track_eps_eq" in L.mpm_last_error(None)

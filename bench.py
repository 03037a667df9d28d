#!/usr/bin/env python
"""Throughput of the explicit MPM step on one MI355X.

Workload: 3-D granular cylinder collapse -- 256 x 256 x 64 cells, dx = 5 mm,
a sand cylinder of radius and height 48 cells at 2x2x2 particles per cell
(2,780,928 particles), Drucker-Prager sand with the Hencky return, floor
Coulomb mu = 0.5, dt = 2e-5 s.  Synthetic seeded input (no dataset).

A step is one pass of the whole hot path: cell-key sort, P2G, grid update,
G2P with the constitutive update.  Inputs are resident in HBM before the
timed region starts.  Prints one JSON line.

The forward+adjoint leg times a checkpointed rollout with a tracer loss and
its backward sweep on the same cylinder (FP32 and FP64; 1000 steps with a
checkpoint every 100 by default), keeping as many trailing segments on the
tape as three quarters of the free device memory holds (the backward sweep
recomputes only the others).

The late_phase leg times the FP32 step again after 3000 steps, when the
sand has spread and moves faster (the headline value is the first 1000
steps from rest).  The other_configs leg times the forward step of the other benchmark
configurations (the 2-D dam-breaks and granular block, the 3-D dam-break)
without per-kernel events.  The variants leg times the other forms of the step: the cylinder with the
hypoelastic Drucker-Prager material (Jaumann rate, App. A) and with the PIC,
TPIC and FLIP transfers, the 3-D dam-break against two rigid columns
with a viscous fluid (Sec. 4.2.1, 1,920,000 particles on 200 x 100 x 80),
and the paper's two granular timing cases on its own grids: the cylinder
collapse on 400 x 400 x 100 (2,713,580 particles) and the column of aspect
ratio 3 on 400 x 32 x 200 (2,408,448 particles), each set beside the
paper's single-A100 figures.  The paper_inverse leg times forward+gradient
in binary64 on the 2-D dam-breaks of the paper's inverse problems (10,000,
40,000 and 6,000 particles) beside its "sim + grad" figures.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s fwd & fwd+adjoint, 3D 2.7M-particle collapse; % of HBM peak"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E peak

# Algorithmic scalars per particle moved by each kernel (3-D sand).  The
# state is x3 v3 C9 F9; a forward step must read it once and write it once
# (48 scalars), and the forward kernels split that as
#   G2P reads x, F and writes x, v, C, F        36
#   P2G reads v, C                              12
# The reverse step must read the state (24) and the output adjoint (24) and
# write the input adjoint (24):
#   reverse G2P reads x, F and the output adjoint of x v C F      36
#   reverse P2G reads v, C and writes the input adjoint of x v C F 36
# Everything else a kernel moves is design overhead, reported beside it:
# the stress cache (6 symmetric scalars written by G2P, read by P2G; its
# adjoint in the reverse kernels), P2G's second read of x, the 12-scalar
# intermediate between the reverse kernels, and the int32 sort arrays
# (pid read and written, key written, permutation and bucket indices).
ALG_SCALARS = {"g2p": 3 + 9 + 3 + 3 + 9 + 9, "p2g": 3 + 9,
               "g2p_adj": 3 + 9 + 24, "p2g_adj": 3 + 9 + 24}
OVERHEAD_SCALARS = {"g2p": 6, "p2g": 6 + 3, "g2p_adj": 6 + 12, "p2g_adj": 3 + 6 + 12 + 6}
OVERHEAD_INT_BYTES = {"g2p": 4 + 4 + 4 + 4, "p2g": 4 + 4 + 4, "g2p_adj": 4, "p2g_adj": 4 + 4}
ALG_INT_BYTES = {"bucket": 8}
STEP_SCALARS = 48                # forward step: the state read once, written once
ADJ_STEP_SCALARS = 168           # forward+adjoint: two forward passes (96) + reverse (72)
# Vector-ALU work of a 3-D sand particle-step with the gradient-form force
# and velocity gradient (P2G ~0.95k, G2P ~1.25k, constitutive ~1.2k flops,
# an FMA counted as 2), and the vector peak it is set against: packed FP32
# is disabled in every build here, so FP32 issues at the FP64 rate,
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s.
VALU_FLOPS_PER_PSTEP = 3400.0
VALU_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(cfg, x, precision, steps, warmup, profile=True):
    import torch
    from paper_2507_04192_amd.native import Solver
    s = Solver(cfg, precision, capacity=x.shape[1])
    s.mpm_init_particles(x)
    s.mpm_step(warmup)
    rc, bad = s.mpm_sync_status()
    if rc != 0:
        raise RuntimeError(f"solver status {rc} (pid {bad}) during warm-up")
    torch.cuda.synchronize()
    s.mpm_profile_enable(profile)
    s.mpm_profile_read()                     # reset
    t0 = time.perf_counter()
    s.mpm_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.mpm_profile_read()
    s.mpm_profile_enable(False)
    rc, bad = s.mpm_sync_status()
    if rc != 0:
        raise RuntimeError(f"solver status {rc} (pid {bad}) in the timed region")
    if not profile:
        s.close()
        return (t1 - t0), None, prof
    # same number of steps without events, to show their cost
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.mpm_step(steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.close()
    return (t1 - t0), (t3 - t2), prof


def run_adjoint(cfg, x, precision, steps, ckpt_every, n_tracers=500, frame_every=20, tape_segments=1):
    """Forward rollout with the loss, then the checkpointed backward sweep:
    tracer positions every frame_every steps against their starting
    positions; gradients with respect to v0 and a per-node floor friction
    field (uniform at the floor's mu).  The trailing tape_segments segments
    stay on the tape (the backward sweep recomputes only the others)."""
    import numpy as np
    import torch
    from paper_2507_04192_amd import workloads as W
    from paper_2507_04192_amd.native import Solver
    n = x.shape[1]
    s = Solver(cfg, precision, capacity=n, tape_steps=steps, ckpt_every=ckpt_every, tape_segments=tape_segments)
    ws_bytes = s.ws.numel()
    s.mpm_set_floor_mu(np.full(cfg.floor_nodes(), cfg.wall_mu[4 if cfg.dim == 3 else 2]))
    tr = W.pick_tracers(n, n_tracers, 7)
    frame_every = min(frame_every, steps)
    frames = list(range(frame_every, steps + 1, frame_every))
    tgt = np.repeat(x[:, tr][None], len(frames), axis=0)
    s.mpm_set_observations(frames=frames, tracer_pid=tr, lag_field="x", lag_target=tgt)

    def once(prof):
        s.mpm_init_particles(x)
        torch.cuda.synchronize()
        s.mpm_profile_enable(prof)
        s.mpm_profile_read()
        t0 = time.perf_counter()
        loss = s.mpm_forward_loss(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gv, gm = s.mpm_backward(True, True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p = s.mpm_profile_read()
        s.mpm_profile_enable(False)
        return loss, gv, gm, t1 - t0, t2 - t1, p

    once(False)                                  # warm-up
    loss, gv, gm, tf, tb, prof = once(True)
    ok = bool(np.isfinite(loss) and torch.isfinite(gv).all().item() and torch.isfinite(gm).all().item())
    s.close()
    return {"value": n * steps / (tf + tb), "unit": "particle-steps/s", "steps": steps,
            "ckpt_every": ckpt_every, "tape_segments": tape_segments, "ms_per_step": (tf + tb) / steps * 1e3,
            "forward_loss_ms": tf * 1e3, "backward_ms": tb * 1e3, "loss": loss, "finite": ok,
            "workspace_bytes": ws_bytes, "max_memory_allocated": torch.cuda.max_memory_allocated(),
            "observations": f"{n_tracers} tracer positions every {frame_every} steps; "
                            f"gradients wrt v0 and the floor friction field"}, prof


def run_paper_inverse(steps=1000, ckpt_every=100):
    """The paper's "sim + grad" timing cases (Table tab:simulation_params,
    binary64): forward rollout with the loss and the checkpointed backward
    sweep on the 2-D dam-breaks of its inverse problems, with their
    observations: the velocity problem (Sec. 5.1-5.2) at 10,000 particles
    (150 x 60 cells) and 40,000 (300 x 120), observed by the nine velocity
    monitors every 10 steps, gradients with respect to v0; the friction
    problem (Sec. 5.3, 6,000 particles) observed by 500 tracers every 10
    steps, gradients with respect to v0 and the floor friction.  Every
    segment stays on the tape (at most 5 GB here), so the backward
    sweep recomputes none.  Seconds per 1000 steps beside the paper's
    single-A100 figures (its network or segment parameters add a few small
    kernels per epoch, not timed)."""
    import numpy as np
    import torch
    from paper_2507_04192_amd import workloads as W
    from paper_2507_04192_amd.native import Solver, max_tape_segments
    cases = []
    for name, fine, paper_s in (("velocity inverse, 10,000 particles, 150 x 60 cells", False, 0.62),
                                ("velocity inverse, 40,000 particles, 300 x 120 cells", True, 1.52)):
        cfg, x, H0 = W.inverse_dam_break_2d(fine=fine)
        v0 = np.stack([2.0 * (H0 - x[1]), np.zeros(x.shape[1])])
        lo, hi = W.velocity_monitors_2d()
        cases.append((name, cfg, x, v0, dict(box_lo=lo, box_hi=hi, eul_field="v"), False, paper_s))
    cfg, x, seg = W.friction_segments_2d()
    cases.append(("friction inverse, 6,000 particles, 160 x 40 cells", cfg, x, None,
                  dict(tracer_pid=W.pick_tracers(x.shape[1], 500, 13), lag_field="x"), True, 0.59))
    out = []
    for name, cfg, x, v0, obs, fric, paper_s in cases:
        n = x.shape[1]
        # small problems: every segment fits on the tape, so the backward
        # sweep recomputes none
        ns = max_tape_segments(cfg, "f64", n, steps, ckpt_every, 8 << 30)
        s = Solver(cfg, "f64", capacity=n, tape_steps=steps, ckpt_every=ckpt_every, tape_segments=ns)
        if fric:
            s.mpm_set_floor_mu(W.segment_mu(cfg, np.asarray(W.FRICTION_SEGMENTS_TRUE), seg_len=seg))
        frames = list(range(10, steps + 1, 10))
        if "box_lo" in obs:
            tgt = np.zeros((len(frames), cfg.dim, obs["box_lo"].shape[0]))
            s.mpm_set_observations(frames=frames, eul_target=tgt, **obs)
        else:
            tgt = np.repeat(x[:, obs["tracer_pid"]][None], len(frames), axis=0)
            s.mpm_set_observations(frames=frames, lag_target=tgt, **obs)
        times = []
        for _ in range(3):                       # the first is the warm-up
            s.mpm_init_particles(x, v0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.mpm_forward_loss(steps)
            s.mpm_backward(True, fric)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        s.close()
        best = min(times[1:])
        per1000 = best / steps * 1000
        out.append({"workload": name, "particles": n, "grid": list(cfg.n), "precision": "f64",
                    "steps": steps, "ckpt_every": ckpt_every, "tape_segments": ns, "s_per_1000_steps": per1000,
                    "value": n * steps / best, "unit": "particle-steps/s",
                    "paper_context": {"s_per_1000_steps": paper_s, "ratio": paper_s / per1000,
                                      "note": "paper, one A100, sim + grad in binary64"}})
        log(f"[bench] paper inverse {name}: {per1000:.4f} s per 1000 steps (paper {paper_s})")
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_cylinder.txt")


def traffic_kernels(cls, elem):
    """The 3-D sand kernels behind a timed class (template arguments:
    precision, dimension, material, then FLIP for P2G and the transfer for
    G2P)."""
    t = "float" if elem == 4 else "double"
    names = {"p2g": f"k_p2g<{t}, 3, 1, false>", "g2p": f"k_g2p<{t}, 3, 1, 0>",
             "g2p_adj": f"k_g2p_adj<{t}, 3, 1, false>", "p2g_adj": f"k_p2g_adj<{t}, 3, 1, false>"}
    return [names.get(cls, cls)]


def measured_traffic(kernels):
    """HBM bytes per launch of a kernel (or the sum over a list of kernels)
    from the committed counter summary (FETCH_SIZE + WRITE_SIZE scaled by a
    plain copy), or None when there is none or the kernel sources changed
    since it was taken."""
    if isinstance(kernels, str):
        kernels = [kernels]
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        from paper_2507_04192_amd.rocprof_summary import kernel_sources_hash
        if t.get("csrc_sha256") != kernel_sources_hash():
            return None
        total = 0.0
        for k in kernels:
            v = t["kernels"][k]
            total += v["fetch_bytes"] + v["write_bytes"]
        return total
    except (OSError, KeyError, TypeError, ValueError):
        return None


def calibrate_copy(mib):
    """A plain device-to-device copy of mib MiB (the scale of the HBM byte
    counters is read off its FETCH_SIZE and WRITE_SIZE)."""
    import torch
    n = mib * 2**20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {mib * 2**20} bytes")
    del a, b


def roofline(prof, n_particles, elem):
    kernels = {}
    for k, (ms, n) in prof.items():
        if n > 0:
            kernels[k] = {"avg_ms": ms / n, "launches": n, "total_ms": ms}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    for k, v in kernels.items():
        if k in ALG_SCALARS:
            v["alg_bytes"] = ALG_SCALARS[k] * elem * n_particles
            v["overhead_bytes"] = (OVERHEAD_SCALARS[k] * elem + OVERHEAD_INT_BYTES[k]) * n_particles
        elif k in ALG_INT_BYTES:
            v["alg_bytes"] = ALG_INT_BYTES[k] * n_particles
        if "alg_bytes" in v:
            v["gbs"] = v["alg_bytes"] / (v["avg_ms"] * 1e-3) / 1e9
    d = kernels[dom]
    ach = d.get("gbs")
    return dom, kernels, {
        "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": (ach / HBM_PEAK_GBS) if ach else None, "traffic": None,
        "kernel": dom, "alg_bytes_per_launch": d.get("alg_bytes"),
        "overhead_bytes_per_launch": d.get("overhead_bytes"), "avg_launch_ms": d["avg_ms"],
    }


# State scalars per particle of each form of the step (3-D), read once and
# written once per step: the carried state of the method, nothing else.
#   sand, APIC or TPIC: x v C F          3 + 3 + 9 + 9 = 24
#   sand, PIC or FLIP (no carried C):   x v F            15
#   hypoelastic D-P: x v C J sigma      3 + 3 + 9 + 1 + 6 = 22
#   (viscous) fluid: x v C J            16
VARIANT_STATE_SCALARS = {"sand_apic": 24, "sand_tpic": 24, "sand_pic": 15, "sand_flip": 15,
                         "dp_jaumann": 22, "fluid": 16}
FORM_OF = {"paper_cylinder": "dp_jaumann", "paper_column": "dp_jaumann"}


def run_variants(steps, steps64, warmup, only=""):
    """Forward throughput of the other forms of the step, each at full size in
    the bench's launch configuration (only: run just the legs whose form
    name contains it, e.g. "paper_" for the paper's two timing cases)."""
    from paper_2507_04192_amd import workloads as W
    cyl, xc = W.cylinder_collapse_3d(seed=0)
    col, xd = W.dam_break_columns_3d(seed=0)
    pcy, xpc = W.cylinder_paper_grid(seed=0)
    pco, xpo = W.granular_column_paper(seed=0)
    legs = [
        ("cylinder, hypoelastic Drucker-Prager (Jaumann rate, App. A)", "dp_jaumann",
         cyl.replace(material=W.DP_JAUMANN), xc, ("f32", "f64")),
        ("cylinder, PIC transfer", "sand_pic", cyl.replace(transfer=W.PIC), xc, ("f32",)),
        ("cylinder, TPIC transfer", "sand_tpic", cyl.replace(transfer=W.TPIC), xc, ("f32",)),
        ("cylinder, FLIP/PIC blend alpha = 0.95", "sand_flip", cyl.replace(transfer=W.FLIP, flip_alpha=0.95), xc,
         ("f32",)),
        ("3-D dam-break against two rigid columns, viscous fluid (Sec. 4.2.1)", "fluid", col, xd, ("f32", "f64")),
        ("3-D cylinder collapse on the paper's 400 x 400 x 100 grid, hypoelastic Drucker-Prager (Sec. 4.2.3)",
         "paper_cylinder", pcy, xpc, ("f32", "f64")),
        ("3-D granular column a = 3 on the paper's 400 x 32 x 200 grid, hypoelastic Drucker-Prager (Sec. 4.2.2)",
         "paper_column", pco, xpo, ("f32", "f64")),
    ]
    # the paper's single-A100 timings of the same cases (s per 1000 steps,
    # FP32 / FP64, Table tab:simulation_params) and its particle counts
    paper = {"fluid": (1920000, 8.2, 35.1), "paper_cylinder": (2712960, 22.3, 98.4),
             "paper_column": (2408448, 16.2, 69.3)}
    out = []
    for name, form, cfg, x, precs in legs:
        if only and only not in form:
            continue
        n = x.shape[1]
        r = {"workload": name, "particles": n, "grid": list(cfg.n)}
        for prec in precs:
            elem = 4 if prec == "f32" else 8
            k = steps if prec == "f32" else steps64
            t, _, prof = run_gpu(cfg, x, prec, k, warmup)
            val = n * k / t
            r[prec] = {"value": val, "unit": "particle-steps/s", "steps": k, "ms_per_step": t / k * 1e3,
                       "step_roofline": step_roofline(val, 2 * VARIANT_STATE_SCALARS[FORM_OF.get(form, form)],
                                                      elem),
                       "kernels_us": {kk: round(v[0] / v[1] * 1e3, 2) for kk, v in prof.items() if v[1] > 0}}
            log(f"[bench] variant {name} {prec}: {t / k * 1e3:.4f} ms/step, {val:.4e} particle-steps/s")
        if form in paper:
            pn, s32, s64 = paper[form]
            ctx = {"value_f32": pn * 1000 / s32, "value_f64": pn * 1000 / s64,
                   "note": f"paper, one A100: {s32} / {s64} s per 1000 steps, {pn:,} particles on the same grid"}
            for prec in precs:
                ctx[f"ratio_{prec}"] = r[prec]["value"] / ctx[f"value_{prec}"]
            r["paper_context"] = ctx
        out.append(r)
    return out


def run_late_phase(cfg, x, precision, before, steps):
    """The same step later in the collapse: time `steps` steps after
    `before` untimed ones, when the sand has spread over more tiles and
    moves faster (per-kernel events on)."""
    import torch
    from paper_2507_04192_amd.native import Solver
    s = Solver(cfg, precision, capacity=x.shape[1])
    s.mpm_init_particles(x)
    s.mpm_step(before)
    rc, bad = s.mpm_sync_status()
    if rc != 0:
        raise RuntimeError(f"solver status {rc} (pid {bad}) before the late phase")
    torch.cuda.synchronize()
    s.mpm_profile_enable(True)
    s.mpm_profile_read()
    t0 = time.perf_counter()
    s.mpm_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.mpm_profile_read()
    rc, bad = s.mpm_sync_status()
    s.close()
    if rc != 0:
        raise RuntimeError(f"solver status {rc} (pid {bad}) in the late phase")
    n = x.shape[1]
    return {"after_steps": before, "steps": steps, "value": n * steps / (t1 - t0), "unit": "particle-steps/s",
            "ms_per_step": (t1 - t0) / steps * 1e3,
            "kernels_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items() if v[1] > 0}}


def run_other_configs(steps, warmup):
    """Forward throughput of the other benchmark configurations (binary32 and
    binary64, the same kernels and launch shapes as the cylinder): the 2-D
    dam-break, the 2-D friction dam-break, the 2-D granular block and the
    3-D dam-break of the learned-friction problem."""
    from paper_2507_04192_amd import workloads as W
    gb = W.granular_block_2d()
    legs = [("2-D water column (dam-break), 128 x 64 cells", W.dam_break_2d()),
            ("2-D friction dam-break, 256 x 128 cells", W.friction_dam_break_2d()),
            ("2-D granular block, 256 x 128 cells", (gb[0], gb[1])),
            ("3-D dam-break, 192 x 96 x 64 cells", W.dam_break_3d())]
    out = []
    for name, (cfg, x) in legs:
        n = x.shape[1]
        r = {"workload": name, "particles": n}
        for prec in ("f32", "f64"):
            t, _, _ = run_gpu(cfg, x, prec, steps, warmup, profile=False)
            r[prec] = {"value": n * steps / t, "unit": "particle-steps/s", "steps": steps,
                       "ms_per_step": t / steps * 1e3}
            log(f"[bench] {name} {prec}: {t / steps * 1e3:.4f} ms/step, {n * steps / t:.4e} particle-steps/s")
        out.append(r)
    return out


def step_roofline(value, scalars, elem):
    """The whole step against HBM: the algorithmic bytes per particle-step
    (the state read once and written once; forward+adjoint: two forward
    passes and the reverse step) times particle-steps/s."""
    b = scalars * elem
    ach = value * b / 1e9
    return {"bound": "hbm", "bytes_per_particle_step": b, "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}


def valu_roofline(value, passes=1.0):
    """The whole step against the vector ALUs: VALU_FLOPS_PER_PSTEP per
    particle-step and pass, against the FP32/FP64 vector peak without packed
    FP32."""
    ach = value * VALU_FLOPS_PER_PSTEP * passes / 1e12
    return {"bound": "alu", "flops_per_particle_step": VALU_FLOPS_PER_PSTEP * passes, "achieved": ach,
            "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / VALU_PEAK_TFLOPS}


def copy_probe(mib=1024, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second),
    timed with events on torch's stream, on which the copy runs."""
    import torch
    n = mib * 2**20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    return {"bytes_per_copy": n * 4, "ms": ms, "gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def cpu_baseline(cfg, x, steps):
    import numpy as np
    import oracle
    o = oracle.Oracle(cfg)
    st = oracle.State(cfg, x)
    t0 = time.perf_counter()
    o.run(st, steps, cfg.dt)
    t1 = time.perf_counter()
    n = x.shape[1]
    return {
        "value": n * steps / (t1 - t0), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
        "sample": f"{steps} step(s) of the full {n}-particle cylinder from rest, binary64 C oracle, "
                  f"1 thread ({t1 - t0:.1f} s)",
        "host_cpu": _cpu_name(), "nproc": os.cpu_count(),
    }


def cpu_baseline_adjoint(steps_cyl=20, steps_fric=50):
    """The oracle's forward rollout with a tracer loss and its reverse sweep
    (binary64, one thread), on two bounded samples: the 1/8-scale cylinder
    (the benchmark's forward+adjoint leg shrunk in every length, 500 tracers
    every 10 steps, gradients wrt v0 and the floor friction) and the 2-D
    friction dam-break (32,768 particles, 32 friction segments, 64 tracers
    every 10 steps) for the first steps_fric of its 500 steps."""
    import numpy as np
    import oracle
    from paper_2507_04192_amd import workloads as W
    out = {}
    cfg, x = W.cylinder_collapse_3d(scale_div=8, seed=0)
    n = x.shape[1]
    tr = W.pick_tracers(n, 500, 7)
    frames = list(range(10, steps_cyl + 1, 10))
    obs = oracle.Observations(frames, tracer_pid=tr, lag_field="x",
                              lag_target=np.repeat(x[:, tr][None], len(frames), axis=0))
    mu = np.full(cfg.floor_nodes(), 0.5)
    t0 = time.perf_counter()
    oracle.rollout_grad(cfg, x, np.zeros_like(x), steps_cyl, cfg.dt, floor_mu=mu, obs=obs)
    t1 = time.perf_counter()
    out["cylinder_div8"] = {"value": n * steps_cyl / (t1 - t0), "unit": "particle-steps/s", "cores": 1,
                            "kind": "oracle", "sample": f"{steps_cyl} steps forward+adjoint of the "
                            f"{n}-particle cylinder (1/8 scale), binary64, 1 thread ({t1 - t0:.1f} s)"}
    cfg, x = W.friction_dam_break_2d()
    n = x.shape[1]
    tr = W.pick_tracers(n, 64, 4)
    frames = list(range(10, steps_fric + 1, 10))
    obs = oracle.Observations(frames, tracer_pid=tr, lag_field="x",
                              lag_target=np.repeat(x[:, tr][None], len(frames), axis=0))
    mu = W.segment_mu(cfg, W.uniform_mu_segments(3))
    t0 = time.perf_counter()
    oracle.rollout_grad(cfg, x, np.zeros_like(x), steps_fric, cfg.dt, floor_mu=mu, obs=obs)
    t1 = time.perf_counter()
    out["friction_dam_break"] = {"value": n * steps_fric / (t1 - t0), "unit": "particle-steps/s",
                                 "cores": 1, "kind": "oracle",
                                 "sample": f"{steps_fric} of 500 steps forward+adjoint of the {n}-particle "
                                           f"friction dam-break, binary64, 1 thread ({t1 - t0:.1f} s)"}
    return out


def _cpu_name():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--f64-steps", type=int, default=None, help="binary64 timed steps (default steps/2)")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--adj-steps", type=int, default=1000, help="rollout length of the forward+adjoint leg")
    ap.add_argument("--adj-ckpt", type=int, default=100, help="checkpoint interval of the forward+adjoint leg")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adj-memory-frac", type=float, default=0.75,
                    help="share of the free device memory the forward+adjoint workspace may take "
                         "(trailing segments kept on the tape instead of recomputed)")
    ap.add_argument("--no-variants", action="store_true", help="skip the other forms of the step")
    ap.add_argument("--variant-steps", type=int, default=500, help="binary32 steps per variant (binary64: half)")
    ap.add_argument("--variant-filter", default="", help="run only the variants whose form name contains this")
    ap.add_argument("--no-configs", action="store_true", help="skip the other benchmark configurations")
    ap.add_argument("--no-paper-inverse", action="store_true",
                    help="skip the paper's forward+gradient timing cases of its inverse problems")
    ap.add_argument("--no-late", action="store_true", help="skip the late-phase timing of the collapse")
    ap.add_argument("--late-after", type=int, default=3000, help="untimed steps before the late-phase timing")
    ap.add_argument("--config-steps", type=int, default=1000, help="steps per other configuration")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--scale-div", type=int, default=1, help="shrink the cylinder (tests only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(multi-GPU sharding is designed but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_04192_amd import workloads as W
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
    cfg, x = W.cylinder_collapse_3d(scale_div=args.scale_div, seed=0)
    n = x.shape[1]
    log(f"[bench] cylinder collapse N={n} grid={cfg.n} device={torch.cuda.get_device_name(0)}")

    t32, t32_noev, prof32 = run_gpu(cfg, x, "f32", args.steps, args.warmup)
    ms32 = t32 / args.steps * 1e3
    val32 = n * args.steps / t32
    log(f"[bench] f32: {ms32:.4f} ms/step, {val32:.4e} particle-steps/s "
        f"(no events: {t32_noev / args.steps * 1e3:.4f} ms/step)")
    dom, kernels, roof = roofline(prof32, n, 4)
    if args.scale_div == 1:
        roof["traffic"] = measured_traffic(traffic_kernels(dom, 4))
    for k, v in kernels.items():
        log(f"[bench]   {k:7s} {v['avg_ms'] * 1e3:9.2f} us/launch" +
            (f"  {v['gbs']:8.1f} GB/s algorithmic" if "gbs" in v else ""))

    out_f64 = None
    if not args.no_f64:
        k64 = args.f64_steps or max(1, args.steps // 2)
        t64, t64_noev, prof64 = run_gpu(cfg, x, "f64", k64, args.warmup)
        dom64, kern64, roof64 = roofline(prof64, n, 8)
        if args.scale_div == 1:
            roof64["traffic"] = measured_traffic(traffic_kernels(dom64, 8))
        out_f64 = {"value": n * k64 / t64, "unit": "particle-steps/s", "steps": k64,
                   "ms_per_step": t64 / k64 * 1e3, "ms_per_step_no_events": t64_noev / k64 * 1e3,
                   "hbm_frac_step": n * k64 / t64 * STEP_SCALARS * 8 / (HBM_PEAK_GBS * 1e9),
                   "roofline": roof64,
                   "step_roofline": step_roofline(n * k64 / t64, STEP_SCALARS, 8),
                   "valu_roofline": valu_roofline(n * k64 / t64),
                   "kernels_us": {k: round(v["avg_ms"] * 1e3, 2) for k, v in kern64.items()}}
        log(f"[bench] f64: {out_f64['ms_per_step']:.4f} ms/step, {out_f64['value']:.4e} particle-steps/s")

    adj = None
    if not args.no_adjoint:
        adj = {}
        for prec, elem, T in (("f32", 4, args.adj_steps), ("f64", 8, args.adj_steps)):
            if prec == "f64" and args.no_f64:
                continue
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            free, _ = torch.cuda.mem_get_info()
            from paper_2507_04192_amd.native import max_tape_segments
            nts = max_tape_segments(cfg, prec, n, T, args.adj_ckpt, args.adj_memory_frac * free)
            r, prof = run_adjoint(cfg, x, prec, T, args.adj_ckpt, tape_segments=nts)
            dom_a, kern, roof_a = roofline({k: prof[k] for k in ("g2p_adj", "p2g_adj") if k in prof}, n, elem)
            if args.scale_div == 1:
                roof_a["traffic"] = measured_traffic(traffic_kernels(dom_a, elem))
            r["roofline"] = roof_a
            r["step_roofline"] = step_roofline(r["value"], ADJ_STEP_SCALARS, elem)
            # the forward step runs twice (rollout, segment recompute) and the
            # reverse step costs about two forward steps of VALU work
            r["valu_roofline"] = valu_roofline(r["value"], passes=4.0)
            r["kernels_us"] = {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items() if v[1] > 0}
            adj[prec] = r
            log(f"[bench] fwd+adjoint {prec}: {nts} taped segment(s), {r['ms_per_step']:.4f} ms/step, {r['value']:.4e} particle-steps/s "
                f"(forward {r['forward_loss_ms']:.1f} ms, backward {r['backward_ms']:.1f} ms, "
                f"peak memory {r['max_memory_allocated'] / 2**30:.1f} GiB)")
            for k, v in r["kernels_us"].items():
                log(f"[bench]   {k:8s} {v:9.2f} us/launch")

    variants = None
    if not args.no_variants and args.scale_div == 1:
        variants = run_variants(args.variant_steps, max(1, args.variant_steps // 2), args.warmup,
                                args.variant_filter)
    configs = None
    if not args.no_configs and args.scale_div == 1:
        configs = run_other_configs(args.config_steps, args.warmup)
    paper_inv = None
    if not args.no_paper_inverse and args.scale_div == 1:
        paper_inv = run_paper_inverse()
    late = None
    if not args.no_late:
        late = run_late_phase(cfg, x, "f32", args.late_after, min(args.steps, 500))
        log(f"[bench] f32 after {args.late_after} steps: {late['ms_per_step']:.4f} ms/step, "
            f"{late['value']:.4e} particle-steps/s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] timing the oracle for {args.cpu_steps} step(s) on the host ...")
        cpu = cpu_baseline(cfg, x, args.cpu_steps)
        log(f"[bench] oracle: {cpu['value']:.4e} particle-steps/s")
        if adj is not None:
            log("[bench] timing the oracle's forward+adjoint on bounded samples ...")
            cpu_adj = cpu_baseline_adjoint()
            for k, v in cpu_adj.items():
                log(f"[bench] oracle forward+adjoint {k}: {v['value']:.4e} particle-steps/s")
            adj["cpu_baseline"] = cpu_adj
    copy = copy_probe()
    log(f"[bench] device copy: {copy['gbs']:.1f} GB/s ({copy['frac_of_peak']:.3f} of the HBM peak)")
    roof["frac_of_copy"] = roof["achieved"] / copy["gbs"] if roof["achieved"] else None

    res = {
        "metric": METRIC, "value": val32, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D granular cylinder collapse: 256x256x64 cells, dx=0.005 m, "
                               "cylinder R=H=48 cells, 8 particles/cell, Drucker-Prager sand "
                               "(Hencky return), floor mu=0.5, dt=2e-5 s",
                   "particles": n, "grid": list(cfg.n), "precision": "f32",
                   "scale_div": args.scale_div},
        "ms_per_step_no_events": t32_noev / args.steps * 1e3,
        "hbm_frac_step": val32 * STEP_SCALARS * 4 / (HBM_PEAK_GBS * 1e9),
        "step_roofline": step_roofline(val32, STEP_SCALARS, 4),
        "valu_roofline": valu_roofline(val32),
        "copy_probe": copy,
        "kernels_us": {k: round(v["avg_ms"] * 1e3, 2) for k, v in kernels.items()},
        "f64": out_f64,
        "fwd_adjoint": adj,
        "late_phase": late,
        "variants": variants,
        "other_configs": configs,
        "paper_inverse": paper_inv,
        "paper_context": {"value_f32": 1.22e8, "value_f64": 2.76e7,
                          "note": "paper, one A100, 2,712,960-particle cylinder on 400x400x100; "
                                  "a different machine and grid, not this workload (the variants "
                                  "leg times that case)"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

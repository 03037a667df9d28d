"""Learned fields against the plain per-cell field, trained through the
solver's adjoint on observations that a ground-truth run of the solver
generates (Sec. 3.2 parameter forms; Sec. 5 inverse problems).

Both forms are fitted by Adam to the same loss from the same data, and
each estimate is scored against the seeded ground-truth field, not
against the loss.  The network's
gain is its smoothness: the table fits the observations more tightly (lower
loss) but is piecewise constant, the network recovers the field better."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_learned_initial_velocity_beats_cell_table():
    """Granular block, hidden v0 = four Gaussian bumps; 200 tracer velocities
    and 8 box means every 20 steps over 400 steps (32,768 particles, FP32).
    2-64-64-2 tanh network (BF16 MFMA) vs 16 x 8 table.  The table's best
    possible error (cell means of the hidden field) is 0.131."""
    from paper_2507_04192_amd import inverse as I
    print("[case] learned initial velocity, 2-D granular block", flush=True)
    m = I.learned_velocity_2d(epochs=600, fit=("mlp",), math="bf16", mlp_lr=1e-2, mlp_decay=0.998)["mlp"]
    c = I.learned_velocity_2d(epochs=300, fit=("cells",), cell_lr=0.1, cell_decay=0.99)["cells"]
    print(f"  network: field error {m['start_err']:.3f} -> {m['field_err']:.3f}, loss {m['loss'][0]:.3e} -> "
          f"{m['loss'][-1]:.3e} ({m['seconds']:.1f} s)", flush=True)
    print(f"  table:   field error 1.000 -> {c['field_err']:.3f}, loss {c['loss'][0]:.3e} -> {c['loss'][-1]:.3e} "
          f"({c['seconds']:.1f} s)", flush=True)
    assert m["loss"][-1] < 0.01 * m["loss"][0]
    assert c["loss"][-1] < 0.01 * c["loss"][0]
    assert m["field_err"] < 0.2
    assert m["field_err"] < 0.75 * c["field_err"]


def test_learned_friction_small_dam_break():
    """Hidden base friction under a 3-D dam-break shrunk 4x (28,800
    particles, 1000 steps, checkpoint every 100): 2-128-128-1 sigmoid
    network vs 24 x 12 table, both from mu = 0.5, 20 epochs.  Errors over
    the floor under the initial column."""
    from paper_2507_04192_amd import inverse as I
    print("[case] learned friction, 3-D dam-break / 4", flush=True)
    r = I.learned_friction_3d(scale_div=4, steps=1000, epochs=20, cells=(24, 12))
    m, c = r["mlp"], r["cells"]
    print(f"  network: field error {m['start_err']:.3f} -> {m['field_err']:.3f}, loss {m['loss'][0]:.3e} -> "
          f"{m['loss'][-1]:.3e}", flush=True)
    print(f"  table:   field error {m['start_err']:.3f} -> {c['field_err']:.3f}, loss {c['loss'][0]:.3e} -> "
          f"{c['loss'][-1]:.3e}", flush=True)
    print(f"  device memory high-water mark {r['max_memory_allocated'] / 2**20:.0f} MiB", flush=True)
    assert m["loss"][-1] < 0.5 * m["loss"][0] and c["loss"][-1] < 0.5 * c["loss"][0]
    assert m["field_err"] < 0.6 * m["start_err"]
    assert m["field_err"] < c["field_err"]


def test_learned_friction_full_size():
    """The learned base-friction problem at its full size (1,843,200
    particles, 192 x 96 x 64 cells, 2000 steps, checkpoint every 100) with
    500 tracers observed every 20 steps (100 frames): network and table
    from mu = 0.5 for 20 epochs each."""
    from paper_2507_04192_amd import inverse as I
    print("[case] learned friction, full 3-D dam-break, frames every 20 steps", flush=True)
    r = I.learned_friction_3d(scale_div=1, steps=2000, epochs=20)
    m, c = r["mlp"], r["cells"]
    print(f"  network: field error {m['start_err']:.3f} -> {m['field_err']:.3f}, loss {m['loss'][0]:.3e} -> "
          f"{m['loss'][-1]:.3e} ({m['seconds']:.1f} s)", flush=True)
    print(f"  table:   field error {m['start_err']:.3f} -> {c['field_err']:.3f}, loss {c['loss'][0]:.3e} -> "
          f"{c['loss'][-1]:.3e} ({c['seconds']:.1f} s)", flush=True)
    print(f"  workspace {r['workspace_bytes'] / 2**30:.1f} GiB, high-water mark "
          f"{r['max_memory_allocated'] / 2**30:.1f} GiB", flush=True)
    assert m["loss"][-1] < 0.5 * m["loss"][0] and c["loss"][-1] < 0.5 * c["loss"][0]
    assert m["field_err"] < 0.75 * m["start_err"]
    assert m["field_err"] < c["field_err"]

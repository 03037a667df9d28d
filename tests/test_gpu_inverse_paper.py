"""The paper's inverse experiments (Sec. 5.1-5.3) as synthetic
reproductions, trained through the HIP adjoint on observations that a
ground-truth run of the solver generates: bounded epoch counts, each
problem held to recovering its hidden parameters within a stated error.

- Sec. 5.1: the scalar alpha of v_x = alpha (H0 - y), truth 2, start 0.1,
  supervised by the nine Eulerian velocity monitors (case 3) over the last
  100 frames of 10,000 steps (the two Lagrangian cases run the same code
  with other observations; their full runs are recorded with the design).
- Sec. 5.2: the velocity profile as a 1-30-30-30-1 ReLU network from the
  positions of 1000 particles.
- Sec. 5.3: the Coulomb friction of four floor segments (truth 0.0, 0.5,
  0.1, 0.2) from 500 tracers at 1000 frames.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# Epoch counts and bounds from full runs on the MI355X (Adam from lr 0.1,
# decay 0.98 per epoch): alpha reaches 2.04 (monitors) and 2.06 (100
# particles) after 60 epochs, overshooting to 2.19 / 2.10 on the way; the
# segments are within 0.015 of the truth after 80 epochs with 500 tracers;
# the profile network's error is 0.054 after 120 epochs (1000 particles).
EPOCHS_ALPHA, ALPHA_TOL = 60, 0.1
EPOCHS_SEGMENTS, SEGMENT_TOL = 80, 0.03
EPOCHS_PROFILE, PROFILE_TOL = 120, 0.1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("case", [3])
def test_initial_velocity_constant(case):
    from paper_2507_04192_amd import inverse as I
    print(f"[case] Sec. 5.1 alpha, observation case {case}", flush=True)
    r = I.alpha_inverse(case, epochs=EPOCHS_ALPHA)
    a = r["alpha"]
    print(f"  alpha {a[0]:.3f} -> {a[-1]:.4f} (truth 2), loss {r['loss'][0]:.3e} -> {r['loss'][-1]:.3e}, "
          f"{r['seconds']:.1f} s", flush=True)
    assert abs(a[-1] - 2.0) <= ALPHA_TOL
    assert r["loss"][-1] < 5e-3 * r["loss"][0]


def test_velocity_profile_network():
    from paper_2507_04192_amd import inverse as I
    print("[case] Sec. 5.2 velocity profile, 1000 observed particles", flush=True)
    r = I.profile_inverse(n_obs=1000, epochs=EPOCHS_PROFILE)
    print(f"  profile error {r['start_err']:.3f} -> {r['field_err']:.4f}, loss {r['loss'][0]:.3e} -> "
          f"{r['loss'][-1]:.3e}, {r['seconds']:.1f} s", flush=True)
    assert r["field_err"] <= PROFILE_TOL


def test_friction_segments():
    from paper_2507_04192_amd import inverse as I
    print("[case] Sec. 5.3 four friction segments, 500 tracers", flush=True)
    r = I.friction_segments_inverse(n_tracers=500, epochs=EPOCHS_SEGMENTS)
    mu = np.asarray(r["mu"][-1])
    true = np.asarray(r["mu_true"])
    print(f"  mu {np.round(mu, 4).tolist()} (truth {true.tolist()}), loss {r['loss'][0]:.3e} -> "
          f"{r['loss'][-1]:.3e}, {r['seconds']:.1f} s", flush=True)
    assert np.abs(mu - true).max() <= SEGMENT_TOL

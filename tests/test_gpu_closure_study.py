"""End-to-end learned-closure workflow at a small size on the GPU: a fine
channel run generates box-filtered training data, the network is trained by
the library's own forward/backward/Adam kernels, and the result is compared
with the Smagorinsky closure a priori (held-out snapshot) and a posteriori
(coarse runs against the filtered fine run)."""
import math

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_closure_study_small():
    from paper_2305_09910_amd import closure
    cfg = closure.ClosureConfig(coarse=(32, 16, 16), factor=4, tau_c=0.51, noise=0.3, spinup=300, snapshots=3,
                                every=100, train_steps=300, batch=8192, lr=3e-3, eval_coarse_steps=40)
    res, P = closure.study(cfg, log=print)
    ap = res["a_priori_heldout"]
    print(res)
    # the trained network predicts the filtered-fine correction better than
    # the Smagorinsky correction and better than no correction
    assert ap["mse_mlp"] < ap["mse_smagorinsky"]
    assert ap["mse_mlp"] < ap["mse_zero"]
    hist = res["loss_history"]
    assert hist[-1][1] < hist[0][1]
    post = res["a_posteriori"]
    for name in ("smagorinsky", "mlp"):
        assert post[name]["finite"] and math.isfinite(post[name]["l2_velocity_error"])


def test_closure_beats_smagorinsky_a_posteriori_vortical_channel():
    """One-sided a-posteriori test.  With a vortical start (band-limited
    solenoidal perturbation, rms 0.02, peak wavelength 16 fine cells) the
    filtered fine flow has a resolved subgrid stress.  Coarse 64x32x32
    against the filtered 256x128x128 run, 100 coarse steps.  The network is
    trained on 3 x the a-priori target dtau* (the scale chosen on a separate
    validation seed at full size: a-priori targets under-supply the
    dissipation the coarse lattice needs).  Its coarse run is closer to the
    filtered fine run than the Smagorinsky run (Cs = 0.1) and the run without
    a model.  Measured over seeds 1234, 99, 7: 3.4% below Smagorinsky,
    6.0-6.1% below no model (with the unscaled target: 0.08-0.19% below
    Smagorinsky); the bounds leave margin."""
    from paper_2305_09910_amd import closure
    cfg = closure.ClosureConfig(coarse=(64, 32, 32), factor=4, tau_c=0.503, noise=0.05, vortical_rms=0.02,
                                vortical_wavelength=16, seed=1234, spinup=400, snapshots=3, every=200,
                                train_steps=400, batch=16384, lr=2e-3, eval_coarse_steps=100, target_scale=3.0)
    res, _ = closure.study(cfg, log=print)
    post = {k: v["l2_velocity_error"] for k, v in res["a_posteriori"].items()}
    print(post)
    assert post["mlp"] < 0.99 * post["smagorinsky"]
    assert post["mlp"] < 0.97 * post["none"]


def test_closure_study_with_lattice_features():
    """Training inputs taken from coarse lattices' own populations
    (lbm_closure_features after 25 coarse steps from an earlier filtered
    state) instead of the filtered strain: the network then meets the input
    distribution it was trained on, so almost no cell update falls back to
    Smagorinsky (measured: none; with filtered-strain inputs 7.5-8.7%
    fall back at this size), and the run stays finite."""
    from paper_2305_09910_amd import closure
    cfg = closure.ClosureConfig(coarse=(64, 32, 32), factor=4, tau_c=0.503, noise=0.05, vortical_rms=0.02,
                                vortical_wavelength=16, seed=1234, spinup=400, snapshots=3, every=200,
                                train_steps=400, batch=16384, lr=2e-3, eval_coarse_steps=100, features="lattice",
                                lead=25)
    res, _ = closure.study(cfg, log=print)
    mlp = res["a_posteriori"]["mlp"]
    assert mlp["finite"] and math.isfinite(mlp["l2_velocity_error"])
    assert mlp["fallback_fraction"] < 0.005

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

"""The allocation-free loss/gradient entry point (static scratch array) against
the entry point that takes a caller workspace: same kernels, so the same
results bit for bit, on two calls in a row, the second with a smaller batch
(the scratch keeps the first call's partials and must not leak them)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.normal(0, 0.4, 192), rng.normal(0, 0.2, 32), rng.normal(0, 0.2, 1024),
                        rng.normal(0, 0.2, 32), rng.normal(0, 0.3, 32), [-3.0]])
    norm = np.concatenate([rng.normal(0, 0.3, 6), rng.uniform(0.5, 2.0, 6), np.full(6, -1e30), np.full(6, 1e30)])
    x = rng.normal(0, 1.0, (n, 6))
    t = np.abs(rng.normal(0, 0.05, n))
    f = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")
    return f(np.r_[p, norm]), f(x), f(t)


def test_noalloc_loss_grad_matches_workspace_entry_point():
    from paper_2305_09910_amd import lbm
    params, x, t = _batch(70001, seed=3)
    for n in (70001, 1234):  # second call smaller: stale partials would show
        print(f"[case] mlp_loss_grad_noalloc n={n}", flush=True)
        xs, ts = x[:n].contiguous(), t[:n].contiguous()
        loss_ref, grad_ref = lbm.mlp_loss_grad(params, xs, ts)
        grad = torch.full((1313,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        lbm.mlp_loss_grad_noalloc(params, xs, ts, grad, loss)
        torch.cuda.synchronize()
        assert torch.isfinite(grad).all() and torch.isfinite(loss).all()
        assert torch.equal(grad, grad_ref), float((grad - grad_ref).abs().max())
        assert torch.equal(loss, loss_ref)


def test_noalloc_rejects_bad_arguments():
    from paper_2305_09910_amd import lbm
    L = lbm.lib()
    params, x, t = _batch(10, seed=4)
    grad = torch.empty(1313, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    rc = L.lbm_mlp_loss_grad_noalloc(params.data_ptr(), x.data_ptr(), t.data_ptr(), 0, grad.data_ptr(),
                                     loss.data_ptr(), None)
    assert rc == lbm.LBM_EINVAL
    rc = L.lbm_mlp_loss_grad_noalloc(params.data_ptr(), None, t.data_ptr(), 10, grad.data_ptr(), loss.data_ptr(),
                                     None)
    assert rc == lbm.LBM_EINVAL
    assert b"NULL" in L.lbm_last_error(ctypes.c_void_p(0))

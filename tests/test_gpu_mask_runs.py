"""Masked domains with sparse solids read a cell's mask word only where its
run of 64 cells along x touches a solid (the run words after the mask).
Rows of 100 cells (a full run and a partial one): solids only in the partial
run of some rows, only in the full run of others, and a solid whose cut links
reach cells of neighbouring rows that hold no solid themselves; with velocity
and pressure faces on x.  25 steps against the oracle, D3Q19 and D3Q27, TRT
and MRT, FP32 (1e-6) and the 16-bit forms' bound."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import MRT27_RATES, max_rel, pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (100, 7, 6)
BC = ("velocity", "pressure", "periodic", "periodic", "noslip", "noslip")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solid():
    nx, ny, nz = SHAPE
    s = np.zeros((nz, ny, nx), np.uint8)
    s[1, 2, 70:74] = 1   # partial run only
    s[3, 4, 10:13] = 1   # first run only
    s[4, 0, 63:65] = 1   # across the run boundary, on a periodic y face
    s[2, 6, 99] = 1      # last cell of a row, at the pressure face; cuts links of rows y = 5 and (wrapped) y = 0
    assert s.mean() < 0.2  # sparse: the run words are used
    return s


@pytest.mark.parametrize("q,collision", [(19, "trt"), (27, "trt"), (27, "mrt")])
def test_mask_runs_against_oracle(q, collision):
    solid = _solid()
    uw = np.zeros((6, 3))
    uw[0] = (0.03, 0.0, 0.0)
    kw = dict(mrt_rates=MRT27_RATES) if (collision == "mrt" and q == 27) else {}
    g, o = pair(SHAPE, q=q, tau=0.6, force=(1e-5, 0, 0), bc=BC, u_bc=uw, solid=solid, collision=collision, **kw)
    rng = np.random.default_rng(7 + q)
    nx, ny, nz = SHAPE
    rho = 1 + rng.uniform(-0.01, 0.01, (nz, ny, nx))
    u = rng.uniform(-0.02, 0.02, (3, nz, ny, nx))
    u[:, solid == 1] = 0.0
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    for n in (1, 24):
        g.step(n)
        o.step(n)
        err = max_rel(g.get_pdfs(), o.get_pdfs(), solid)
        print(f"mask runs q={q} {collision} after {n}: max rel err {err:.2e}")
        assert err <= 1e-6, n


@pytest.mark.parametrize("storage,unit", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_mask_runs_16bit(storage, unit):
    solid = _solid()
    uw = np.zeros((6, 3))
    uw[0] = (0.03, 0.0, 0.0)
    g, o = pair(SHAPE, q=19, tau=0.6, force=(1e-5, 0, 0), bc=BC, u_bc=uw, solid=solid, storage=storage)
    g.init_equilibrium(np.ones(SHAPE[::-1]), np.zeros((3,) + SHAPE[::-1]))
    o.init_equilibrium(np.ones(SHAPE[::-1]), np.zeros((3,) + SHAPE[::-1]))
    g.step(2)
    o.step(2)
    a = g.get_pdfs().cpu().numpy()[:, solid == 0]
    b = o.get_pdfs()[:, solid == 0]
    w = oracle.velocity_set(19)[1][:, None]
    dmax = np.abs(b - w).max()
    assert np.all(np.abs(a - b) <= 3 * unit * dmax + 1e-7 * np.abs(b))

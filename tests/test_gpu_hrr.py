"""The hybrid recursive regularised collision (HRR, D3Q19) on the GPU against
the FP64 oracle, element by element: maximum relative population error 1e-5
in FP32 storage, on the Taylor-Green vortex, the channel with walls, every
boundary kind with solids, odd and even step counts, and checkpoints."""
import math

import numpy as np
import pytest

import oracle
from paper_2305_09910_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
BCS = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "velocity": oracle.BC_VELOCITY,
       "pressure": oracle.BC_PRESSURE}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_09910_amd import lbm
    lbm.lib()
    yield
    torch.cuda.synchronize()


def pair(shape, sigma, tau=0.6, force=(0, 0, 0), bc=("periodic",) * 6, u_bc=None, solid=None, storage="f32"):
    from paper_2305_09910_amd import lbm
    print(f"[case] hrr shape={shape} sigma={sigma} tau={tau} bc={bc} solid={solid is not None}", flush=True)
    g = lbm.Lattice(shape, q=19, tau=tau, force=force, bc=bc, u_bc=u_bc, solid=solid, storage=storage,
                    collision="hrr", hrr_sigma=sigma)
    o = oracle.Sim(19, shape, bc=tuple(BCS[b] for b in bc), tau=tau, force=force, u_bc=u_bc, solid=solid)
    o.set_hrr(sigma)
    return g, o


def max_rel(g, o, solid=None):
    a = g.get_pdfs().cpu().numpy()
    b = o.get_pdfs()
    err = np.abs(a - b) / np.abs(b)
    if solid is not None:
        err = err[:, solid.reshape(b.shape[1:]) == 0]
    return float(err.max())


@pytest.mark.parametrize("sigma", [1.0, 0.9])
def test_hrr_taylor_green_32cubed_1000_steps(sigma):
    n, nu = 32, 0.01
    g, o = pair((n, n, n), sigma, tau=3 * nu + 0.5)
    rho, u = inputs.taylor_green(n, n, n, 0.05)
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    k = 2 * math.pi / n
    mode = np.broadcast_to(np.cos(k * np.arange(n)[None, None, :]) * np.sin(k * np.arange(n)[None, :, None]),
                           (n, n, n))

    def amp():
        _, ug = g.moments()
        return float((ug[0].cpu().numpy() * mode).sum() / (mode * mode).sum())

    g.step(100)
    a0 = amp()
    g.step(900)
    o.step(1000)
    err = max_rel(g, o)
    print("HRR TGV err", err)
    assert err <= TOL32
    # decay rate exp(-2 nu k^2 t) over t in [100, 1000], past the start-up
    # transient (the oracle pin measures the same window)
    rate = -math.log(amp() / a0) / 900 / (2 * k * k)
    assert abs(rate / nu - 1) < 0.01


def test_hrr_channel_1000_steps():
    """The channel copy (walls on y, force in x, parabola plus 5% noise),
    64x32x32, tau = 0.51, sigma = 0.995, 1000 steps."""
    nx, ny, nz = 64, 32, 32
    F = 8 * (1 / 300) * 0.05 / ny ** 2
    g, o = pair((nx, ny, nz), 0.995, tau=0.51, force=(F, 0, 0),
                bc=("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"))
    rho, u = inputs.channel(nx, ny, nz, 0.05, 0.05, seed=1234)
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    g.step(1000)
    o.step(1000)
    err = max_rel(g, o)
    print("HRR channel err", err)
    assert err <= TOL32
    mg, _ = g.totals()
    mo, _ = o.totals()
    assert abs(mg - mo) / mo < 1e-7
    assert abs(mg - nx * ny * nz) / (nx * ny * nz) < 1e-7  # FP32 mass drift after 1000 steps


@pytest.mark.parametrize("nsteps", [1, 2, 11, 60])
def test_hrr_every_boundary_kind_and_solids(nsteps):
    """Velocity inlet and pressure outlet on x, no-slip on y, periodic z, and
    a solid block: the gradient's wall rules on every kind of neighbour."""
    shape = (24, 14, 10)
    solid = np.zeros(shape[::-1], np.uint8)
    solid[3:7, 5:9, 9:13] = 1
    uw = np.zeros((6, 3))
    uw[0] = (0.04, 0.005, -0.003)
    g, o = pair(shape, 0.9, tau=0.58, force=(2e-6, 0, 0), u_bc=uw, solid=solid,
                bc=("velocity", "pressure", "noslip", "noslip", "periodic", "periodic"))
    rho, u = inputs.channel(*shape, 0.04, 0.1, seed=5)
    u[:, solid == 1] = 0
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    g.step(nsteps)
    o.step(nsteps)
    err = max_rel(g, o, solid)
    print("HRR all-bc err", err)
    assert err <= TOL32


def test_hrr_set_pdfs_odd_shape_and_checkpoint():
    """A non-equilibrium start through lbm_set_pdfs on a ragged shape; a
    checkpoint taken after an odd step resumes bit for bit (the state holds
    the velocity fields of the gradient too)."""
    shape = (37, 9, 6)
    bc = ("periodic", "periodic", "noslip", "velocity", "periodic", "periodic")
    uw = np.zeros((6, 3))
    uw[3] = (0.03, 0, 0)
    g, o = pair(shape, 0.95, tau=0.7, force=(1e-5, 0, 0), bc=bc, u_bc=uw)
    c, w, _ = oracle.velocity_set(19)
    f = w[:, None, None, None] * (1 + inputs.perturbation((19,) + shape[::-1], 0.02, seed=8))
    g.set_pdfs(f)
    o.set_pdfs(f)
    g.step(7)
    o.step(7)
    assert max_rel(g, o) <= TOL32
    buf, t = g.save_state()
    g.step(20)
    ref = g.get_pdfs().clone()
    g.load_state(buf, t)
    g.step(20)
    assert torch.equal(g.get_pdfs(), ref)
    o.step(20)
    assert max_rel(g, o) <= TOL32


@pytest.mark.parametrize("storage,bound", [("f16", 1e-2), ("bf16", 5e-2)])
def test_hrr_low_precision_storage(storage, bound):
    """16-bit deviation storage with HRR: velocity L2 error against the FP64
    oracle on the 64x32x32 channel after 1000 steps, within the bounds of the
    16-bit forms of the other collisions."""
    nx, ny, nz = 64, 32, 32
    F = 8 * (1 / 300) * 0.05 / ny ** 2
    g, o = pair((nx, ny, nz), 0.995, tau=0.51, force=(F, 0, 0), storage=storage,
                bc=("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"))
    rho, u = inputs.channel(nx, ny, nz, 0.05, 0.05, seed=1234)
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    g.step(1000)
    o.step(1000)
    _, ug = g.moments()
    _, uo = o.moments()
    l2 = float(np.sqrt(((ug.cpu().numpy() - uo) ** 2).sum() / (uo ** 2).sum()))
    print(f"HRR {storage} velocity L2", l2)
    assert l2 < bound

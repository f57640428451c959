"""GPU at the full benchmark shapes, in the launch configuration the
benchmark times, against the oracle on sampled cells.

The GPU runs two steps (one even, one odd kernel) from f^eq of the seeded
fields; the oracle's probe computes the same two steps for each sampled
cell alone (its dependence cone), with no full-size lattice.  Samples mix
random fluid cells with every corner/edge/face class and cells next to
solids.  Properties that hold at any size (mass conservation, determinism)
are checked over longer runs.
"""
import numpy as np
import pytest

import oracle
from paper_2305_09910_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WALLS_Y = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")
INOUT_X = ("velocity", "pressure", "periodic", "periodic", "periodic", "periodic")
BCS = {"periodic": 0, "noslip": 1, "velocity": 2, "pressure": 3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(name):
    if name.startswith("channel"):
        nx, ny, nz = {"channel_256x128x128": (256, 128, 128), "channel_512x256x256": (512, 256, 256)}[name]
        F = 8 * (1 / 300) * 0.05 / ny ** 2
        rho, u = inputs.channel(nx, ny, nz, 0.05, 0.05, seed=1234)
        return dict(shape=(nx, ny, nz), q=19, tau=0.51, force=(F, 0, 0), bc=WALLS_Y, solid=None, u_bc=None), rho, u
    if name == "porous_256":
        # the porous-medium benchmark: 70% solid, periodic, force-driven
        n = 256
        solid = inputs.porous(n, n, n, solid_fraction=0.7, rmin=3.0, rmax=8.0, seed=77)
        rho, u = inputs.uniform_flow(n, n, n, (0.0, 0, 0))
        u += inputs.perturbation(u.shape, 0.002, seed=98) * (solid == 0)
        return dict(shape=(n, n, n), q=19, tau=0.6, force=(1e-5, 0, 0), bc=("periodic",) * 6, solid=solid,
                    u_bc=None), rho, u
    n = 384
    solid, _ = inputs.spheres(n, n, n, fill=0.10, x_margin=32, seed=2024)
    uw = np.zeros((6, 3))
    uw[0] = (0.04, 0, 0)
    rho, u = inputs.uniform_flow(n, n, n, (0.04, 0, 0))
    u[:, solid == 1] = 0.0
    # seeded noise so that the first collisions already see non-equilibrium neighbours
    u += inputs.perturbation(u.shape, 0.002, seed=99) * (solid == 0)
    return dict(shape=(n, n, n), q=27, tau=0.56, force=(0, 0, 0), bc=INOUT_X, solid=solid, u_bc=uw), rho, u


def _samples(shape, solid, n_random=1500, seed=0):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    pts = [rng.integers(0, [nx, ny, nz], size=(n_random, 3))]
    # every corner/edge/face class of the box
    for xs in (0, 1, nx // 2, nx - 2, nx - 1):
        for ys in (0, 1, ny // 2, ny - 2, ny - 1):
            for zs in (0, nz // 2, nz - 1):
                pts.append(np.array([[xs, ys, zs]]))
    p = np.concatenate(pts)
    cells = (p[:, 2] * ny + p[:, 1]) * nx + p[:, 0]
    if solid is not None:
        flat = solid.reshape(-1)
        # fluid cells touching a solid
        sol = np.flatnonzero(flat)
        near = []
        for d in (1, -1, nx, -nx, nx * ny, -nx * ny):
            c = sol + d
            c = c[(c >= 0) & (c < flat.size)]
            near.append(c[flat[c] == 0])
        near = np.unique(np.concatenate(near))
        cells = np.concatenate([cells, rng.choice(near, 1000, replace=False)])
        cells = cells[flat[cells] == 0]
    return np.unique(cells)


@pytest.mark.parametrize("name,storage,collision", [
    ("channel_256x128x128", "f32", "trt"),
    ("channel_512x256x256", "f32", "trt"),
    ("channel_512x256x256", "f16", "trt"),
    ("channel_512x256x256", "bf16", "trt"),
    ("obstacles_384_d3q27", "f32", "trt"),
    ("channel_512x256x256", "f32", "mrt"),
    ("obstacles_384_d3q27", "f32", "mrt"),
])
def test_two_steps_sampled_against_probe(name, storage, collision):
    from paper_2305_09910_amd import lbm
    cfg, rho, u = _case(name)
    print(f"[case] {name} storage={storage} collision={collision}", flush=True)
    rates = (1.6, 1.75, 1.55, 1.65, 1.7) if cfg["q"] == 27 else oracle.MRT_DHUMIERES
    g = lbm.Lattice(cfg["shape"], q=cfg["q"], tau=cfg["tau"], force=cfg["force"], bc=cfg["bc"],
                    u_bc=cfg["u_bc"], solid=cfg["solid"], storage=storage, collision=collision, mrt_rates=rates)
    g.init_equilibrium(rho, u)
    g.step(2)
    cells = _samples(cfg["shape"], cfg["solid"])
    got = g.gather(cells).cpu().numpy()
    o = oracle.Sim(cfg["q"], cfg["shape"], bc=tuple(BCS[b] for b in cfg["bc"]), tau=cfg["tau"], force=cfg["force"],
                   u_bc=cfg["u_bc"], solid=cfg["solid"])
    if collision == "mrt":
        o.set_mrt(rates)
    ref = o.probe(rho, u, 2, cells)
    c, w, _ = oracle.velocity_set(cfg["q"])
    err = np.abs(got - ref)
    if storage == "f32":
        bound = 1e-6 * np.abs(ref)
    else:
        # three roundings (initial state, two stores) of a deviation of size
        # |f - w| with unit roundoff 2^-11 (FP16) or 2^-8 (BF16)
        unit = 2.0 ** -11 if storage == "f16" else 2.0 ** -8
        dmax = np.abs(ref - w[None, :]).max()
        bound = 3 * unit * dmax + 1e-7 * np.abs(ref)
    print(name, storage, "max abs err", err.max(), "max rel", (err / np.abs(ref)).max())
    assert np.all(err <= bound)
    del g
    torch.cuda.empty_cache()


def _timing_network(seed=9):
    """The seeded network the benchmark times the fused closure with: smooth
    weights, inputs standardised to unit scale, unbounded trusted range."""
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.normal(0, 0.3, 192), rng.normal(0, 0.1, 32), rng.normal(0, 0.15, 1024),
                        rng.normal(0, 0.1, 32), rng.normal(0, 0.1, 32), [-5.0]])
    norm = np.concatenate([np.zeros(6), [1e-3, 1e-3, 1e-3, 1e-2, 1e-2, 1.0], np.full(6, -1e30), np.full(6, 1e30)])
    return p.astype(np.float32), norm.astype(np.float32)


@pytest.mark.parametrize("name,storage,streaming,closure", [
    ("channel_256x128x128", "f32", "aa", "smagorinsky"),
    ("channel_256x128x128", "f32", "aa", "mlp"),
    ("channel_512x256x256", "f32", "aa", "mlp"),
    ("channel_256x128x128", "f32", "et", "none"),
    ("channel_256x128x128", "f32", "et", "mlp"),
    ("channel_512x256x256", "f32", "et", "none"),
    ("channel_512x256x256", "f16", "et", "none"),
    ("obstacles_384_d3q27", "f32", "et", "none"),
    ("porous_256", "f32", "aa", "none"),
    ("porous_256", "f32", "sparse", "none"),
    ("porous_256", "f16", "sparse", "none"),
    ("porous_256", "f32", "sparse", "mlp"),
    ("obstacles_384_d3q27", "f32", "sparse", "none"),
])
def test_closure_et_and_sparse_forms_sampled_against_probe(name, storage, streaming, closure):
    """The closure forms, the Esoteric Twist forms and the sparse-addressing
    forms at their benchmark shapes: two steps, sampled cells against the
    oracle's probe."""
    from paper_2305_09910_amd import lbm
    cfg, rho, u = _case(name)
    print(f"[case] {name} storage={storage} streaming={streaming} closure={closure}", flush=True)
    g = lbm.Lattice(cfg["shape"], q=cfg["q"], tau=cfg["tau"], force=cfg["force"], bc=cfg["bc"], u_bc=cfg["u_bc"],
                    solid=cfg["solid"], storage=storage, closure=closure, cs=0.1, streaming=streaming)
    ocl = {"none": oracle.CL_NONE, "smagorinsky": oracle.CL_SMAG, "mlp": oracle.CL_MLP}[closure]
    o = oracle.Sim(cfg["q"], cfg["shape"], bc=tuple(BCS[b] for b in cfg["bc"]), tau=cfg["tau"], force=cfg["force"],
                   u_bc=cfg["u_bc"], solid=cfg["solid"], closure=ocl, cs=0.1)
    if closure == "mlp":
        p, norm = _timing_network()
        g.set_closure_weights(np.concatenate([p, norm]))
        o.set_mlp(p, norm)
    g.init_equilibrium(rho, u)
    g.step(2)
    cells = _samples(cfg["shape"], cfg["solid"])
    got = g.gather(cells).cpu().numpy()
    ref = o.probe(rho, u, 2, cells)
    c, w, _ = oracle.velocity_set(cfg["q"])
    err = np.abs(got - ref)
    if storage == "f32":
        # the closures' FP32 features and rates (hardware reciprocal and
        # square root) sit a few ulp from the oracle's FP64 values
        bound = (1e-6 if closure == "none" else 2e-6) * np.abs(ref)
    else:
        unit = 2.0 ** -11
        dmax = np.abs(ref - w[None, :]).max()
        bound = 3 * unit * dmax + 1e-7 * np.abs(ref)
    print(name, storage, streaming, closure, "max abs err", err.max(), "max rel", (err / np.abs(ref)).max())
    assert np.all(err <= bound)
    if closure == "mlp":
        assert g.closure_fallbacks() == 0
    del g
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["channel_256x128x128", "channel_512x256x256"])
def test_mass_conserved_and_deterministic_at_full_size(name):
    from paper_2305_09910_amd import lbm
    cfg, rho, u = _case(name)
    print(f"[case] {name} 200 steps mass + determinism", flush=True)
    kw = dict(q=cfg["q"], tau=cfg["tau"], force=cfg["force"], bc=cfg["bc"])
    g = lbm.Lattice(cfg["shape"], **kw)
    g.init_equilibrium(rho, u)
    m0, _ = g.totals()
    g.step(200)
    m1, p1 = g.totals()
    n = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    assert abs(m1 - m0) / n < 1e-6
    h = lbm.Lattice(cfg["shape"], **kw)
    h.init_equilibrium(rho, u)
    h.step(200)
    m2, p2 = h.totals()
    assert m1 == m2 and np.array_equal(p1, p2)
    del g, h
    torch.cuda.empty_cache()

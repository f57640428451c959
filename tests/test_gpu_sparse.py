"""Sparse addressing (the AA pattern over the fluid cells only) on the GPU,
beyond the oracle parity cases of test_gpu_parity.py (which run every
scheme): porous media against the oracle, agreement with the dense AA
kernel in every storage format, with every boundary kind and with the
learned closure, and the state functions."""
import numpy as np
import pytest

import oracle
from paper_2305_09910_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BCS = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "velocity": oracle.BC_VELOCITY,
       "pressure": oracle.BC_PRESSURE}
INOUT = ("velocity", "pressure", "noslip", "noslip", "periodic", "periodic")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_09910_amd import lbm
    lbm.lib()
    yield
    torch.cuda.synchronize()


def _medium(shape, fraction, seed):
    solid = inputs.porous(*shape, solid_fraction=fraction, rmin=2.0, rmax=4.5, seed=seed)
    rho, u = inputs.uniform_flow(*shape, (0.01, 0.0, 0.0))
    u += inputs.perturbation(u.shape, 0.004, seed=seed + 1)
    u[:, solid == 1] = 0.0
    return solid, rho, u


def _max_rel(g, o, solid):
    a = g.get_pdfs().cpu().numpy()
    b = o.get_pdfs()
    fl = solid == 0
    return float(np.max(np.abs(a[:, fl] - b[:, fl]) / np.abs(b[:, fl])))


@pytest.mark.parametrize("q,collision,closure,walls", [
    (19, "trt", "none", "periodic"),
    (27, "trt", "none", "periodic"),
    (19, "mrt", "none", "inout"),
    (27, "trt", "smagorinsky", "inout"),
    (19, "trt", "smagorinsky", "periodic"),
    (27, "mrt", "none", "inout"),
])
def test_porous_medium_against_oracle(q, collision, closure, walls):
    """A force-driven periodic porous medium (the solid-heavy case sparse
    addressing is for, 60% solid) and an inlet/outlet duct through it:
    300 steps in FP32 against the oracle, 1e-5 max relative error."""
    from paper_2305_09910_amd import lbm
    shape = (40, 24, 20)
    solid, rho, u = _medium(shape, 0.6, seed=q + len(walls))
    bc = ("periodic",) * 6 if walls == "periodic" else INOUT
    uw = np.zeros((6, 3))
    uw[0] = (0.01, 0.0, 0.0)
    rates = (1.6, 1.75, 1.55, 1.65, 1.7) if q == 27 else oracle.MRT_DHUMIERES
    force = (2e-5, 0, 1e-6) if walls == "periodic" else (0, 0, 0)
    print(f"[case] q={q} {collision} {closure} {walls}", flush=True)
    g = lbm.Lattice(shape, q=q, tau=0.6, force=force, bc=bc, u_bc=uw, solid=solid, closure=closure,
                    collision=collision, mrt_rates=rates, streaming="sparse")
    cl = {"none": oracle.CL_NONE, "smagorinsky": oracle.CL_SMAG}[closure]
    o = oracle.Sim(q, shape, bc=tuple(BCS[b] for b in bc), tau=0.6, force=force, u_bc=uw, solid=solid, closure=cl)
    if collision == "mrt":
        o.set_mrt(rates)
    g.init_equilibrium(rho, u)
    o.init_equilibrium(rho, u)
    for n in (299, 300):  # an odd and an even step count
        g.step(n - g.time)
        o.step(n - (0 if n == 299 else 299))
        err = _max_rel(g, o, solid)
        print(f"n={n}: max rel err {err:.3e}")
        assert err <= 1e-5


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_sparse_agrees_with_dense(q, storage):
    """Same collision on the same values: the sparse and dense AA kernels
    differ only by the FP32 rounding order each kernel's compiled code
    takes, with solids, velocity / pressure / no-slip faces and a force,
    after odd and even step counts (the bound of the Esoteric Twist
    comparison: n steps of a few ulps of the storage format)."""
    from paper_2305_09910_amd import lbm
    shape = (44, 20, 14)
    solid, rho, u = _medium(shape, 0.5, seed=5 * q)
    uw = np.zeros((6, 3))
    uw[0] = (0.01, 0.001, 0.0)
    kw = dict(q=q, tau=0.58, force=(1e-5, 0, -2e-6), bc=INOUT, u_bc=uw, solid=solid, storage=storage)
    print(f"[case] q={q} storage={storage}", flush=True)
    a = lbm.Lattice(shape, streaming="aa", **kw)
    s = lbm.Lattice(shape, streaming="sparse", **kw)
    a.init_equilibrium(rho, u)
    s.init_equilibrium(rho, u)
    fluid = torch.as_tensor(solid == 0, device=a.device)
    w = torch.as_tensor(oracle.velocity_set(q)[1], device=a.device, dtype=torch.float64)[:, None, None, None]
    for n in (1, 50, 51):
        a.step(n - a.time)
        s.step(n - s.time)
        fa, fs = a.get_pdfs(), s.get_pdfs()
        diff = float((fa - fs)[:, fluid].abs().max())
        if storage == "f32":
            bound = n * 4 * 2.0 ** -24 * float(fa[:, fluid].abs().max())
        else:
            dmax = float((fa - w)[:, fluid].abs().max())
            rel = 2.0 ** -10 if storage == "f16" else 2.0 ** -7
            bound = n * 2 * rel * 2.0 ** np.floor(np.log2(dmax))
        print(f"n={n}: max |f_dense - f_sparse| = {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound, (n, diff, bound)
        # solid cells report w_i in both
        assert torch.equal(fa[:, ~fluid], fs[:, ~fluid])
    ma, pa = a.totals()
    ms, ps = s.totals()
    assert abs(ma - ms) <= 1e-6 * ma and np.abs(pa - ps).max() <= 1e-6 * ma


def test_state_functions_and_checkpoint():
    """Moments, gather, set/get round trip, totals and save/load on a porous
    medium with sparse addressing; the stored state is sized by the fluid
    cells."""
    from paper_2305_09910_amd import lbm
    shape = (36, 20, 12)
    solid, rho, u = _medium(shape, 0.65, seed=3)
    kw = dict(tau=0.62, force=(1e-5, 0, 0), solid=solid)
    d = lbm.Lattice(shape, **kw)
    s = lbm.Lattice(shape, streaming="sparse", **kw)
    for g in (d, s):
        g.init_equilibrium(rho, u)
        g.step(37)
    assert s.state_bytes() < d.state_bytes() / 2
    rd, ud = d.moments()
    rs, us = s.moments()
    assert float((rd - rs).abs().max()) < 1e-6 and float((ud - us).abs().max()) < 1e-6
    cells = np.arange(0, d.n, 7, dtype=np.int64)
    assert float((d.gather(cells) - s.gather(cells)).abs().max()) < 1e-6
    md, _ = d.totals()
    ms, _ = s.totals()
    assert abs(md - ms) < 1e-6 * md
    # odd step count: the canonical view goes through the neighbour table
    f = s.get_pdfs()
    t = lbm.Lattice(shape, streaming="sparse", **kw)
    t.set_pdfs(f.cpu().numpy())
    assert torch.equal(t.get_pdfs(), f)
    buf, tm = s.save_state()
    s.step(20)
    t.load_state(buf, tm)
    t.step(20)
    assert torch.equal(t.get_pdfs(), s.get_pdfs())


@pytest.mark.parametrize("q", [19, 27])
def test_learned_closure_in_porous_medium(q):
    """The learned closure fused into the sparse kernel on a 50%-solid porous
    medium with inlet/outlet faces: against the dense AA kernel (the same
    network on the same values; FP32 rounding order only) and against the
    oracle (1e-5), with no fallbacks.  The fluid count is not a multiple of
    64, so the last wavefront carries idle lanes through the network."""
    from paper_2305_09910_amd import lbm
    from test_gpu_closure import _smooth_net
    shape = (44, 20, 14)
    solid, rho, u = _medium(shape, 0.5, seed=7 * q)
    assert int((solid == 0).sum()) % 64 != 0
    uw = np.zeros((6, 3))
    uw[0] = (0.01, 0.001, 0.0)
    kw = dict(q=q, tau=0.56, force=(1e-5, 0, -2e-6), bc=INOUT, u_bc=uw, solid=solid, closure="mlp", cs=0.1)
    print(f"[case] q={q} mlp", flush=True)
    p, norm = _smooth_net()
    a = lbm.Lattice(shape, streaming="aa", **kw)
    s = lbm.Lattice(shape, streaming="sparse", **kw)
    for g in (a, s):
        g.set_closure_weights(np.r_[p, norm].astype(np.float32))
        g.init_equilibrium(rho, u)
    o = oracle.Sim(q, shape, bc=tuple(BCS[b] for b in INOUT), tau=0.56, force=(1e-5, 0, -2e-6), u_bc=uw, solid=solid,
                   closure=oracle.CL_MLP, cs=0.1)
    o.set_mlp(p.astype(np.float32), norm.astype(np.float32))
    o.init_equilibrium(rho, u)
    fluid = torch.as_tensor(solid == 0, device=a.device)
    for n in (1, 40, 41):
        a.step(n - a.time)
        s.step(n - s.time)
        o.step(n - (0 if n == 1 else (1 if n == 40 else 40)))
        fa, fs = a.get_pdfs(), s.get_pdfs()
        diff = float((fa - fs)[:, fluid].abs().max())
        bound = n * 4 * 2.0 ** -24 * float(fa[:, fluid].abs().max())
        err = _max_rel(s, o, solid)
        print(f"n={n}: max |f_dense - f_sparse| = {diff:.3e} (bound {bound:.3e}), vs oracle {err:.3e}")
        assert diff <= bound and err <= 1e-5
    assert a.closure_fallbacks() == 0 and s.closure_fallbacks() == 0

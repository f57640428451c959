"""Esoteric Twist streaming on the GPU beyond the oracle parity cases of
test_gpu_parity.py (which run every scheme): the Esoteric Twist and the AA
pattern give the same populations, in every storage format, with every
closure (the learned one included)."""
import numpy as np
import pytest

from paper_2305_09910_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_09910_amd import lbm
    lbm.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_et_agrees_with_aa(q, storage):
    """Same collision on the same values: AA and the Esoteric Twist differ
    only by the FP32 rounding order the compiler picks in each kernel, with
    solids, velocity / pressure / no-slip faces (ghost layers on x and y) and
    a force, after odd and even step counts.

    Bound after n steps: each step may round each value differently by a few
    ulps of its storage format, and the differences stay at most linear in n
    for a stable run.  FP32: n * 4 * 2^-24 * max|f|; 16-bit: n * 2 * ulp of
    the largest stored deviation (2^-10 and 2^-7 relative for FP16 / BF16)."""
    from paper_2305_09910_amd import lbm
    shape = (40, 18, 12)
    solid = np.zeros(shape[::-1], np.uint8)
    solid[3:7, 5:9, 10:15] = 1
    solid[:, 0, 20] = 1
    uw = np.zeros((6, 3))
    uw[0] = (0.03, 0.002, 0.0)
    kw = dict(q=q, tau=0.58, force=(1e-5, 0, -2e-6), bc=("velocity", "pressure", "noslip", "noslip", "periodic",
                                                          "periodic"), u_bc=uw, solid=solid, storage=storage)
    print(f"[case] q={q} storage={storage}", flush=True)
    a = lbm.Lattice(shape, streaming="aa", **kw)
    e = lbm.Lattice(shape, streaming="et", **kw)
    rho, u = inputs.uniform_flow(*shape, (0.03, 0.0, 0.0))
    u += inputs.perturbation(u.shape, 0.005, seed=q)
    u[:, solid == 1] = 0.0
    a.init_equilibrium(rho, u)
    e.init_equilibrium(rho, u)
    fluid = torch.as_tensor(solid == 0, device=a.device)
    w = torch.as_tensor(lbm_weights(q), device=a.device, dtype=torch.float64)[:, None, None, None]
    for n in (1, 50, 51):
        a.step(n - a.time)
        e.step(n - e.time)
        fa, fe = a.get_pdfs(), e.get_pdfs()
        diff = float((fa - fe)[:, fluid].abs().max())
        if storage == "f32":
            bound = n * 4 * 2.0 ** -24 * float(fa[:, fluid].abs().max())
        else:
            dmax = float((fa - w)[:, fluid].abs().max())
            rel = 2.0 ** -10 if storage == "f16" else 2.0 ** -7
            bound = n * 2 * rel * 2.0 ** np.floor(np.log2(dmax))
        print(f"n={n}: max |f_aa - f_et| = {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound, (n, diff, bound)
    ma, pa = a.totals()
    me, pe = e.totals()
    assert abs(ma - me) <= 1e-6 * ma and np.abs(pa - pe).max() <= 1e-6 * ma


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_paired_16bit_even_step(q, storage):
    """16-bit storage without a mask on rows of a multiple of 128 cells: the
    AA even step runs two cells per thread (one 32-bit access per direction),
    with velocity / pressure / no-slip faces on both ends of the pairs' rows
    and a force.  The Esoteric Twist runs one cell per thread; the two differ
    only by FP32 rounding order (the bound of test_et_agrees_with_aa)."""
    from paper_2305_09910_amd import lbm
    shape = (128, 12, 6)
    uw = np.zeros((6, 3))
    uw[0] = (0.03, 0.002, 0.0)
    kw = dict(q=q, tau=0.58, force=(1e-5, 0, -2e-6), bc=("velocity", "pressure", "noslip", "noslip", "periodic",
                                                          "periodic"), u_bc=uw, storage=storage)
    print(f"[case] q={q} storage={storage} paired even step", flush=True)
    a = lbm.Lattice(shape, streaming="aa", **kw)
    e = lbm.Lattice(shape, streaming="et", **kw)
    rho, u = inputs.uniform_flow(*shape, (0.03, 0.0, 0.0))
    u += inputs.perturbation(u.shape, 0.005, seed=3 * q)
    for g in (a, e):
        g.init_equilibrium(rho, u)
    w = torch.as_tensor(lbm_weights(q), device=a.device, dtype=torch.float64)[:, None, None, None]
    for n in (1, 50, 51):
        a.step(n - a.time)
        e.step(n - e.time)
        fa, fe = a.get_pdfs(), e.get_pdfs()
        dmax = float((fa - w).abs().max())
        rel = 2.0 ** -10 if storage == "f16" else 2.0 ** -7
        bound = n * 2 * rel * 2.0 ** np.floor(np.log2(dmax))
        diff = float((fa - fe).abs().max())
        print(f"n={n}: max |f_aa - f_et| = {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound, (n, diff, bound)


def lbm_weights(q):
    import oracle
    return oracle.velocity_set(q)[1]


@pytest.mark.parametrize("q", [19, 27])
def test_et_learned_closure_agrees_with_aa(q):
    """The learned closure fused into the Esoteric Twist kernel, with solids,
    velocity / pressure / no-slip faces and a force: the same network on the
    same values as the AA kernel, so the two differ only by FP32 rounding
    order (the FP32 bound of test_et_agrees_with_aa), and neither falls back."""
    from paper_2305_09910_amd import lbm
    from test_gpu_closure import _smooth_net
    shape = (40, 18, 12)
    solid = np.zeros(shape[::-1], np.uint8)
    solid[3:7, 5:9, 10:15] = 1
    uw = np.zeros((6, 3))
    uw[0] = (0.03, 0.002, 0.0)
    kw = dict(q=q, tau=0.56, force=(1e-5, 0, -2e-6), bc=("velocity", "pressure", "noslip", "noslip", "periodic",
                                                          "periodic"), u_bc=uw, solid=solid, closure="mlp")
    print(f"[case] q={q} mlp", flush=True)
    p, norm = _smooth_net()
    a = lbm.Lattice(shape, streaming="aa", **kw)
    e = lbm.Lattice(shape, streaming="et", **kw)
    rho, u = inputs.uniform_flow(*shape, (0.03, 0.0, 0.0))
    u += inputs.perturbation(u.shape, 0.005, seed=q)
    u[:, solid == 1] = 0.0
    for g in (a, e):
        g.set_closure_weights(np.r_[p, norm].astype(np.float32))
        g.init_equilibrium(rho, u)
    fluid = torch.as_tensor(solid == 0, device=a.device)
    for n in (1, 40, 41):
        a.step(n - a.time)
        e.step(n - e.time)
        fa, fe = a.get_pdfs(), e.get_pdfs()
        diff = float((fa - fe)[:, fluid].abs().max())
        bound = n * 4 * 2.0 ** -24 * float(fa[:, fluid].abs().max())
        print(f"n={n}: max |f_aa - f_et| = {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound, (n, diff, bound)
    assert a.closure_fallbacks() == 0 and e.closure_fallbacks() == 0


@pytest.mark.parametrize("q,storage,closure,collision", [
    (27, "f32", "smagorinsky", "mrt"),
    (19, "f16", "smagorinsky", "trt"),
    (19, "bf16", "none", "mrt"),
    (27, "f16", "none", "trt"),
    (19, "f32", "smagorinsky", "mrt"),
])
def test_kernel_combinations(q, storage, closure, collision):
    """Step-kernel instantiations that the other cases do not reach together:
    solids, velocity / pressure / no-slip faces, a force, both streaming
    schemes.  FP32 runs against the oracle (1e-5); 16-bit runs compare the
    two schemes, which differ only by FP32 rounding order (the bound of
    test_et_agrees_with_aa)."""
    import oracle
    from paper_2305_09910_amd import lbm
    from test_gpu_parity import BCS, max_rel
    shape = (24, 12, 10)
    solid = np.zeros(shape[::-1], np.uint8)
    solid[4:6, 3:6, 8:12] = 1
    uw = np.zeros((6, 3))
    uw[0] = (0.02, 0.0, 0.001)
    bc = ("velocity", "pressure", "noslip", "noslip", "periodic", "periodic")
    rates = (1.6, 1.75, 1.55, 1.65, 1.7) if q == 27 else None
    kw = dict(q=q, tau=0.62, force=(1e-5, 0, 2e-6), bc=bc, u_bc=uw, solid=solid, storage=storage, closure=closure,
              collision=collision, mrt_rates=rates)
    print(f"[case] q={q} {storage} {closure} {collision}", flush=True)
    a = lbm.Lattice(shape, streaming="aa", **kw)
    e = lbm.Lattice(shape, streaming="et", **kw)
    rho, u = inputs.uniform_flow(*shape, (0.02, 0.0, 0.0))
    u += inputs.perturbation(u.shape, 0.004, seed=q)
    u[:, solid == 1] = 0.0
    for g in (a, e):
        g.init_equilibrium(rho, u)
        g.step(60)
    fluid = solid == 0
    if storage == "f32":
        cl = {"none": oracle.CL_NONE, "smagorinsky": oracle.CL_SMAG}[closure]
        o = oracle.Sim(q, shape, bc=tuple(BCS[b] for b in bc), tau=0.62, force=(1e-5, 0, 2e-6), u_bc=uw,
                       solid=solid, closure=cl)
        if collision == "mrt":
            o.set_mrt(oracle.MRT_DHUMIERES if rates is None else rates)
        o.init_equilibrium(rho, u)
        o.step(60)
        for g in (a, e):
            assert max_rel(g.get_pdfs(), o.get_pdfs(), solid) <= 1e-5
    else:
        fa, fe = a.get_pdfs(), e.get_pdfs()
        fl = torch.as_tensor(fluid, device=a.device)
        w = torch.as_tensor(lbm_weights(q), device=a.device, dtype=torch.float64)[:, None, None, None]
        dmax = float((fa - w)[:, fl].abs().max())
        rel = 2.0 ** -10 if storage == "f16" else 2.0 ** -7
        bound = 60 * 2 * rel * 2.0 ** np.floor(np.log2(dmax))
        diff = float((fa - fe)[:, fl].abs().max())
        print(f"max |f_aa - f_et| = {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound

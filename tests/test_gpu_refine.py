"""2:1 grid refinement on the GPU (lbm_refine_step) against the FP64 oracle
(orc_refine_step), element by element on every level: maximum relative
population error 1e-5 in FP32 storage. Cases: D3Q19 and D3Q27 with fine
levels on both sides, walls, a moving lid, a solid block and a body force,
after 1, 2, 7 and 40 coarse steps; one fine level only; MRT; mixed storage
(16-bit fine levels); mass conservation; the force-driven channel's exact
profile; checkpoints; and the rejection of lattices that do not fit."""

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
OBC = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "velocity": oracle.BC_VELOCITY,
       "pressure": oracle.BC_PRESSURE, "interface": oracle.BC_INTERFACE}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_09910_amd import lbm
    lbm.lib()
    yield
    torch.cuda.synchronize()


def build(shape_c, nyf, tau, F=(0.0, 0.0, 0.0), q=19, outer=("noslip", "noslip"), u_bc=None, lo=True, hi=True,
          solid_c=None, storage=("f32", "f32", "f32"), mrt=False):
    """GPU and oracle lattices of a coarse level with fine levels below/above."""
    from paper_2305_09910_amd import lbm
    nxc, nyc, nzc = shape_c
    tf, Ff = 0.5 + 2 * (tau - 0.5), tuple(0.5 * np.asarray(F, float))
    ub = np.zeros((6, 3)) if u_bc is None else u_bc
    per = ("periodic", "periodic")
    spec = [("c", (nxc, nyc, nzc), per + ("interface" if lo else outer[0], "interface" if hi else outer[1]) + per, tau,
             F, solid_c, storage[0])]
    if lo:
        spec.append(("lo", (2 * nxc, nyf, 2 * nzc), per + (outer[0], "interface") + per, tf, Ff, None, storage[1]))
    if hi:
        spec.append(("hi", (2 * nxc, nyf, 2 * nzc), per + ("interface", outer[1]) + per, tf, Ff, None, storage[2]))
    gpu, orc = {}, {}
    for name, shape, bc, t, f, solid, st in spec:
        print(f"[case] refine {name} q={q} shape={shape} bc={bc} tau={t} storage={st}", flush=True)
        kw = dict(collision="mrt", mrt_rates=oracle.MRT_DHUMIERES) if mrt else {}
        gpu[name] = lbm.Lattice(shape, q=q, tau=t, force=f, bc=bc, u_bc=ub, solid=solid, storage=st, **kw)
        orc[name] = oracle.Sim(q, shape, bc=tuple(OBC[b] for b in bc), tau=t, force=f, u_bc=ub, solid=solid)
        if mrt:
            orc[name].set_mrt(oracle.MRT_DHUMIERES)
    return gpu, orc


def random_start(gpu, orc, seed):
    """A seeded non-equilibrium state (f^eq of random rho, u times 1 + 2%
    noise), the same FP64 populations on both sides."""
    for k, name in enumerate(sorted(gpu)):
        s = orc[name]
        nx, ny, nz = s.shape
        rng = np.random.default_rng(seed + k)
        rho = 1 + 0.02 * rng.standard_normal((nz, ny, nx))
        u = 0.03 * rng.standard_normal((3, nz, ny, nx))
        c, w, _ = oracle.velocity_set(s.q)
        cu = np.einsum("ia,azyx->izyx", c.astype(float), u)
        usq = (u * u).sum(0)
        f = w[:, None, None, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * usq)
        f *= 1 + 0.02 * rng.standard_normal(f.shape)
        s.set_pdfs(f)
        gpu[name].set_pdfs(f)


def step_both(gpu, orc, n):
    from paper_2305_09910_amd import lbm
    lbm.refine_step(gpu["c"], gpu.get("lo"), gpu.get("hi"), n)
    oracle.refine_step(orc["c"], orc.get("lo"), orc.get("hi"), n)


def max_rel(g, o, solid=None):
    a = g.get_pdfs().cpu().numpy()
    b = o.get_pdfs()
    if solid is not None:  # solid cells hold zeros on both sides
        a, b = a[:, solid == 0], b[:, solid == 0]
    err = np.abs(a - b) / np.abs(b)
    return float(err.max())


@pytest.mark.parametrize("q", [19, 27])
def test_refine_matches_oracle_on_every_level(q):
    shape_c, nyf = (6, 6, 4), 4
    solid = np.zeros(shape_c[::-1], np.uint8)
    solid[1:3, 2:4, 2:4] = 1
    ub = np.zeros((6, 3))
    ub[3] = (0.04, 0, 0.01)
    gpu, orc = build(shape_c, nyf, 0.62, (2e-5, -1e-5, 0), q=q, outer=("noslip", "velocity"), u_bc=ub,
                     solid_c=solid)
    random_start(gpu, orc, 11)
    done = 0
    for n in (1, 2, 7, 40):
        step_both(gpu, orc, n - done)
        done = n
        for name in gpu:
            err = max_rel(gpu[name], orc[name], solid if name == "c" else None)
            print(f"refine q={q} coarse steps {n} level {name}: max rel err {err:.2e}")
            assert err <= TOL32
    assert gpu["c"].time == 40 and gpu["lo"].time == 80 and gpu["hi"].time == 80


@pytest.mark.parametrize("side", ["lo", "hi"])
def test_refine_one_fine_level(side):
    gpu, orc = build((8, 5, 4), 6, 0.7, (1e-5, 0, 0), lo=side == "lo", hi=side == "hi")
    random_start(gpu, orc, 3)
    step_both(gpu, orc, 15)
    for name in gpu:
        assert max_rel(gpu[name], orc[name]) <= TOL32


def test_refine_mrt():
    gpu, orc = build((6, 4, 4), 4, 0.6, (1e-5, 0, 0), mrt=True)
    random_start(gpu, orc, 5)
    step_both(gpu, orc, 20)
    for name in gpu:
        assert max_rel(gpu[name], orc[name]) <= TOL32


def test_refine_mixed_storage():
    """FP32 coarse level, FP16 and BF16 deviations on the fine levels:
    velocity L2 error against the oracle after 50 coarse steps within the
    16-bit forms' bounds (1e-2 FP16, 5e-2 BF16)."""
    gpu, orc = build((8, 6, 4), 6, 0.65, (1e-5, 0, 0), storage=("f32", "f16", "bf16"))
    random_start(gpu, orc, 9)
    step_both(gpu, orc, 50)
    assert max_rel(gpu["c"], orc["c"]) < 1e-2
    for name, bound in (("lo", 1e-2), ("hi", 5e-2)):
        ug = gpu[name].moments()[1].cpu().numpy()
        uo = orc[name].moments()[1]
        l2 = float(np.sqrt(((ug - uo) ** 2).sum() / (uo ** 2).sum()))
        print(f"refine mixed storage {name}: velocity L2 {l2:.2e}")
        assert l2 < bound


def test_refine_conserves_mass():
    """sum rho_c + sum rho_f / 8 over 300 coarse steps with walls and a solid
    block: FP32 storage keeps it within 1e-6 (the oracle's is exact)."""
    shape_c = (8, 6, 4)
    solid = np.zeros(shape_c[::-1], np.uint8)
    solid[1:3, 2:4, 3:6] = 1
    gpu, orc = build(shape_c, 4, 0.6, (1e-5, 0, 0), solid_c=solid)
    random_start(gpu, orc, 13)

    def mass():
        return gpu["c"].totals()[0] + (gpu["lo"].totals()[0] + gpu["hi"].totals()[0]) / 8

    m0 = mass()
    from paper_2305_09910_amd import lbm
    lbm.refine_step(gpu["c"], gpu["lo"], gpu["hi"], 300)
    assert abs(mass() - m0) / m0 < 1e-6


def test_refine_poiseuille_profile():
    """Fine (8 rows) / coarse (8) / fine (8) channel, body force: after 4000
    coarse steps the profile on every level is the parabola F/(2 nu) y (H - y)
    (exact for the scheme) within FP32 rounding."""
    nyc, nyf, tau, F = 8, 8, 0.8, 3e-5
    gpu, _ = build((4, nyc, 2), nyf, tau, (F, 0, 0))
    for g in gpu.values():
        nx, ny, nz = g.shape
        g.init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    from paper_2305_09910_amd import lbm
    lbm.refine_step(gpu["c"], gpu["lo"], gpu["hi"], 4000)
    H, nu = nyc + nyf, (tau - 0.5) / 3
    for name, y0, h in (("lo", 0.0, 0.5), ("c", nyf / 2, 1.0), ("hi", nyf / 2 + nyc, 0.5)):
        g = gpu[name]
        u = g.moments()[1].cpu().numpy()
        y = y0 + (np.arange(g.shape[1]) + 0.5) * h
        exact = F / (2 * nu) * y * (H - y)
        err = np.abs(u[0] - exact[None, :, None]).max() / exact.max()
        print(f"refine Poiseuille {name}: max rel err {err:.2e}")
        assert err < 2e-4


def test_refine_checkpoint_resumes_bit_for_bit():
    gpu, orc = build((6, 4, 4), 4, 0.7, (1e-5, 0, 0))
    random_start(gpu, orc, 21)
    from paper_2305_09910_amd import lbm
    lbm.refine_step(gpu["c"], gpu["lo"], gpu["hi"], 3)
    saved = {k: g.save_state() for k, g in gpu.items()}
    lbm.refine_step(gpu["c"], gpu["lo"], gpu["hi"], 9)
    ref = {k: g.get_pdfs().clone() for k, g in gpu.items()}
    for k, g in gpu.items():
        g.load_state(*saved[k])
    lbm.refine_step(gpu["c"], gpu["lo"], gpu["hi"], 9)
    for k, g in gpu.items():
        assert torch.equal(g.get_pdfs(), ref[k])


@pytest.mark.parametrize("case", ["nx", "tau", "force", "missing", "extra", "closure", "magic", "same", "work",
                                  "second_interface", "collision"])
def test_refine_rejects_lattices_that_do_not_fit(case):
    from paper_2305_09910_amd import lbm
    per = ("periodic", "periodic")
    tau, tf = 0.7, 0.9
    kc = dict(q=19, tau=tau, force=(2e-5, 0, 0), bc=per + ("noslip", "interface") + per)
    kf = dict(q=19, tau=tf, force=(1e-5, 0, 0), bc=per + ("interface", "noslip") + per)
    shape_c, shape_f = (4, 3, 2), (8, 3, 4)
    if case == "nx":
        shape_f = (6, 3, 4)
    elif case == "tau":
        kf["tau"] = tau
    elif case == "force":
        kf["force"] = (2e-5, 0, 0)
    elif case == "closure":
        kf["closure"] = "smagorinsky"
    elif case == "magic":
        kf["magic"] = 0.25
    elif case == "second_interface":
        kf["bc"] = per + ("interface", "interface") + per
    elif case == "collision":
        kf["collision"] = "mrt"
    c = lbm.Lattice(shape_c, **kc)
    f = lbm.Lattice(shape_f, **kf)
    lo, hi = None, f
    if case == "missing":
        hi = None
    elif case == "extra":
        lo = f
    elif case == "same":
        hi = c
    if case == "work":
        rc = lbm.lib().lbm_refine_step(c._h, None, f._h, None, 0, 1)
        assert rc == lbm.LBM_EINVAL
        return
    with pytest.raises(lbm.LBMError) as e:
        lbm.refine_step(c, lo, hi, 1)
    assert e.value.code == lbm.LBM_EINVAL
    assert c.time == 0 and f.time == 0  # nothing ran

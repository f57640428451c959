"""Hierarchies of 2:1 levels on the GPU (lbm_refine_tree_step) against the
FP64 oracle (orc_refine_tree_step), element by element on every level:
maximum relative population error 1e-5 in FP32 storage.  Cases: the
five-level stack fine / medium / coarse / medium / fine (D3Q19 and D3Q27,
walls, a moving lid, a body force); a one-sided chain four levels deep; mass
over levels (sum of M / 8^depth); the force-driven channel's exact profile
across four interfaces; and the rejection of malformed trees."""

import ctypes

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
OBC = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "velocity": oracle.BC_VELOCITY,
       "pressure": oracle.BC_PRESSURE, "interface": oracle.BC_INTERFACE}
PER = ("periodic", "periodic")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_09910_amd import lbm
    lbm.lib()
    yield
    torch.cuda.synchronize()


def make(spec, q, tau, F, u_bc):
    """GPU and oracle node lists from (shape, depth, y faces, lo, hi)."""
    from paper_2305_09910_amd import lbm
    gpu, orc = [], []
    for shape, depth, faces, lo, hi in spec:
        bc = PER + faces + PER
        t = 0.5 + 2 ** depth * (tau - 0.5)
        f = tuple(np.asarray(F, float) / 2 ** depth)
        print(f"[case] refine tree q={q} shape={shape} depth={depth} bc={bc} tau={t}", flush=True)
        gpu.append((lbm.Lattice(shape, q=q, tau=t, force=f, bc=bc, u_bc=u_bc), lo, hi))
        orc.append((oracle.Sim(q, shape, bc=tuple(OBC[b] for b in bc), tau=t, force=f, u_bc=u_bc), lo, hi))
    return gpu, orc


def stack_spec(nxc, nyc, nzc, nym, nyf, outer=("noslip", "noslip")):
    """fine (4x) / medium (2x) / coarse / medium / fine along y, coarse first."""
    I = "interface"
    return [((nxc, nyc, nzc), 0, (I, I), 1, 2),
            ((2 * nxc, nym, 2 * nzc), 1, (I, I), 3, None),
            ((2 * nxc, nym, 2 * nzc), 1, (I, I), None, 4),
            ((4 * nxc, nyf, 4 * nzc), 2, (outer[0], I), None, None),
            ((4 * nxc, nyf, 4 * nzc), 2, (I, outer[1]), None, None)]


def chain_spec():
    """Coarse lattice with three ever finer levels below it (depth 0..3)."""
    I = "interface"
    return [((2, 3, 2), 0, (I, "velocity"), 1, None),
            ((4, 3, 4), 1, (I, I), 2, None),
            ((8, 3, 8), 2, (I, I), 3, None),
            ((16, 4, 16), 3, ("noslip", I), None, None)]


def random_start(gpu, orc, seed):
    """f^eq of random rho, u times 1 + 2% noise: the same FP64 populations on
    both sides."""
    for k, ((g, _, _), (o, _, _)) in enumerate(zip(gpu, orc)):
        nx, ny, nz = o.shape
        rng = np.random.default_rng(seed + k)
        rho = 1 + 0.02 * rng.standard_normal((nz, ny, nx))
        u = 0.03 * rng.standard_normal((3, nz, ny, nx))
        c, w, _ = oracle.velocity_set(o.q)
        cu = np.einsum("ia,azyx->izyx", c.astype(float), u)
        f = w[:, None, None, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u * u).sum(0))
        f *= 1 + 0.02 * rng.standard_normal(f.shape)
        o.set_pdfs(f)
        g.set_pdfs(f)


def max_rel(g, o):
    a = g.get_pdfs().cpu().numpy()
    b = o.get_pdfs()
    return float((np.abs(a - b) / np.abs(b)).max())


@pytest.mark.parametrize("q", [19, 27])
def test_tree_matches_oracle_on_every_level(q):
    from paper_2305_09910_amd import lbm
    ub = np.zeros((6, 3))
    ub[3] = (0.03, 0, -0.01)
    spec = stack_spec(3, 4, 2, 4, 4, outer=("noslip", "velocity"))
    gpu, orc = make(spec, q, 0.6, (2e-5, -1e-5, 0), ub)
    random_start(gpu, orc, 31)
    done = 0
    for n in (1, 3, 10):
        lbm.refine_tree_step(gpu, n - done)
        oracle.refine_tree_step(orc, n - done)
        done = n
        for k, ((g, _, _), (o, _, _)) in enumerate(zip(gpu, orc)):
            err = max_rel(g, o)
            print(f"refine tree q={q} coarse steps {n} node {k}: max rel err {err:.2e}")
            assert err <= TOL32
    assert [g.time for g, _, _ in gpu] == [10, 20, 20, 40, 40]


def test_chain_four_levels_deep_matches_oracle():
    from paper_2305_09910_amd import lbm
    ub = np.zeros((6, 3))
    ub[3] = (0.04, 0, 0)
    gpu, orc = make(chain_spec(), 19, 0.55, (1e-5, 0, 0), ub)
    random_start(gpu, orc, 7)
    lbm.refine_tree_step(gpu, 6)
    oracle.refine_tree_step(orc, 6)
    for k, ((g, _, _), (o, _, _)) in enumerate(zip(gpu, orc)):
        err = max_rel(g, o)
        print(f"refine chain node {k}: max rel err {err:.2e}, time {g.time}")
        assert err <= TOL32
        assert g.time == 6 * 2 ** k


def test_tree_conserves_mass():
    """sum over levels of M / 8^depth over 100 coarse steps (400 on the finest
    levels), walls and a moving lid: FP32 storage keeps it within 1e-6 (the
    oracle's is exact)."""
    from paper_2305_09910_amd import lbm
    ub = np.zeros((6, 3))
    ub[3] = (0.03, 0, 0)
    spec = stack_spec(4, 4, 2, 4, 4, outer=("noslip", "velocity"))
    gpu, orc = make(spec, 19, 0.6, (1e-5, 0, 0), ub)
    random_start(gpu, orc, 3)
    depth = [d for _, d, _, _, _ in spec]

    def mass():
        return sum(g.totals()[0] / 8.0 ** d for (g, _, _), d in zip(gpu, depth))

    m0 = mass()
    lbm.refine_tree_step(gpu, 100)
    print(f"refine tree mass drift {abs(mass() - m0) / m0:.2e}")
    assert abs(mass() - m0) / m0 < 1e-6


def test_tree_poiseuille_profile():
    """fine (8 rows) / medium (8) / coarse (8) / medium (8) / fine (8), body
    force, walls: after 6000 coarse steps the profile on every level is the
    parabola F/(2 nu) y (H - y) (exact for the scheme) within FP32 rounding."""
    from paper_2305_09910_amd import lbm
    tau, F = 0.8, 2e-5
    spec = stack_spec(4, 8, 2, 8, 8)
    gpu, _ = make(spec, 19, tau, (F, 0, 0), np.zeros((6, 3)))
    for g, _, _ in gpu:
        nx, ny, nz = g.shape
        g.init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    lbm.refine_tree_step(gpu, 6000)
    H, nu = 2.0 + 4.0 + 8.0 + 4.0 + 2.0, (tau - 0.5) / 3
    origin = {3: (0.0, 0.25), 1: (2.0, 0.5), 0: (6.0, 1.0), 2: (14.0, 0.5), 4: (18.0, 0.25)}
    for k, (y0, h) in origin.items():
        g = gpu[k][0]
        u = g.moments()[1].cpu().numpy()
        y = y0 + (np.arange(g.shape[1]) + 0.5) * h
        exact = F / (2 * nu) * y * (H - y)
        err = np.abs(u[0] - exact[None, :, None]).max() / exact.max()
        print(f"refine tree Poiseuille node {k}: max rel err {err:.2e}")
        assert err < 2e-4


@pytest.mark.parametrize("case", ["order", "two_parents", "lone_interface", "parent_side", "not_interface"])
def test_tree_rejects_malformed_trees(case):
    from paper_2305_09910_amd import lbm
    spec = stack_spec(2, 3, 2, 3, 3)
    if case == "order":  # a child before its parent
        spec[1] = spec[1][:3] + (0, None)
    elif case == "two_parents":
        spec[2] = spec[2][:3] + (None, 3)
    elif case == "lone_interface":  # an interface face that meets nothing
        spec[3] = spec[3][:2] + (("interface", "interface"), None, None)
    elif case == "parent_side":  # a child on the side of the node's parent
        spec[1] = spec[1][:3] + (3, 4)
        spec[2] = spec[2][:2] + (("interface", "noslip"), None, None)
    elif case == "not_interface":
        spec[4] = spec[4][:2] + (("noslip", "noslip"), None, None)
    gpu, _ = make(spec, 19, 0.6, (0, 0, 0), np.zeros((6, 3)))
    with pytest.raises(lbm.LBMError) as e:
        lbm.refine_tree_step(gpu, 1)
    assert e.value.code == lbm.LBM_EINVAL
    print(f"refine tree {case}: {e.value}")
    assert all(g.time == 0 for g, _, _ in gpu)  # nothing ran


def test_tree_rejects_overlapping_work_buffers():
    """A parent's sums live across its child's own exchanges, so two parents
    sharing a work buffer are rejected before anything runs."""
    from paper_2305_09910_amd import lbm
    I = "interface"
    spec = [((2, 3, 2), 0, (I, "noslip"), 1, None),
            ((4, 3, 4), 1, (I, I), 2, None),
            ((8, 3, 8), 2, ("noslip", I), None, None)]
    gpu, _ = make(spec, 19, 0.6, (0, 0, 0), np.zeros((6, 3)))
    need = ctypes.c_size_t(0)
    L = lbm.lib()
    assert L.lbm_refine_work_bytes(ctypes.byref(gpu[1][0].domain), 19, ctypes.byref(need)) == lbm.LBM_OK
    work = torch.empty(2 * need.value, dtype=torch.uint8, device="cuda")
    arr = (lbm.RefineNode * 3)()
    for k, (lat, lo, hi) in enumerate(gpu):
        arr[k].ctx = lat._h
        arr[k].fine_lo = -1 if lo is None else lo
        arr[k].fine_hi = -1 if hi is None else hi
    arr[0].work_dev, arr[0].work_bytes = work.data_ptr(), need.value
    arr[1].work_dev, arr[1].work_bytes = work.data_ptr() + 256, need.value
    assert L.lbm_refine_tree_step(arr, 3, 1) == lbm.LBM_EINVAL
    assert b"overlap" in L.lbm_last_error(gpu[0][0]._h)
    arr[1].work_dev = work.data_ptr() + need.value  # disjoint: runs
    assert L.lbm_refine_tree_step(arr, 3, 1) == lbm.LBM_OK
    torch.cuda.synchronize()
    assert [g.time for g, _, _ in gpu] == [1, 2, 4]

"""Pins of the oracle's 2:1 grid refinement (orc_refine_step), CPU only.

The paper's block forest refines 2:1 and joins the levels with coarse-to-fine
and fine-to-coarse kernels (Sections 3 and 5.2); the scheme is the volumetric
exchange stated in the oracle's header. Its pins:

- the exchange geometry and timing, brute force on tiny lattices: a Python
  emulation of one refinement step from single-lattice oracle steps (the
  interface faces as no-slip faces) and point-in-cell tests in real
  coordinates;
- exact mass conservation, M_c + M_f / 8;
- a uniform moving state is a fixed point on all levels;
- force-driven Poiseuille flow across both interfaces is exact to roundoff
  (TRT with the magic parameter 3/16, exact on one level);
- a decaying 2-D vortex flow converges to a run that is fine everywhere
  (first order: the interface spreads packets evenly);
- geometry and parameter checks reject lattices that do not fit.
"""
import math

import numpy as np
import pytest

import oracle

P, NS, V, I = oracle.BC_PERIODIC, oracle.BC_NOSLIP, oracle.BC_VELOCITY, oracle.BC_INTERFACE


def levels(nxc, nyc, nzc, nyf, tau, F=(0.0, 0.0, 0.0), q=19, outer=(NS, NS), u_bc=None, lo=True, hi=True,
           solid_c=None):
    """Coarse lattice (nxc, nyc, nzc) with fine lattices (2 nxc, nyf, 2 nzc)
    below and/or above; acoustic scaling tau_f = 1/2 + 2 (tau - 1/2), F_f = F/2."""
    tf = 0.5 + 2 * (tau - 0.5)
    Ff = tuple(0.5 * np.asarray(F, float))
    ub = np.zeros((6, 3)) if u_bc is None else u_bc
    c = oracle.Sim(q, (nxc, nyc, nzc), bc=(P, P, I if lo else outer[0], I if hi else outer[1], P, P), tau=tau,
                   force=F, u_bc=ub, solid=solid_c)
    fl = oracle.Sim(q, (2 * nxc, nyf, 2 * nzc), bc=(P, P, outer[0], I, P, P), tau=tf, force=Ff, u_bc=ub) if lo else None
    fh = oracle.Sim(q, (2 * nxc, nyf, 2 * nzc), bc=(P, P, I, outer[1], P, P), tau=tf, force=Ff, u_bc=ub) if hi else None
    return c, fl, fh


def total_mass(c, fl, fh):
    """M_c + M_f / 8: a fine cell holds an eighth of a coarse cell's volume."""
    return c.totals()[0] + sum(f.totals()[0] / 8.0 for f in (fl, fh) if f is not None)


def random_state(s, seed, amp=0.02, u0=0.03):
    nx, ny, nz = s.shape
    rng = np.random.default_rng(seed)
    cvec, w, _ = oracle.velocity_set(s.q)
    rho = 1 + amp * rng.standard_normal((nz, ny, nx))
    u = u0 * rng.standard_normal((3, nz, ny, nx))
    f = np.empty((s.q, nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f[:, z, y, x] = oracle.equilibrium(s.q, rho[z, y, x], u[:, z, y, x])
    f *= 1 + amp * rng.standard_normal(f.shape)  # non-equilibrium part
    s.set_pdfs(f)


# --------------------------------------------------------------------------
# exchange geometry, brute force
# --------------------------------------------------------------------------
def _emulate(cpdf, lopdf, hipdf, shape_c, nyf, tau, F, q):
    """One refinement step from single-lattice oracle steps. Interface faces
    act as no-slip faces within a lattice. A packet a coarse interface cell
    emits across the interface arrives, after each of the two fine substeps,
    in every fine interface cell whose source point (cell centre minus c_j
    fine spacings) lies inside that coarse cell; the fine packets of both
    substeps are averaged (weight 1/8) into the coarse cell containing their
    target point (centre plus c_i fine spacings)."""
    nxc, nyc, nzc = shape_c
    cvec, _, _ = oracle.velocity_set(q)
    opp = [int(np.nonzero((cvec == -cvec[i]).all(1))[0][0]) for i in range(q)]
    tf, Ff = 0.5 + 2 * (tau - 0.5), tuple(0.5 * np.asarray(F, float))
    cs = oracle.Sim(q, shape_c, bc=(P, P, NS, NS, P, P), tau=tau, force=F)
    cs.set_pdfs(cpdf)
    cs.step(1)
    cnew = cs.get_pdfs()
    out = {}
    for side, fpdf in (("lo", lopdf), ("hi", hipdf)):
        above = side == "hi"
        dy = 1 if above else -1
        yc, yf = (nyc - 1, 0) if above else (0, nyf - 1)
        fs = oracle.Sim(q, (2 * nxc, nyf, 2 * nzc), bc=(P, P, NS, NS, P, P), tau=tf, force=Ff)
        f = fpdf.copy()

        def coarse_cell(xf, zf, j, sign):
            # fine cell centre in coarse units, moved by sign * c_j fine spacings
            px = ((xf + 0.5) / 2 + sign * cvec[j][0] * 0.5) % nxc
            pz = ((zf + 0.5) / 2 + sign * cvec[j][2] * 0.5) % nzc
            return int(math.floor(px)), int(math.floor(pz))

        def fill(f):
            for j in range(q):
                if cvec[j][1] != dy:
                    continue
                for zf in range(2 * nzc):
                    for xf in range(2 * nxc):
                        X, Z = coarse_cell(xf, zf, j, -1)
                        # the packet coarse cell (X, Z) sent in direction j bounced into slot opp(j)
                        f[j, zf, yf, xf] = cnew[opp[j], Z, yc, X]

        acc = np.zeros((q, nzc, nxc))
        for sub in range(2):
            fs.set_pdfs(f)
            fs.step(1)
            f = fs.get_pdfs()
            for i in range(q):
                if cvec[i][1] != -dy:
                    continue
                for zf in range(2 * nzc):
                    for xf in range(2 * nxc):
                        X, Z = coarse_cell(xf, zf, i, +1)
                        acc[i, Z, X] += f[opp[i], zf, yf, xf] / 8.0
            fill(f)
        out[side] = f
        for i in range(q):
            if cvec[i][1] == -dy:
                cnew[i, :, yc, :] = acc[i]
    return cnew, out["lo"], out["hi"]


@pytest.mark.parametrize("q", [19, 27])
def test_refine_step_matches_brute_force_exchange(q):
    shape_c, nyf, tau, F = (3, 3, 2), 3, 0.7, (1e-4, -2e-5, 3e-5)
    c, fl, fh = levels(*shape_c, nyf, tau, F, q=q)
    for s, seed in ((c, 1), (fl, 2), (fh, 3)):
        random_state(s, seed)
    cref, loref, hiref = _emulate(c.get_pdfs(), fl.get_pdfs(), fh.get_pdfs(), shape_c, nyf, tau, F, q)
    oracle.refine_step(c, fl, fh, 1)
    for s, ref in ((c, cref), (fl, loref), (fh, hiref)):
        np.testing.assert_allclose(s.get_pdfs(), ref, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# conservation and exact solutions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", [19, 27])
def test_refine_conserves_mass_exactly(q):
    """Random non-equilibrium state, walls on the outer faces (a moving lid on
    top), a solid block inside the coarse level: M_c + M_f / 8 stays
    constant to roundoff over 30 coarse steps."""
    shape_c, nyf = (6, 6, 4), 4
    solid = np.zeros(shape_c[::-1], np.uint8)
    solid[1:3, 2:4, 2:4] = 1
    ub = np.zeros((6, 3))
    ub[3] = (0.04, 0, 0.01)
    c, fl, fh = levels(*shape_c, nyf, 0.62, (2e-5, 0, 0), q=q, outer=(NS, V), u_bc=ub, solid_c=solid)
    for s, seed in ((c, 4), (fl, 5), (fh, 6)):
        random_state(s, seed)
    m0 = total_mass(c, fl, fh)
    for _ in range(3):
        oracle.refine_step(c, fl, fh, 10)
        assert abs(total_mass(c, fl, fh) - m0) <= 2e-14 * m0


def test_refine_uniform_moving_state_is_a_fixed_point():
    """Uniform rho = 1, u = u0 tangential to the interfaces, velocity faces
    moving with u0 outside: every population of every level stays put."""
    u0 = np.array([0.04, 0.0, -0.025])
    ub = np.tile(u0, (6, 1))
    c, fl, fh = levels(4, 4, 2, 4, 0.66, outer=(V, V), u_bc=ub)
    for s in (c, fl, fh):
        nx, ny, nz = s.shape
        s.init_equilibrium(np.ones((nz, ny, nx)), np.broadcast_to(u0[:, None, None, None], (3, nz, ny, nx)).copy())
    ref = [s.get_pdfs() for s in (c, fl, fh)]
    oracle.refine_step(c, fl, fh, 6)
    for s, r in zip((c, fl, fh), ref):
        np.testing.assert_allclose(s.get_pdfs(), r, rtol=0, atol=2e-15)  # a few ulps of w_0


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_refine_poiseuille_exact_across_both_interfaces(tau):
    """Fine (8 rows) / coarse (8 rows) / fine (8 rows), no-slip outside, body
    force in x: the steady profile is the parabola F/(2 nu) y (H - y) of the
    physical height H = 16 coarse cells on every level, to roundoff."""
    nyc, nyf, F = 8, 8, 1e-5
    c, fl, fh = levels(1, nyc, 1, nyf, tau, (F, 0, 0))
    for s in (c, fl, fh):
        nx, ny, nz = s.shape
        s.init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    oracle.refine_step(c, fl, fh, 12000)
    H, nu = nyc + nyf, (tau - 0.5) / 3
    for s, y0, h in ((fl, 0.0, 0.5), (c, nyf / 2, 1.0), (fh, nyf / 2 + nyc, 0.5)):
        _, u = s.moments()
        y = y0 + (np.arange(s.shape[1]) + 0.5) * h
        exact = F / (2 * nu) * y * (H - y)
        assert np.abs(u[0][0, :, 0] - exact).max() <= 1e-10 * exact.max()


def _vortex_errors(N, tau=0.6):
    """A decaying 2-D vortex pair (stream function sin(2 pi x / L) sin^2(pi y / H))
    between no-slip walls, crossing both interfaces: fine (N rows) / coarse
    (N rows) / fine (N rows), L = 2N coarse cells. Diffusive scaling: the
    amplitude falls as 1/N and the run lasts 40 (N/8)^2 coarse steps. Returns
    the RMS velocity error of the fine levels and of the coarse level (against
    the mean of its 8 fine cells) relative to a run that is fine everywhere,
    over the peak velocity."""
    nxc, nyc, nyf = 2 * N, N, N
    amp, steps = 0.05 * 8 / N, 40 * (N // 8) ** 2
    c, fl, fh = levels(nxc, nyc, 1, nyf, tau)
    H, L = nyc + nyf, float(nxc)
    ref = oracle.Sim(19, (2 * nxc, 2 * (nyf + nyc), 2), bc=(P, P, NS, NS, P, P), tau=0.5 + 2 * (tau - 0.5))

    def init(s, y0, h):
        nx, ny, nz = s.shape
        X, Y = np.meshgrid((np.arange(nx) + 0.5) * h, y0 + (np.arange(ny) + 0.5) * h, indexing="xy")
        u = np.zeros((3, nz, ny, nx))
        u[0] = amp * H / 16 * np.sin(2 * np.pi * X / L) * (np.pi / H) * np.sin(2 * np.pi * Y / H)
        u[1] = -amp * H / 16 * (2 * np.pi / L) * np.cos(2 * np.pi * X / L) * np.sin(np.pi * Y / H) ** 2
        s.init_equilibrium(np.ones((nz, ny, nx)), u)

    init(fl, 0.0, 0.5)
    init(c, nyf / 2, 1.0)
    init(fh, nyf / 2 + nyc, 0.5)
    init(ref, 0.0, 0.5)
    oracle.refine_step(c, fl, fh, steps)
    ref.step(2 * steps)
    ur = ref.moments()[1]
    umax = np.abs(ur).max()
    ulo, uc, uhi = fl.moments()[1], c.moments()[1], fh.moments()[1]
    e_f = np.sqrt(0.5 * (((ulo - ur[:, :, :nyf]) ** 2).mean() + ((uhi - ur[:, :, nyf + 2 * nyc:]) ** 2).mean()))
    avg = ur[:, :, nyf:nyf + 2 * nyc, :].reshape(3, 1, 2, nyc, 2, nxc, 2).mean(axis=(2, 4, 6))
    e_c = np.sqrt(((uc - avg) ** 2).mean())
    return e_f / umax, e_c / umax


def test_refine_vortex_flow_converges_to_a_fine_run():
    """The refined vortex flow converges to the run that is fine everywhere at
    first order (the evenly spread interface packets; each level alone is
    second order): doubling the resolution at least about halves both
    levels' errors, and at N = 16 they are below 0.4% of the peak velocity.
    A misplaced packet (a sign of c, a substep rule used on one side only)
    leaves errors of several percent that do not converge."""
    e8 = _vortex_errors(8)
    e16 = _vortex_errors(16)
    for a, b in zip(e8, e16):
        assert a / b > 1.7
        assert b < 4e-3


def test_refine_with_one_fine_level():
    """A fine level on one side only (the other outer face a wall): mass is
    conserved and the uniform state at rest stays put."""
    for lo, hi in ((True, False), (False, True)):
        c, fl, fh = levels(3, 4, 2, 4, 0.7, lo=lo, hi=hi)
        for s, seed in ((c, 7), (fl, 8), (fh, 9)):
            if s is not None:
                random_state(s, seed)
        m0 = total_mass(c, fl, fh)
        oracle.refine_step(c, fl, fh, 8)
        assert abs(total_mass(c, fl, fh) - m0) <= 1e-14 * m0


@pytest.mark.parametrize("case", ["nx", "tau", "force", "face", "missing", "hrr", "solid_row", "magic"])
def test_refine_rejects_lattices_that_do_not_fit(case):
    tau, F = 0.7, (1e-5, 0, 0)
    shape_c, nyf = (3, 4, 2), 4
    tf, Ff = 0.5 + 2 * (tau - 0.5), (0.5e-5, 0, 0)
    fshape = (6, nyf, 4)
    cbc, fbc = (P, P, NS, I, P, P), (P, P, I, NS, P, P)
    kw_c, kw_f = dict(tau=tau, force=F), dict(tau=tf, force=Ff)
    solid = None
    if case == "nx":
        fshape = (4, nyf, 4)
    elif case == "tau":
        kw_f["tau"] = tau
    elif case == "force":
        kw_f["force"] = F
    elif case == "face":
        fbc = (P, P, NS, NS, P, P)
    elif case == "magic":
        kw_f["magic"] = 0.25
    elif case == "solid_row":
        solid = np.zeros(shape_c[::-1], np.uint8)
        solid[0, shape_c[1] - 1, 1] = 1
    c = oracle.Sim(19, shape_c, bc=cbc, solid=solid, **kw_c)
    f = oracle.Sim(19, fshape, bc=fbc, **kw_f)
    if case == "hrr":
        c.set_hrr(0.9)
        f.set_hrr(0.9)
    with pytest.raises(ValueError):
        if case == "missing":
            oracle.refine_step(c, None, None)
        else:
            oracle.refine_step(c, None, f)


# --------------------------------------------------------------------------
# hierarchies of levels (orc_refine_tree_step)
# --------------------------------------------------------------------------
def stack(nxc, nyc, nzc, nym, nyf, tau, F=(0.0, 0.0, 0.0), q=19, outer=(NS, NS), u_bc=None):
    """Five lattices, finest at both walls: fine (4x) / medium (2x) / coarse /
    medium / fine along y; tau and F scaled per level. Returns the node list
    (Sim, lower child, upper child) with the coarse lattice first."""
    ub = np.zeros((6, 3)) if u_bc is None else u_bc
    F = np.asarray(F, float)
    tm, tf = 0.5 + 2 * (tau - 0.5), 0.5 + 4 * (tau - 0.5)
    c = oracle.Sim(q, (nxc, nyc, nzc), bc=(P, P, I, I, P, P), tau=tau, force=tuple(F), u_bc=ub)
    ml = oracle.Sim(q, (2 * nxc, nym, 2 * nzc), bc=(P, P, I, I, P, P), tau=tm, force=tuple(F / 2), u_bc=ub)
    mh = oracle.Sim(q, (2 * nxc, nym, 2 * nzc), bc=(P, P, I, I, P, P), tau=tm, force=tuple(F / 2), u_bc=ub)
    fl = oracle.Sim(q, (4 * nxc, nyf, 4 * nzc), bc=(P, P, outer[0], I, P, P), tau=tf, force=tuple(F / 4), u_bc=ub)
    fh = oracle.Sim(q, (4 * nxc, nyf, 4 * nzc), bc=(P, P, I, outer[1], P, P), tau=tf, force=tuple(F / 4), u_bc=ub)
    return [(c, 1, 2), (ml, 3, None), (mh, None, 4), (fl, None, None), (fh, None, None)]


DEPTH = [0, 1, 1, 2, 2]


def tree_mass(nodes):
    return sum(nd[0].totals()[0] / 8.0 ** d for nd, d in zip(nodes, DEPTH))


def test_refine_tree_conserves_mass_exactly():
    """Random non-equilibrium states on all five lattices, walls outside (a
    moving lid on top): sum over levels of M / 8^depth stays constant."""
    ub = np.zeros((6, 3))
    ub[3] = (0.03, 0, -0.01)
    nodes = stack(3, 4, 2, 4, 4, 0.6, (1e-5, 0, 0), outer=(NS, V), u_bc=ub)
    for k, nd in enumerate(nodes):
        random_state(nd[0], 40 + k)
    m0 = tree_mass(nodes)
    for _ in range(3):
        oracle.refine_tree_step(nodes, 4)
        assert abs(tree_mass(nodes) - m0) <= 2e-14 * m0


def test_refine_tree_uniform_moving_state_is_a_fixed_point():
    u0 = np.array([0.03, 0.0, 0.02])
    nodes = stack(2, 3, 2, 3, 3, 0.7, outer=(V, V), u_bc=np.tile(u0, (6, 1)))
    ref = []
    for nd in nodes:
        nx, ny, nz = nd[0].shape
        nd[0].init_equilibrium(np.ones((nz, ny, nx)), np.broadcast_to(u0[:, None, None, None], (3, nz, ny, nx)).copy())
        ref.append(nd[0].get_pdfs())
    oracle.refine_tree_step(nodes, 3)
    for nd, r in zip(nodes, ref):
        np.testing.assert_allclose(nd[0].get_pdfs(), r, rtol=0, atol=2e-15)


def test_refine_tree_poiseuille_exact_across_four_interfaces():
    """Fine (8 rows, 1/4 cells) / medium (8 rows, 1/2) / coarse (8) / medium /
    fine: the steady force-driven profile is the parabola of the physical
    height 20 on every level, to roundoff."""
    tau, F = 0.8, 1e-5
    nodes = stack(1, 8, 1, 8, 8, tau, (F, 0, 0))
    for nd in nodes:
        nx, ny, nz = nd[0].shape
        nd[0].init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    oracle.refine_tree_step(nodes, 12000)
    H, nu = 2 + 4 + 8 + 4 + 2, (tau - 0.5) / 3
    placed = [(nodes[3][0], 0.0, 0.25), (nodes[1][0], 2.0, 0.5), (nodes[0][0], 6.0, 1.0), (nodes[2][0], 14.0, 0.5),
              (nodes[4][0], 18.0, 0.25)]
    for s, y0, h in placed:
        _, u = s.moments()
        y = y0 + (np.arange(s.shape[1]) + 0.5) * h
        exact = F / (2 * nu) * y * (H - y)
        assert np.abs(u[0][0, :, 0] - exact).max() <= 1e-10 * exact.max()


def _emulate_tree(specs, pdfs, q):
    """One step of node 0 of a refinement tree, recursively, from
    single-lattice oracle steps (interface faces as no-slip) and the
    point-in-cell rules of the two-level emulation above."""
    cvec, _, _ = oracle.velocity_set(q)
    opp = [int(np.nonzero((cvec == -cvec[i]).all(1))[0][0]) for i in range(q)]

    def advance(k):
        shape, tau, F, lo, hi = specs[k]
        s = oracle.Sim(q, shape, bc=(P, P, NS, NS, P, P), tau=tau, force=F)
        s.set_pdfs(pdfs[k])
        s.step(1)
        pdfs[k] = s.get_pdfs()
        nxc, nyc, nzc = shape
        sums = {}
        for side, child in ((0, lo), (1, hi)):
            if child is None:
                continue
            dy = 1 if side else -1
            yc = nyc - 1 if side else 0
            yf = 0 if side else specs[child][0][1] - 1
            cnew = pdfs[k].copy()

            def cell(xf, zf, j, sign):
                px = ((xf + 0.5) / 2 + sign * cvec[j][0] * 0.5) % nxc
                pz = ((zf + 0.5) / 2 + sign * cvec[j][2] * 0.5) % nzc
                return int(math.floor(px)), int(math.floor(pz))

            acc = np.zeros((q, nzc, nxc))
            for sub in range(2):
                advance(child)
                f = pdfs[child]
                for i in range(q):
                    if cvec[i][1] != -dy:
                        continue
                    for zf in range(2 * nzc):
                        for xf in range(2 * nxc):
                            X, Z = cell(xf, zf, i, +1)
                            acc[i, Z, X] += f[opp[i], zf, yf, xf] / 8.0
                for j in range(q):
                    if cvec[j][1] != dy:
                        continue
                    for zf in range(2 * nzc):
                        for xf in range(2 * nxc):
                            X, Z = cell(xf, zf, j, -1)
                            f[j, zf, yf, xf] = cnew[opp[j], Z, yc, X]
            sums[side] = (yc, dy, acc)
        for side, (yc, dy, acc) in sums.items():
            for i in range(q):
                if cvec[i][1] == -dy:
                    pdfs[k][i, :, yc, :] = acc[i]

    advance(0)
    return pdfs


def test_refine_tree_matches_brute_force_recursion():
    q, tau, F = 19, 0.7, np.array([1e-4, -2e-5, 3e-5])
    nodes = stack(2, 3, 1, 3, 3, tau, tuple(F), q=q)
    for k, nd in enumerate(nodes):
        random_state(nd[0], 60 + k)
    specs = []
    for nd, d in zip(nodes, DEPTH):
        s = nd[0]
        specs.append((s.shape, 0.5 + 2 ** d * (tau - 0.5), tuple(F / 2 ** d), nd[1], nd[2]))
    ref = _emulate_tree(specs, [nd[0].get_pdfs() for nd in nodes], q)
    oracle.refine_tree_step(nodes, 1)
    for nd, r in zip(nodes, ref):
        np.testing.assert_allclose(nd[0].get_pdfs(), r, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("case", ["child_before_parent", "two_parents", "orphan", "face_without_child",
                                  "child_facing_parent"])
def test_refine_tree_rejects_malformed_trees(case):
    nodes = stack(2, 3, 1, 3, 3, 0.7)
    if case == "child_before_parent":
        nodes = [nodes[1], nodes[0]] + nodes[2:]
    elif case == "two_parents":
        nodes[2] = (nodes[2][0], None, 3)
    elif case == "orphan":
        nodes[1] = (nodes[1][0], None, None)
    elif case == "face_without_child":
        nodes[0] = (nodes[0][0], 1, None)
        nodes[2] = (nodes[2][0], None, None)
        nodes = nodes[:2] + nodes[3:4]
    elif case == "child_facing_parent":
        nodes[1] = (nodes[1][0], None, 3)
    with pytest.raises(ValueError):
        oracle.refine_tree_step(nodes, 1)

"""Host check of the Esoteric Twist addressing used by the GPU kernel.

A plain Python emulation of the in-place scheme (read f_i at
x + max(-c_i, 0) from slot P(i), write f*_i to x + max(c_i, 0) into slot
P(opposite(i)), or into slot P(i) when the link is cut by a wall or a solid
neighbour; P alternates between identity and opposite; one ghost layer
beyond every non-periodic + face) on small lattices with walls and solids.
Per step it checks that every index lies inside the store, that no slot is
written twice, and that no slot written by one cell is read by another (so
the in-place update is race free; a cut link writes into the slot its solid
neighbour or the ghost layer would read, and leaves unwritten the slot it
reads itself), and that the populations equal the oracle's two-lattice run
after odd and even step counts.  The collision of each cell
is the oracle's own, so only the streaming is under test.
"""
import numpy as np
import pytest

import oracle

NOSLIP, PERIODIC = oracle.BC_NOSLIP, oracle.BC_PERIODIC


class EtEmulation:
    def __init__(self, q, shape, bc, solid, tau, force):
        self.q, self.shape, self.bc = q, shape, bc
        self.c, self.w, self.opp = oracle.velocity_set(q)
        nx, ny, nz = shape
        self.per = [bc[2 * k] == PERIODIC for k in range(3)]
        self.store = [n + (0 if p else 1) for n, p in zip(shape, self.per)]  # sx, sy, sz
        sx, sy, sz = self.store
        self.A = np.full((q, sz, sy, sx), np.nan)
        self.solid = solid
        self.tau, self.force = tau, force
        self.t = 0

    def _loc(self, x, off):
        """x + off (off in {0, 1}^3): wrapped on periodic axes, the ghost layer otherwise."""
        out = []
        for k in range(3):
            v = x[k] + off[k]
            if v == self.shape[k]:
                v = 0 if self.per[k] else self.shape[k]
            assert 0 <= v < self.store[k]
            out.append(v)
        return tuple(out)

    def _cut(self, x, i):
        """Link x -> x + c_i leaves through a non-periodic face or ends in a solid cell."""
        y = []
        for k in range(3):
            v = x[k] + self.c[i, k]
            if v < 0 or v >= self.shape[k]:
                if not self.per[k]:
                    return True
                v %= self.shape[k]
            y.append(v)
        return bool(self.solid[y[2], y[1], y[0]])

    def _P(self, i):
        return self.opp[i] if self.t & 1 else i

    def cells(self):
        nx, ny, nz = self.shape
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if not self.solid[z, y, x]:
                        yield (x, y, z)

    def set_canonical(self, f):
        assert self.t == 0
        for x in self.cells():
            for i in range(self.q):
                lx = self._loc(x, tuple(int(v < 0) for v in self.c[i]))
                self.A[i, lx[2], lx[1], lx[0]] = f[i, x[2], x[1], x[0]]

    def get_canonical(self):
        nx, ny, nz = self.shape
        f = np.zeros((self.q, nz, ny, nx))
        for x in self.cells():
            for i in range(self.q):
                lx = self._loc(x, tuple(int(v < 0) for v in self.c[i]))
                f[i, x[2], x[1], x[0]] = self.A[self._P(i), lx[2], lx[1], lx[0]]
        return f

    def step(self):
        old = self.A.copy()
        reader, writer = {}, {}
        for x in self.cells():
            f = np.zeros(self.q)
            for i in range(self.q):
                lx = self._loc(x, tuple(int(v < 0) for v in self.c[i]))
                key = (int(self._P(i)),) + lx
                assert key not in reader, "slot read twice in one step"
                reader[key] = x
                f[i] = old[key[0], lx[2], lx[1], lx[0]]
            assert np.all(np.isfinite(f)), "read a slot nobody wrote"
            fs, _ = oracle.collide(self.q, f, self.tau, F=self.force)
            for i in range(self.q):
                lx = self._loc(x, tuple(int(v > 0) for v in self.c[i]))
                slot = int(self._P(i) if self._cut(x, i) else self._P(self.opp[i]))
                key = (slot,) + lx
                assert key not in writer, "slot written twice in one step"
                writer[key] = x
                self.A[slot, lx[2], lx[1], lx[0]] = fs[i]
        for key, x in writer.items():
            assert reader.get(key, x) == x, "slot written by one cell and read by another"
        self.t += 1


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("walls", ["periodic", "channel", "box"])
def test_et_scheme_matches_two_lattice_oracle(q, walls):
    shape = (6, 5, 4)
    nx, ny, nz = shape
    bc = {"periodic": (PERIODIC,) * 6,
          "channel": (PERIODIC, PERIODIC, NOSLIP, NOSLIP, PERIODIC, PERIODIC),
          "box": (NOSLIP,) * 6}[walls]
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[1, 2, 2:4] = 1
    solid[2, 2, 3] = 1
    solid[nz - 1, ny - 1, nx - 1] = 1  # a solid cell in the + corner
    tau, F = 0.7, (2e-4, -1e-4, 5e-5)
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.02 * rng.uniform(-1, 1, (nz, ny, nx))
    u = 0.03 * rng.uniform(-1, 1, (3, nz, ny, nx))
    u[:, solid == 1] = 0.0
    o = oracle.Sim(q, shape, bc=bc, tau=tau, force=F, solid=solid)
    o.init_equilibrium(rho, u)
    e = EtEmulation(q, shape, bc, solid, tau, F)
    e.set_canonical(o.get_pdfs())
    fluid = solid == 0
    for k in range(1, 5):
        o.step(1)
        e.step()
        a, b = e.get_canonical()[:, fluid], o.get_pdfs()[:, fluid]
        assert np.max(np.abs(a - b)) <= 1e-14, (walls, k)

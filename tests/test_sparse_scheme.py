"""Host check of the sparse (fluid-cells-only) addressing used by the GPU
kernel.

A plain Python emulation of the scheme: fluid cells numbered in row order
and stored in chunks of 64 ([chunk][q][64]); a neighbour table per fluid
cell ([chunk][q-1][64]) holding the fluid index of x + c_j or a cut code;
the AA pattern over the fluid index (even step: own slots, opposite(i)
written; odd step: slot opposite(i) of x - c_i read, slot i of x + c_i
written, the cell's own slot standing in for cut links).  Per step it
checks that every index lies inside the stores, that no slot is written
twice, that no slot written by one cell is read by another, and that the
populations equal the oracle's two-lattice run after odd and even step
counts.  The collision of each cell is the oracle's own, so only the
addressing is under test.
"""
import numpy as np
import pytest

import oracle

NOSLIP, PERIODIC = oracle.BC_NOSLIP, oracle.BC_PERIODIC
CHUNK = 64
CUT = -1


class SparseEmulation:
    def __init__(self, q, shape, bc, solid, tau, force):
        self.q, self.shape, self.bc = q, shape, bc
        self.c, self.w, self.opp = oracle.velocity_set(q)
        nx, ny, nz = shape
        self.per = [bc[2 * k] == PERIODIC for k in range(3)]
        flat = solid.reshape(-1)
        self.fmap = np.full(flat.size, -1, np.int64)
        self.fcell = np.flatnonzero(flat == 0)
        self.fmap[self.fcell] = np.arange(self.fcell.size)
        self.nf = self.fcell.size
        self.chunks = (self.nf + CHUNK - 1) // CHUNK
        self.A = np.full(self.chunks * q * CHUNK, np.nan)
        self.T = np.full(self.chunks * (q - 1) * CHUNK, -7, np.int64)
        for k, cell in enumerate(self.fcell):
            x, y, z = cell % nx, (cell // nx) % ny, cell // (nx * ny)
            for j in range(1, q):
                p, cut = [x, y, z], False
                for a in range(3):
                    p[a] += self.c[j, a]
                    if not 0 <= p[a] < shape[a]:
                        if self.per[a]:
                            p[a] %= shape[a]
                        else:
                            cut = True
                e = CUT if cut else self.fmap[(p[2] * ny + p[1]) * nx + p[0]]
                self.T[self.tidx(k, j)] = CUT if e < 0 else e
        assert np.all(self.T[[self.tidx(k, j) for k in range(self.nf) for j in range(1, q)]] != -7)
        self.tau, self.force = tau, force
        self.t = 0

    def pidx(self, k, i):
        r = (k // CHUNK * self.q + i) * CHUNK + k % CHUNK
        assert 0 <= k < self.nf and 0 <= r < self.A.size
        return r

    def tidx(self, k, j):
        r = (k // CHUNK * (self.q - 1) + j - 1) * CHUNK + k % CHUNK
        assert 0 <= r < self.T.size
        return r

    def set_canonical(self, f):
        nx, ny, _ = self.shape
        for k, cell in enumerate(self.fcell):
            z, y, x = cell // (nx * ny), (cell // nx) % ny, cell % nx
            for i in range(self.q):
                self.A[self.pidx(k, i)] = f[i, z, y, x]

    def _read_index(self, k, i):
        if i == 0 or self.t % 2 == 0:
            return self.pidx(k, i)
        s = self.T[self.tidx(k, self.opp[i])]  # neighbour x - c_i
        return self.pidx(k, i) if s == CUT else self.pidx(s, self.opp[i])

    def get_canonical(self):
        nx, ny, nz = self.shape
        f = np.zeros((self.q, nz, ny, nx))
        for k, cell in enumerate(self.fcell):
            z, y, x = cell // (nx * ny), (cell // nx) % ny, cell % nx
            for i in range(self.q):
                f[i, z, y, x] = self.A[self._read_index(k, i)]
        return f

    def step(self):
        old = self.A.copy()
        reader, writer = {}, {}
        for k in range(self.nf):
            f = np.zeros(self.q)
            for i in range(self.q):
                r = self._read_index(k, i)
                assert r not in reader, "slot read twice in one step"
                reader[r] = k
                f[i] = old[r]
            assert np.all(np.isfinite(f)), "read a slot nobody wrote"
            fs, _ = oracle.collide(self.q, f, self.tau, F=self.force)
            for i in range(self.q):
                if self.t % 2 == 0:
                    r = self.pidx(k, self.opp[i])
                elif i == 0:
                    r = self.pidx(k, 0)
                else:
                    e = self.T[self.tidx(k, i)]  # neighbour x + c_i
                    r = self.pidx(k, self.opp[i]) if e == CUT else self.pidx(e, i)
                assert r not in writer, "slot written twice in one step"
                writer[r] = k
                self.A[r] = fs[i]
        for r, k in writer.items():
            assert reader.get(r, k) == k, "slot written by one cell and read by another"
        assert set(reader) == set(writer), "the read set and the write set differ"
        self.t += 1


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("walls", ["periodic", "channel", "box"])
def test_sparse_scheme_matches_two_lattice_oracle(q, walls):
    shape = (7, 5, 4)
    nx, ny, nz = shape
    bc = {"periodic": (PERIODIC,) * 6,
          "channel": (PERIODIC, PERIODIC, NOSLIP, NOSLIP, PERIODIC, PERIODIC),
          "box": (NOSLIP,) * 6}[walls]
    rng = np.random.default_rng(17)
    solid = (rng.uniform(size=(nz, ny, nx)) < 0.4).astype(np.uint8)  # more than two chunks of fluid cells
    tau, F = 0.7, (2e-4, -1e-4, 5e-5)
    rho = 1.0 + 0.02 * rng.uniform(-1, 1, (nz, ny, nx))
    u = 0.03 * rng.uniform(-1, 1, (3, nz, ny, nx))
    u[:, solid == 1] = 0.0
    o = oracle.Sim(q, shape, bc=bc, tau=tau, force=F, solid=solid)
    o.init_equilibrium(rho, u)
    e = SparseEmulation(q, shape, bc, solid, tau, F)
    assert e.nf > CHUNK and e.nf % CHUNK != 0
    e.set_canonical(o.get_pdfs())
    fluid = solid == 0
    for k in range(1, 5):
        o.step(1)
        e.step()
        a, b = e.get_canonical()[:, fluid], o.get_pdfs()[:, fluid]
        assert np.max(np.abs(a - b)) <= 1e-14, (walls, k)

"""FP64 CPU oracle for the lattice Boltzmann stream-collide path.

TEST INFRASTRUCTURE ONLY.  Tests, the package smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports it.  It is a
plain, slow two-lattice implementation of the paper's Eq. (1) (collision,
read as TRT with Guo forcing) and Eq. (2) (streaming) written in C
(``lbm_oracle.c``) and driven here through ctypes.  It shares no code with
the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MLP_NPARAM = 1313
MLP_NNORM = 24

BC_PERIODIC, BC_NOSLIP, BC_VELOCITY, BC_PRESSURE, BC_INTERFACE = 0, 1, 2, 3, 4
CL_NONE, CL_SMAG, CL_MLP = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
             "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_velocity_set.argtypes = [ctypes.c_int, _I, _D, _I]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_round_bf16.argtypes = [ctypes.c_double]
        L.orc_round_bf16.restype = ctypes.c_double
        L.orc_mlp_forward.argtypes = [_D, _D, _D, ctypes.c_int64, ctypes.c_int, _D]
        L.orc_mlp_loss_grad.argtypes = [_D, _D, _D, _D, ctypes.c_int64, _D]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_adam.argtypes = [_D, _D, _D, _D, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_smagorinsky_tau.argtypes = [ctypes.c_double] * 4
        L.orc_smagorinsky_tau.restype = ctypes.c_double
        L.orc_features.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _D, _D, _U8,
                                 ctypes.c_double, ctypes.c_double, _D, ctypes.c_int, ctypes.c_double]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_set_mlp.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_fallbacks.argtypes = [ctypes.c_void_p]
        L.orc_fallbacks.restype = ctypes.c_int64
        L.orc_init_equilibrium.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_set_pdfs.argtypes = [ctypes.c_void_p, _D]
        L.orc_get_pdfs.argtypes = [ctypes.c_void_p, _D]
        L.orc_collide.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_double, _D, ctypes.c_int,
                                  ctypes.c_double, _D, _D]
        L.orc_noneq_flux.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_mrt_basis.argtypes = [ctypes.c_int, _D, _I]
        L.orc_set_mrt.argtypes = [ctypes.c_void_p, _D]
        L.orc_collide_mrt.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D, ctypes.c_int, ctypes.c_double, _D,
                                      _D]
        L.orc_set_hrr.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_hrr_norms.argtypes = [_D]
        L.orc_collide_hrr.argtypes = [_D, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_fd_gradient.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_refine_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.orc_refine_tree_step.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int64]
        L.orc_moments.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_totals.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_probe.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_int, ctypes.c_int64, _I64, _D]
        L.orc_box_filter4.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, _D]
        L.orc_strain.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _D, _D]
        L.orc_closure_dataset.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _D, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, _D, _D]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def velocity_set(q: int):
    """Return (c[q,3] int, w[q] float64, opp[q] int)."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    rc = lib().orc_velocity_set(q, c.ctypes.data_as(_I), _d(w), opp.ctypes.data_as(_I))
    if rc != 0:
        raise ValueError(f"unknown stencil {q}")
    return c.astype(np.int64), w, opp.astype(np.int64)


def equilibrium(q: int, rho: float, u) -> np.ndarray:
    u = _f64(u)
    out = np.zeros(q)
    lib().orc_equilibrium(q, float(rho), _d(u), _d(out))
    return out


def collide(q, f, tau, magic=3.0 / 16.0, F=(0.0, 0.0, 0.0), closure=CL_NONE, cs=0.1):
    """Post-collision populations of one cell; returns (fstar, tau_used)."""
    f = _f64(f)
    F = _f64(F)
    out = np.zeros(q)
    tu = np.zeros(1)
    lib().orc_collide(q, _d(f), float(tau), float(magic), _d(F), int(closure), float(cs), _d(out), _d(tu))
    return out, float(tu[0])


MRT_DHUMIERES = (1.19, 1.4, 1.2, 1.4, 1.98)  # s_e, s_eps, s_q, s_pi, s_m


def mrt_basis(q):
    """Moment matrix M[q, q] and the rate group of every row."""
    M = np.zeros((q, q))
    g = np.zeros(q, dtype=np.int32)
    if lib().orc_mrt_basis(q, _d(M), g.ctypes.data_as(_I)) != 0:
        raise ValueError(q)
    return M, g


def collide_mrt(q, f, tau, rates=MRT_DHUMIERES, F=(0.0, 0.0, 0.0), closure=CL_NONE, cs=0.1):
    f = _f64(f)
    F = _f64(F)
    r = _f64(rates)
    out = np.zeros(q)
    tu = np.zeros(1)
    if lib().orc_collide_mrt(q, _d(f), float(tau), _d(r), _d(F), int(closure), float(cs), _d(out), _d(tu)) != 0:
        raise ValueError("singular MRT basis")
    return out, float(tu[0])


def hrr_norms() -> np.ndarray:
    """Lattice norms of the six D3Q19 third-order Hermite combinations."""
    out = np.zeros(6)
    lib().orc_hrr_norms(_d(out))
    return out


def collide_hrr(f, tau, sigma, F=(0.0, 0.0, 0.0), grad=None) -> np.ndarray:
    """One D3Q19 HRR collision of a single cell; grad[3][3] = d u_a / d x_b
    of the velocity field (zero if None)."""
    f = _f64(f)
    F = _f64(F)
    G = _f64(np.zeros((3, 3)) if grad is None else grad).reshape(9)
    out = np.zeros(19)
    lib().orc_collide_hrr(_d(f), float(tau), float(sigma), _d(F), _d(G), _d(out))
    return out


def noneq_flux(q, f, F=(0.0, 0.0, 0.0)) -> np.ndarray:
    f = _f64(f)
    F = _f64(F)
    out = np.zeros(6)
    lib().orc_noneq_flux(q, _d(f), _d(F), _d(out))
    return out


def round_bf16(x: float) -> float:
    return lib().orc_round_bf16(float(x))


def smagorinsky_tau(tau, cs, Q, rho) -> float:
    return lib().orc_smagorinsky_tau(float(tau), float(cs), float(Q), float(rho))


def features(P6, rho, tau, cs) -> np.ndarray:
    P6 = _f64(P6)
    out = np.zeros(6)
    lib().orc_features(_d(P6), float(rho), float(tau), float(cs), _d(out))
    return out


def mlp_forward(params, norm, x, bf16=False) -> np.ndarray:
    params, norm, x = _f64(params), _f64(norm), _f64(x).reshape(-1, 6)
    y = np.zeros(x.shape[0])
    lib().orc_mlp_forward(_d(params), _d(norm), _d(x), x.shape[0], int(bool(bf16)), _d(y))
    return y


def mlp_loss_grad(params, norm, x, t):
    params, norm, x, t = _f64(params), _f64(norm), _f64(x).reshape(-1, 6), _f64(t)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_d(params), _d(norm), _d(x), _d(t), x.shape[0], _d(g))
    return loss, g


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays p, m, v."""
    g = _f64(g)
    lib().orc_adam(_d(p), _d(g), _d(m), _d(v), p.size, int(step), float(lr), float(beta1), float(beta2),
                   float(eps))


def box_filter4(rho, u) -> np.ndarray:
    """rho[nz,ny,nx], u[3,nz,ny,nx] -> out[10, nz/4, ny/4, nx/4]."""
    rho = _f64(rho)
    u = _f64(u)
    nz, ny, nx = rho.shape
    out = np.zeros((10, nz // 4, ny // 4, nx // 4))
    lib().orc_box_filter4(nx, ny, nz, _d(rho), _d(u), _d(out))
    return out


def strain(u, periodic) -> np.ndarray:
    u = _f64(u)
    _, cz, cy, cx = u.shape
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    out = np.zeros((6, cz, cy, cx))
    lib().orc_strain(cx, cy, cz, per.ctypes.data_as(_I), _d(u), _d(out))
    return out


def closure_dataset(filt, periodic, tau, cs=0.1, eps=1e-30):
    filt = _f64(filt)
    _, cz, cy, cx = filt.shape
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    n = cx * cy * cz
    x = np.zeros((n, 6))
    t = np.zeros(n)
    lib().orc_closure_dataset(cx, cy, cz, per.ctypes.data_as(_I), _d(filt), float(tau), float(cs), float(eps),
                              _d(x), _d(t))
    return x, t


def refine_tree_step(nodes, n=1):
    """Advance a hierarchy of 2:1 levels: nodes is a list of (Sim, lo, hi)
    with lo / hi the indices of the finer Sims below / above (None for
    none), children after their parent, node 0 the coarsest; node 0 takes n
    steps, a node at depth d 2^d n steps."""
    k = len(nodes)
    sims = (ctypes.c_void_p * k)(*[nd[0]._h.value for nd in nodes])
    lo = (ctypes.c_int * k)(*[-1 if nd[1] is None else int(nd[1]) for nd in nodes])
    hi = (ctypes.c_int * k)(*[-1 if nd[2] is None else int(nd[2]) for nd in nodes])
    if lib().orc_refine_tree_step(sims, lo, hi, k, int(n)) != 0:
        raise ValueError("these lattices do not form a 2:1 refinement tree")


def refine_step(coarse, fine_lo=None, fine_hi=None, n=1):
    """Advance a 2:1 refinement: the coarse Sim n steps and the fine Sims
    (below its -y face / above its +y face, nullable) 2n steps, exchanging the
    packets that cross the BC_INTERFACE faces."""
    lo = fine_lo._h if fine_lo is not None else None
    hi = fine_hi._h if fine_hi is not None else None
    if lib().orc_refine_step(coarse._h, lo, hi, int(n)) != 0:
        raise ValueError("these lattices do not form a 2:1 refinement")


class Sim:
    """Two-lattice FP64 simulation.  Arrays are [q][nz][ny][nx] (x fastest)."""

    def __init__(self, q, shape, bc=(0, 0, 0, 0, 0, 0), tau=0.6, magic=3.0 / 16.0, force=(0.0, 0.0, 0.0),
                 u_bc=None, rho_bc=None, solid=None, closure=CL_NONE, cs=0.1):
        nx, ny, nz = shape
        self.q, self.shape = q, (nx, ny, nz)
        self.n = nx * ny * nz
        bc_a = np.ascontiguousarray(bc, dtype=np.int32)
        ubc = _f64(np.zeros((6, 3)) if u_bc is None else u_bc).reshape(6, 3)
        rbc = _f64(np.ones(6) if rho_bc is None else rho_bc)
        F = _f64(force)
        self._solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        sp = self._solid.ctypes.data_as(_U8) if self._solid is not None else None
        h = lib().orc_create(q, nx, ny, nz, bc_a.ctypes.data_as(_I), _d(ubc), _d(rbc), sp, float(tau),
                             float(magic), _d(F), int(closure), float(cs))
        if not h:
            raise ValueError("oracle: invalid arguments")
        self._h = ctypes.c_void_p(h)
        self.force = F

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def set_mrt(self, rates=MRT_DHUMIERES):
        if lib().orc_set_mrt(self._h, _d(_f64(rates))) != 0:
            raise ValueError("singular MRT basis")

    def set_hrr(self, sigma=0.995):
        """Hybrid recursive regularised collision (D3Q19); sigma is the weight
        of the projected non-equilibrium flux against the finite-difference one."""
        if lib().orc_set_hrr(self._h, float(sigma)) != 0:
            raise ValueError("HRR needs D3Q19 and sigma in [0, 1]")

    def fd_gradient(self, u):
        """Velocity gradient [3, 3, nz, ny, nx] (d u_a / d x_b) of a field u [3, nz, ny, nx]
        with the HRR finite-difference rules at walls, solids and faces."""
        nx, ny, nz = self.shape
        u = _f64(u).reshape(3, -1)
        out = np.zeros((3, 3, nz, ny, nx))
        lib().orc_fd_gradient(self._h, _d(u), _d(out))
        return out

    def set_mlp(self, params, norm):
        lib().orc_set_mlp(self._h, _d(_f64(params)), _d(_f64(norm)))

    @property
    def fallbacks(self) -> int:
        return int(lib().orc_fallbacks(self._h))

    def init_equilibrium(self, rho, u):
        rho = _f64(rho).reshape(-1)
        u = _f64(u).reshape(3, -1)
        lib().orc_init_equilibrium(self._h, _d(rho), _d(u))

    def set_pdfs(self, f):
        f = _f64(f)
        assert f.size == self.q * self.n
        lib().orc_set_pdfs(self._h, _d(f))

    def get_pdfs(self) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.zeros((self.q, nz, ny, nx))
        lib().orc_get_pdfs(self._h, _d(out))
        return out

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def moments(self):
        nx, ny, nz = self.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        lib().orc_moments(self._h, _d(rho), _d(u))
        return rho, u

    def totals(self):
        m = np.zeros(1)
        p = np.zeros(3)
        lib().orc_totals(self._h, _d(m), _d(p))
        return float(m[0]), p

    def probe(self, rho, u, k, cells) -> np.ndarray:
        """Canonical state at `cells` after k steps from f^eq(rho, u), [len(cells), q]."""
        rho = _f64(rho).reshape(-1)
        u = _f64(u).reshape(3, -1)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((cells.size, self.q))
        lib().orc_probe(self._h, _d(rho), _d(u), int(k), cells.size, cells.ctypes.data_as(_I64), _d(out))
        return out

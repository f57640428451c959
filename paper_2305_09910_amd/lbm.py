"""ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  torch provides the device memory (the context workspace and the
field tensors) and the stream.  If the library is not built the binding
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
BC = {"periodic": 0, "noslip": 1, "velocity": 2, "pressure": 3, "interface": 4}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
CLOSURE = {"none": 0, "smagorinsky": 1, "mlp": 2}
COLLISION = {"trt": 0, "mrt": 1, "hrr": 2}
STREAMING = {"aa": 0, "et": 1, "sparse": 2}
MRT_DEFAULT_RATES = (1.19, 1.4, 1.2, 1.4, 1.98)
MLP_NPARAM, MLP_NNORM = 1313, 24

_ERRNAMES = {-1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}

EXPORTED = [
    "lbm_domain_defaults", "lbm_workspace_bytes", "lbm_workspace_bytes_flags", "lbm_create", "lbm_destroy", "lbm_last_error",
    "lbm_init_equilibrium", "lbm_set_pdfs", "lbm_get_pdfs", "lbm_gather_pdfs", "lbm_step", "lbm_time",
    "lbm_moments", "lbm_totals", "lbm_state_bytes", "lbm_save_state", "lbm_load_state",
    "lbm_set_closure_weights", "lbm_closure_fallbacks", "lbm_box_filter4", "lbm_closure_dataset",
    "lbm_mlp_forward", "lbm_mlp_work_bytes", "lbm_mlp_loss_grad", "lbm_mlp_loss_grad_noalloc", "lbm_mlp_adam",
    "lbm_stream_copy", "lbm_refine_work_bytes", "lbm_refine_step", "lbm_refine_tree_step", "lbm_closure_features",
]


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Domain(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("u_bc", (ctypes.c_double * 3) * 6),
        ("rho_bc", ctypes.c_double * 6),
        ("storage", ctypes.c_int32), ("closure", ctypes.c_int32), ("use_flags", ctypes.c_int32),
        ("magic", ctypes.c_double), ("cs_smag", ctypes.c_double),
        ("collision", ctypes.c_int32), ("mrt_rates", ctypes.c_double * 5), ("streaming", ctypes.c_int32),
        ("hrr_sigma", ctypes.c_double),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


class RefineNode(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("fine_lo", ctypes.c_int32), ("fine_hi", ctypes.c_int32),
                ("work_dev", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2305_09910_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
        DP = ctypes.POINTER(Domain)
        sig = {
            "lbm_domain_defaults": (None, [DP]),
            "lbm_workspace_bytes": (ctypes.c_int, [DP, ctypes.c_int, ctypes.POINTER(SZ)]),
            "lbm_workspace_bytes_flags": (ctypes.c_int, [DP, ctypes.c_int, P, ctypes.POINTER(SZ)]),
            "lbm_create": (ctypes.c_int, [DP, ctypes.c_int, P, D, ctypes.POINTER(D), ctypes.POINTER(P)]),
            "lbm_destroy": (ctypes.c_int, [P]),
            "lbm_last_error": (ctypes.c_char_p, [P]),
            "lbm_init_equilibrium": (ctypes.c_int, [P, P, P]),
            "lbm_set_pdfs": (ctypes.c_int, [P, P]),
            "lbm_get_pdfs": (ctypes.c_int, [P, P]),
            "lbm_gather_pdfs": (ctypes.c_int, [P, P, I64, P]),
            "lbm_step": (ctypes.c_int, [P, I64]),
            "lbm_time": (I64, [P]),
            "lbm_moments": (ctypes.c_int, [P, P, P]),
            "lbm_totals": (ctypes.c_int, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
            "lbm_state_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
            "lbm_save_state": (ctypes.c_int, [P, P, ctypes.POINTER(I64)]),
            "lbm_load_state": (ctypes.c_int, [P, P, I64]),
            "lbm_set_closure_weights": (ctypes.c_int, [P, P, SZ]),
            "lbm_closure_fallbacks": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
            "lbm_box_filter4": (ctypes.c_int, [I32, I32, I32, P, P, P, P]),
            "lbm_closure_dataset": (ctypes.c_int, [I32, I32, I32, ctypes.POINTER(I32), P, D, D, P, P, P]),
            "lbm_mlp_forward": (ctypes.c_int, [P, P, I64, P, P]),
            "lbm_mlp_work_bytes": (SZ, [I64]),
            "lbm_mlp_loss_grad": (ctypes.c_int, [P, P, P, I64, P, P, P, P]),
            "lbm_mlp_loss_grad_noalloc": (ctypes.c_int, [P, P, P, I64, P, P, P]),
            "lbm_mlp_adam": (ctypes.c_int, [P, P, P, P, I64, D, D, D, D, P]),
            "lbm_stream_copy": (ctypes.c_int, [P, P, SZ, P]),
            "lbm_refine_work_bytes": (ctypes.c_int, [DP, ctypes.c_int, ctypes.POINTER(SZ)]),
            "lbm_refine_step": (ctypes.c_int, [P, P, P, P, SZ, I64]),
            "lbm_refine_tree_step": (ctypes.c_int, [ctypes.POINTER(RefineNode), I32, I64]),
            "lbm_closure_features": (ctypes.c_int, [P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, ctx=None):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LBMError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _dev(t, dtype, device):
    """Contiguous device tensor of the given dtype from a numpy array or tensor."""
    torch = _torch()
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


def make_domain(shape, bc=("periodic",) * 6, u_bc=None, rho_bc=None, storage="f32", closure="none",
                use_flags=False, magic=3.0 / 16.0, cs=0.1, collision="trt", mrt_rates=None,
                streaming="aa", hrr_sigma=None) -> Domain:
    d = Domain()
    lib().lbm_domain_defaults(ctypes.byref(d))
    d.nx, d.ny, d.nz = (int(v) for v in shape)
    for f in range(6):
        d.bc[f] = BC[bc[f]] if isinstance(bc[f], str) else int(bc[f])
        if u_bc is not None:
            for a in range(3):
                d.u_bc[f][a] = float(u_bc[f][a])
        if rho_bc is not None:
            d.rho_bc[f] = float(rho_bc[f])
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.closure = CLOSURE[closure] if isinstance(closure, str) else int(closure)
    d.use_flags = int(bool(use_flags))
    d.magic = float(magic)
    d.cs_smag = float(cs)
    d.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    if mrt_rates is not None:
        for k in range(5):
            d.mrt_rates[k] = float(mrt_rates[k])
    d.streaming = STREAMING[streaming] if isinstance(streaming, str) else int(streaming)
    if hrr_sigma is not None:
        d.hrr_sigma = float(hrr_sigma)
    return d


def workspace_bytes(domain: Domain, q: int, flags: Optional[np.ndarray] = None) -> int:
    """Workspace bytes of a context; with `flags` (uint8 per cell) sized for
    those solids (sparse addressing stores fluid cells only)."""
    out = ctypes.c_size_t(0)
    if flags is None:
        _check(lib().lbm_workspace_bytes(ctypes.byref(domain), int(q), ctypes.byref(out)))
    else:
        f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
        _check(lib().lbm_workspace_bytes_flags(ctypes.byref(domain), int(q), f.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(out)))
    return int(out.value)


class Lattice:
    """One lattice on one GPU.  shape = (nx, ny, nz); fields are [nz, ny, nx].

    streaming: "aa" (AA pattern), "et" (Esoteric Twist) or "sparse" (the AA
    pattern over the fluid cells only, for domains that `solid` fills to a
    large part; the workspace is then sized by the fluid cells).
    collision: "trt", "mrt" or "hrr" (D3Q19, AA, no closure; hrr_sigma is
    the weight of the projected non-equilibrium flux)."""

    def __init__(self, shape, q: int = 19, tau: float = 0.6, force=(0.0, 0.0, 0.0), bc=("periodic",) * 6,
                 u_bc=None, rho_bc=None, solid: Optional[np.ndarray] = None, storage="f32", closure="none",
                 magic=3.0 / 16.0, cs=0.1, collision="trt", mrt_rates=None, streaming="aa", hrr_sigma=None,
                 device="cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        self.q = int(q)
        self.shape = tuple(int(v) for v in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.domain = make_domain(shape, bc, u_bc, rho_bc, storage, closure, solid is not None, magic, cs,
                                  collision, mrt_rates, streaming, hrr_sigma)
        flags = None
        if solid is not None:
            self._flags = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
            assert self._flags.size == self.n
            flags = self._flags.ctypes.data_as(ctypes.c_void_p)
        nbytes = workspace_bytes(self.domain, self.q, None if solid is None else self._flags)
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.domain.workspace = self.workspace.data_ptr()
        self.domain.workspace_bytes = nbytes
        self.stream = torch.cuda.current_stream(self.device)
        self.domain.stream = self.stream.cuda_stream
        F = (ctypes.c_double * 3)(*[float(v) for v in force])
        h = ctypes.c_void_p(0)
        _check(lib().lbm_create(ctypes.byref(self.domain), self.q, flags, float(tau), F, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, rc):
        _check(rc, self._h)

    # ---- state ------------------------------------------------------------
    def init_equilibrium(self, rho, u):
        torch = _torch()
        r = _dev(rho, torch.float64, self.device).reshape(-1)
        v = _dev(u, torch.float64, self.device).reshape(3, -1)
        assert r.numel() == self.n and v.shape[1] == self.n
        self._ck(lib().lbm_init_equilibrium(self._h, r.data_ptr(), v.data_ptr()))
        self._keep = (r, v)

    def set_pdfs(self, f):
        torch = _torch()
        t = _dev(f, torch.float64, self.device).reshape(-1)
        assert t.numel() == self.q * self.n
        self._ck(lib().lbm_set_pdfs(self._h, t.data_ptr()))
        self._keep = (t,)

    def get_pdfs(self):
        """Canonical FP64 populations as a torch tensor [q, nz, ny, nx] on the device."""
        torch = _torch()
        nx, ny, nz = self.shape
        out = torch.empty((self.q, nz, ny, nx), dtype=torch.float64, device=self.device)
        self._ck(lib().lbm_get_pdfs(self._h, out.data_ptr()))
        return out

    def gather(self, cells):
        torch = _torch()
        c = _dev(np.asarray(cells, dtype=np.int64), torch.int64, self.device).reshape(-1)
        out = torch.empty((c.numel(), self.q), dtype=torch.float64, device=self.device)
        self._ck(lib().lbm_gather_pdfs(self._h, c.data_ptr(), c.numel(), out.data_ptr()))
        self._keep = (c,)
        return out

    def step(self, n: int = 1):
        self._ck(lib().lbm_step(self._h, int(n)))

    @property
    def time(self) -> int:
        return int(lib().lbm_time(self._h))

    def moments(self):
        torch = _torch()
        nx, ny, nz = self.shape
        rho = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device)
        u = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=self.device)
        self._ck(lib().lbm_moments(self._h, rho.data_ptr(), u.data_ptr()))
        return rho, u

    def totals(self, check: bool = True):
        m = ctypes.c_double(0)
        p = (ctypes.c_double * 3)()
        rc = lib().lbm_totals(self._h, ctypes.byref(m), p)
        if check:
            self._ck(rc)
            return float(m.value), np.array(list(p))
        return rc, float(m.value), np.array(list(p))

    def state_bytes(self) -> int:
        out = ctypes.c_size_t(0)
        self._ck(lib().lbm_state_bytes(self._h, ctypes.byref(out)))
        return int(out.value)

    def save_state(self):
        torch = _torch()
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        t = ctypes.c_int64(0)
        self._ck(lib().lbm_save_state(self._h, buf.data_ptr(), ctypes.byref(t)))
        return buf, int(t.value)

    def load_state(self, buf, time: int):
        self._ck(lib().lbm_load_state(self._h, buf.data_ptr(), int(time)))
        self._keep = (buf,)

    def set_closure_weights(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        self._ck(lib().lbm_set_closure_weights(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))

    def closure_features(self):
        """The closure's six inputs of every cell from the current state, as
        the fused closure computes them: [n, 6] FP32 (solid cells NaN)."""
        torch = _torch()
        x = torch.empty((self.n, 6), dtype=torch.float32, device=self.device)
        self._ck(lib().lbm_closure_features(self._h, x.data_ptr()))
        return x

    def closure_fallbacks(self) -> int:
        c = ctypes.c_int64(0)
        self._ck(lib().lbm_closure_fallbacks(self._h, ctypes.byref(c)))
        return int(c.value)


# ---- free functions (closure training path, bandwidth probe) ---------------
def box_filter4(rho, u, stream=None):
    """rho [nz,ny,nx], u [3,nz,ny,nx] FP32 device tensors -> [10, nz/4, ny/4, nx/4]."""
    torch = _torch()
    nz, ny, nx = rho.shape
    out = torch.empty((10, nz // 4, ny // 4, nx // 4), dtype=torch.float32, device=rho.device)
    s = stream if stream is not None else _stream_ptr(rho.device)
    _check(lib().lbm_box_filter4(nx, ny, nz, rho.contiguous().data_ptr(), u.contiguous().data_ptr(),
                                 out.data_ptr(), s))
    return out


def closure_dataset(filt, periodic: Sequence[int], tau: float, cs: float = 0.1, stream=None):
    torch = _torch()
    _, cz, cy, cx = filt.shape
    n = cx * cy * cz
    x = torch.empty((n, 6), dtype=torch.float32, device=filt.device)
    t = torch.empty((n,), dtype=torch.float32, device=filt.device)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    s = stream if stream is not None else _stream_ptr(filt.device)
    _check(lib().lbm_closure_dataset(cx, cy, cz, per, filt.contiguous().data_ptr(), float(tau), float(cs),
                                     x.data_ptr(), t.data_ptr(), s))
    return x, t


def mlp_forward(params, x, stream=None):
    torch = _torch()
    n = x.shape[0]
    y = torch.empty((n,), dtype=torch.float32, device=x.device)
    s = stream if stream is not None else _stream_ptr(x.device)
    _check(lib().lbm_mlp_forward(params.data_ptr(), x.contiguous().data_ptr(), n, y.data_ptr(), s))
    return y


def mlp_loss_grad(params, x, t, work=None, stream=None):
    torch = _torch()
    n = x.shape[0]
    grad = torch.empty((MLP_NPARAM,), dtype=torch.float32, device=x.device)
    loss = torch.empty((1,), dtype=torch.float32, device=x.device)
    if work is None:
        work = torch.empty(max(1, int(lib().lbm_mlp_work_bytes(n))), dtype=torch.uint8, device=x.device)
    s = stream if stream is not None else _stream_ptr(x.device)
    _check(lib().lbm_mlp_loss_grad(params.data_ptr(), x.contiguous().data_ptr(), t.contiguous().data_ptr(), n,
                                   grad.data_ptr(), loss.data_ptr(), work.data_ptr(), s))
    return loss, grad


def mlp_loss_grad_noalloc(params, x, t, grad, loss, stream=None):
    """lbm_mlp_loss_grad_noalloc: loss and gradient into the caller's grad
    [1313] and loss [1] FP32 device tensors, with no workspace (the library's
    static scratch holds the partials; calls that overlap on one device race)."""
    n = x.shape[0]
    s = stream if stream is not None else _stream_ptr(x.device)
    _check(lib().lbm_mlp_loss_grad_noalloc(params.data_ptr(), x.contiguous().data_ptr(), t.contiguous().data_ptr(),
                                           n, grad.data_ptr(), loss.data_ptr(), s))


def mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    s = stream if stream is not None else _stream_ptr(params.device)
    _check(lib().lbm_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), s))


def stream_copy(src, dst, stream=None):
    nbytes = src.numel() * src.element_size()
    s = stream if stream is not None else _stream_ptr(src.device)
    _check(lib().lbm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, s))


def refine_step(coarse, fine_lo=None, fine_hi=None, n=1):
    """lbm_refine_step: advance a 2:1 refinement -- the coarse Lattice n steps
    and each fine Lattice (below / above it, None where the coarse y face is
    not an "interface" face) 2n steps, exchanging the packets that cross the
    interfaces.  The work buffer is allocated once per coarse lattice."""
    work = _refine_work(coarse)
    lo = fine_lo._h if fine_lo is not None else None
    hi = fine_hi._h if fine_hi is not None else None
    _check(lib().lbm_refine_step(coarse._h, lo, hi, work.data_ptr(), work.numel(), int(n)), coarse._h)


def _refine_work(lat):
    """The refinement work buffer of a parent Lattice (allocated once)."""
    work = getattr(lat, "_refine_work", None)
    if work is None:
        nbytes = ctypes.c_size_t(0)
        _check(lib().lbm_refine_work_bytes(ctypes.byref(lat.domain), lat.q, ctypes.byref(nbytes)))
        work = _torch().empty(nbytes.value, dtype=_torch().uint8, device=lat.device)
        lat._refine_work = work
    return work


def refine_tree_step(nodes, n=1):
    """lbm_refine_tree_step: advance a hierarchy of 2:1 levels.  nodes is a
    sequence of (Lattice, fine_lo, fine_hi) with the indices of the finer
    lattices below / above each one (None for none), nodes[0] the coarsest;
    it takes n steps and a lattice at depth d 2^d n steps.  Parents' work
    buffers are allocated once per Lattice."""
    arr = (RefineNode * len(nodes))()
    for k, (lat, lo, hi) in enumerate(nodes):
        arr[k].ctx = lat._h
        arr[k].fine_lo = -1 if lo is None else int(lo)
        arr[k].fine_hi = -1 if hi is None else int(hi)
        if lo is not None or hi is not None:
            work = _refine_work(lat)
            arr[k].work_dev = work.data_ptr()
            arr[k].work_bytes = work.numel()
    _check(lib().lbm_refine_tree_step(arr, len(nodes), int(n)), nodes[0][0]._h if nodes else None)

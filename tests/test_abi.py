"""The C-ABI library loads, exports every function declared in include/lbm.h,
and rejects invalid arguments before touching the GPU (no device calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2305_09910_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2305_09910_amd import build
        build.build()
    return lbm.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTED) == names


def test_domain_defaults(L):
    d = lbm.make_domain((8, 4, 2))
    assert list(d.bc) == [0] * 6 and list(d.rho_bc) == [1.0] * 6
    assert d.magic == 3 / 16 and d.cs_smag == 0.1 and d.storage == 0 and d.closure == 0
    assert d.collision == 0 and d.streaming == 0


def test_rows_are_padded_to_whole_lines(L):
    """Every direction segment starts on a 128-byte line: a 100-cell row
    takes 128 FP32 cells (or 128 16-bit cells)."""
    d32 = lbm.workspace_bytes(lbm.make_domain((100, 8, 4), storage="f32"), 19)
    d16 = lbm.workspace_bytes(lbm.make_domain((100, 8, 4), storage="f16"), 19)
    assert 19 * 4 * 128 * 32 <= d32 and 19 * 2 * 128 * 32 <= d16
    assert d32 - d16 == 19 * 2 * 128 * 32


def test_workspace_bytes_scales_with_storage(L):
    b32 = lbm.workspace_bytes(lbm.make_domain((64, 32, 16), storage="f32"), 19)
    b16 = lbm.workspace_bytes(lbm.make_domain((64, 32, 16), storage="f16"), 19)
    n = 64 * 32 * 16
    assert b32 >= 19 * 4 * n and b16 >= 19 * 2 * n and b32 - b16 == 19 * 2 * n
    bf = lbm.workspace_bytes(lbm.make_domain((64, 32, 16), use_flags=True), 27)
    assert bf >= 27 * 4 * n + 4 * n


@pytest.mark.parametrize("kw,q", [
    (dict(shape=(0, 4, 4)), 19),
    (dict(shape=(4, 4, 4)), 15),
    (dict(shape=(4, 4, 4), storage=7), 19),
    (dict(shape=(4, 4, 4), closure=5), 19),
])
def test_workspace_bytes_rejects(L, kw, q):
    d = lbm.make_domain(**kw)
    out = ctypes.c_size_t(0)
    assert L.lbm_workspace_bytes(ctypes.byref(d), q, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert L.lbm_last_error(None)


def test_et_workspace_holds_the_ghost_layers(L):
    """Esoteric Twist: one more cell along each non-periodic axis (the ghost
    layer beyond its + face); nothing extra for periodic axes."""
    nx, ny, nz = 64, 32, 16
    walls = ("velocity", "pressure", "noslip", "noslip", "periodic", "periodic")
    aa = lbm.workspace_bytes(lbm.make_domain((nx, ny, nz), bc=walls), 19)
    et = lbm.workspace_bytes(lbm.make_domain((nx, ny, nz), bc=walls, streaming="et"), 19)
    # rows are padded to whole 128-byte lines: 65 cells -> 96 in FP32
    extra = 19 * 4 * (96 * (ny + 1) * nz - nx * ny * nz)
    assert extra <= et - aa < extra + 256
    per = lbm.make_domain((nx, ny, nz))
    assert lbm.workspace_bytes(per, 19) == lbm.workspace_bytes(lbm.make_domain((nx, ny, nz), streaming="et"), 19)
    assert d_rejects(L, lbm.make_domain((8, 8, 8), streaming=5))


def test_sparse_workspace_is_sized_by_the_fluid_cells(L):
    """Sparse addressing: populations, fluid list and neighbour table scale
    with the fluid cells (chunks of 64), the fluid map with all cells."""
    nx, ny, nz = 64, 32, 16
    n = nx * ny * nz
    solid = np.zeros(n, np.uint8)
    solid[: 3 * n // 4] = 1  # a quarter of the cells stay fluid
    nf = n - int(solid.sum())
    dense = lbm.workspace_bytes(lbm.make_domain((nx, ny, nz), use_flags=True), 19, solid)
    sp_dom = lbm.make_domain((nx, ny, nz), use_flags=True, streaming="sparse")
    bound = lbm.workspace_bytes(sp_dom, 19)
    exact = lbm.workspace_bytes(sp_dom, 19, solid)
    # q populations + 1 fluid-list word + (q - 1) table words per fluid cell, 4 map bytes per cell
    per_fluid = 19 * 4 + 4 + 18 * 4
    assert bound - exact == pytest.approx(per_fluid * (n - nf), abs=4 * 256)
    assert exact < dense
    # without flags the sparse bound equals the flag-free count
    assert lbm.workspace_bytes(sp_dom, 19) == lbm.workspace_bytes(sp_dom, 19, np.zeros(n, np.uint8))


def d_rejects(L, d):
    out = ctypes.c_size_t(0)
    return L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_EINVAL


def test_domains_beyond_2_31_cells(L):
    """Cell indices are 64-bit: a dense context may hold more than 2^31 (and
    2^32) cells, up to what HBM holds, and its workspace is the plain count.
    Sparse addressing keeps 32-bit indices: ENOMEM from 2^32 cells or 2^31
    fluid cells.
    The launch grid spans ny and nz: each at most 65535."""
    out = ctypes.c_size_t(0)
    for shape in [(2048, 1024, 1025), (4096, 1024, 1025)]:  # 2^31 + 2^21 and 2^32 + 2^22 cells
        d = lbm.make_domain(shape)
        assert L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_OK
        n = shape[0] * shape[1] * shape[2]
        assert out.value >= 19 * 4 * n and out.value - 19 * 4 * n < 1 << 20
        d16 = lbm.make_domain(shape, storage="f16")
        assert L.lbm_workspace_bytes(ctypes.byref(d16), 19, ctypes.byref(out)) == lbm.LBM_OK
        assert out.value >= 19 * 2 * n
    d = lbm.make_domain((4096, 1024, 1025), streaming="sparse")
    assert L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_ENOMEM
    # without flags every cell is fluid: fluid indices are signed 32-bit
    d = lbm.make_domain((2048, 1024, 1025), streaming="sparse")
    assert L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_ENOMEM
    d = lbm.make_domain((2048, 1024, 1023), streaming="sparse")  # 2^31 - 2^21 cells
    assert L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_OK
    d = lbm.make_domain((8, 65536, 4))
    assert L.lbm_workspace_bytes(ctypes.byref(d), 19, ctypes.byref(out)) == lbm.LBM_EINVAL


def _create(L, d, q=19, tau=0.6, flags=None):
    F = (ctypes.c_double * 3)(0, 0, 0)
    h = ctypes.c_void_p(0)
    rc = L.lbm_create(ctypes.byref(d), q, flags, tau, F, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["tau", "pairing", "bcenum", "null_ws", "small_ws", "align", "flags", "mrt_mlp",
                                  "sparse_small_ws", "hrr_d3q27", "hrr_et", "hrr_sparse", "hrr_closure", "hrr_sigma",
                                  "hrr_small_ws", "bcenum5", "iface_x", "iface_et", "iface_sparse", "iface_hrr",
                                  "iface_solid_row"])
def test_create_rejects_before_device(L, case):
    d = lbm.make_domain((8, 8, 8))
    q = 19
    if case.startswith("hrr"):
        d.collision = lbm.COLLISION["hrr"]
        if case == "hrr_d3q27":
            q = 27
        elif case == "hrr_et":
            d.streaming = lbm.STREAMING["et"]
        elif case == "hrr_sparse":
            d.streaming = lbm.STREAMING["sparse"]
        elif case == "hrr_closure":
            d.closure = lbm.CLOSURE["smagorinsky"]
        elif case == "hrr_sigma":
            d.hrr_sigma = 1.5
    need = lbm.workspace_bytes(d, q)
    d.workspace = 0x100000
    d.workspace_bytes = need
    tau = 0.6
    flags = None
    if case == "tau":
        tau = 0.5
    elif case == "pairing":
        d.bc[2] = 1  # -y no-slip, +y periodic
    elif case == "bcenum":
        d.bc[0] = d.bc[1] = 9
    elif case == "null_ws":
        d.workspace = None
    elif case == "small_ws":
        d.workspace_bytes = need - 1
    elif case == "align":
        d.workspace = 0x100010
    elif case == "flags":
        buf = (ctypes.c_uint8 * 512)()
        flags = ctypes.cast(buf, ctypes.c_void_p)
    elif case == "mrt_mlp":
        d.collision = lbm.COLLISION["mrt"]
        d.closure = lbm.CLOSURE["mlp"]
        d.workspace_bytes = lbm.workspace_bytes(d, 19)
    elif case == "sparse_small_ws":
        # sized for half of the cells solid, created with all fluid
        d.streaming = lbm.STREAMING["sparse"]
        d.use_flags = 1
        half = np.zeros(512, np.uint8)
        half[:256] = 1
        d.workspace_bytes = lbm.workspace_bytes(d, 19, half)
        buf = (ctypes.c_uint8 * 512)()
        flags = ctypes.cast(buf, ctypes.c_void_p)
    elif case == "hrr_small_ws":
        # sized without the two velocity fields of HRR
        d.collision = lbm.COLLISION["trt"]
        d.workspace_bytes = lbm.workspace_bytes(d, 19)
        d.collision = lbm.COLLISION["hrr"]
    elif case == "bcenum5":
        d.bc[2] = d.bc[3] = 5
    elif case.startswith("iface"):
        d.bc[2], d.bc[3] = lbm.BC["interface"], lbm.BC["noslip"]
        if case == "iface_x":
            d.bc[2] = d.bc[3] = 0
            d.bc[0], d.bc[1] = lbm.BC["interface"], lbm.BC["noslip"]
        elif case == "iface_et":
            d.streaming = lbm.STREAMING["et"]
        elif case == "iface_sparse":
            d.streaming = lbm.STREAMING["sparse"]
        elif case == "iface_hrr":
            d.collision = lbm.COLLISION["hrr"]
        elif case == "iface_solid_row":
            # one solid cell in the interface row y = 0 (cells [z][y][x])
            d.use_flags = 1
            solid = np.zeros((8, 8, 8), np.uint8)
            solid[3, 0, 5] = 1
            d.workspace_bytes = lbm.workspace_bytes(d, 19, solid.reshape(-1))
            buf = (ctypes.c_uint8 * 512).from_buffer_copy(solid.tobytes())
            flags = ctypes.cast(buf, ctypes.c_void_p)
        if case != "iface_solid_row":
            d.workspace_bytes = lbm.workspace_bytes(d, q)
    rc, h = _create(L, d, q=q, tau=tau, flags=flags)
    assert rc == lbm.LBM_EINVAL and not h.value
    assert len(L.lbm_last_error(None)) > 0
    if case.startswith("iface"):
        assert b"interface" in L.lbm_last_error(None)


def test_refine_work_bytes(L):
    """One FP32 plane of q x nz x nx (the summed fine packets) per interface
    side, two sides."""
    out = ctypes.c_size_t(0)
    d = lbm.make_domain((24, 8, 10))
    for q in (19, 27):
        assert L.lbm_refine_work_bytes(ctypes.byref(d), q, ctypes.byref(out)) == lbm.LBM_OK
        assert out.value == 2 * q * 24 * 10 * 4
    assert L.lbm_refine_work_bytes(ctypes.byref(d), 15, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert L.lbm_refine_work_bytes(None, 19, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert L.lbm_refine_step(None, None, None, None, 0, 1) == lbm.LBM_EINVAL


def test_refine_tree_rejects_without_device(L):
    """A NULL node array, a count outside 1..4096 and a node without a context
    are rejected on the thread's error text before any device call."""
    assert L.lbm_refine_tree_step(None, 1, 1) == lbm.LBM_EINVAL
    nodes = (lbm.RefineNode * 2)()
    for count in (0, -1, 4097):
        assert L.lbm_refine_tree_step(nodes, count, 1) == lbm.LBM_EINVAL
    nodes[0].fine_lo = nodes[0].fine_hi = -1
    assert L.lbm_refine_tree_step(nodes, 1, 1) == lbm.LBM_EINVAL
    assert b"no context" in L.lbm_last_error(None)
    assert ctypes.sizeof(lbm.RefineNode) == 32  # pointer, two int32, pointer, size_t


def test_hrr_workspace_holds_two_velocity_fields(L):
    """HRR keeps the previous and the current velocity field (3 FP32 each per
    cell) next to the populations."""
    d = lbm.make_domain((64, 32, 16))
    trt = lbm.workspace_bytes(d, 19)
    d.collision = lbm.COLLISION["hrr"]
    assert lbm.workspace_bytes(d, 19) - trt == 2 * 12 * 64 * 32 * 16
    d2 = lbm.make_domain((8, 8, 8))
    assert d2.hrr_sigma == 0.995


def test_free_functions_reject(L):
    assert L.lbm_box_filter4(6, 8, 8, 1, 1, 1, None) == lbm.LBM_EINVAL
    assert L.lbm_stream_copy(0x1000, 0x2000, 15, None) == lbm.LBM_EINVAL
    assert L.lbm_stream_copy(0x1004, 0x2000, 16, None) == lbm.LBM_EINVAL  # misaligned source
    assert L.lbm_mlp_forward(None, None, -1, None, None) == lbm.LBM_EINVAL
    assert L.lbm_mlp_adam(0x1000, 0x1000, 0x1000, 0x1000, 0, 1e-3, 0.9, 0.999, 1e-8, None) == lbm.LBM_EINVAL
    per = (ctypes.c_int32 * 3)(1, 0, 1)
    assert L.lbm_closure_dataset(4, 4, 4, per, 0x1000, 0.5, 0.1, 0x1000, 0x1000, None) == lbm.LBM_EINVAL

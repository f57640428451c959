"""A context of more than 2^31 cells on the GPU: the D3Q19 channel 2048 x 1024
x 1025 (2^31 + 2^21 cells) in FP16 deviation storage, 82 GB of populations.
The flow is invariant along x and z (no-slip walls on y, body force along x,
start at rest), so after 20 steps the y profile of the populations must be the
same, bit for bit, at the first cells and at cells whose index is beyond 2^31,
and the same as on a 128 x 1024 x 4 lattice running the same kernels (the
paired even step and the one-cell odd step of unmasked FP16 rows).  A cell
index that wrapped at 32 bits would read or write another row."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (2048, 1024, 1025)
NEED_BYTES = 160 * 2 ** 30  # populations, the FP64 start fields, headroom


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


def _lattice(shape):
    from paper_2305_09910_amd import lbm
    bc = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")
    return lbm.Lattice(shape, q=19, tau=0.6, force=(1e-6, 0.0, 0.0), bc=bc, storage="f16")


def _profile_cells(shape, x, z):
    nx, ny, _ = shape
    return np.array([(z * ny + y) * nx + x for y in range(ny)], dtype=np.int64)


def test_context_beyond_2_31_cells():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # blocks other tests' tensors left in torch's cache
    free, _ = torch.cuda.mem_get_info()
    if free < NEED_BYTES:
        pytest.skip(f"needs {NEED_BYTES >> 30} GiB of free device memory, {free >> 30} GiB free")
    nx, ny, nz = SHAPE
    n = nx * ny * nz
    assert n > 2 ** 31
    print(f"[case] {SHAPE} FP16, {n} cells", flush=True)
    big = _lattice(SHAPE)
    rho = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    big.init_equilibrium(rho, u)
    torch.cuda.synchronize()
    del rho, u
    torch.cuda.empty_cache()
    big.step(20)
    near = big.gather(_profile_cells(SHAPE, 3, 0)).cpu()
    far_cells = _profile_cells(SHAPE, nx - 1, nz - 1)
    assert int(far_cells.min()) > 2 ** 31
    far = big.gather(far_cells).cpu()
    mass, _ = big.totals()
    del big
    torch.cuda.empty_cache()

    small_shape = (128, ny, 4)
    small = _lattice(small_shape)
    small.init_equilibrium(np.ones((4, ny, 128)), np.zeros((3, 4, ny, 128)))
    small.step(20)
    ref = small.gather(_profile_cells(small_shape, 5, 2)).cpu()

    print(f"mass {mass:.6f} of {n}; far vs near identical {torch.equal(far, near)}; "
          f"vs small lattice identical {torch.equal(far, ref)}")
    assert torch.equal(near, far)
    assert torch.equal(far, ref)
    assert not torch.equal(far[0], far[ny // 2])  # the profile is not flat
    assert abs(mass / n - 1.0) < 1e-6

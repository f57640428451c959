"""Seeded synthetic inputs: macroscopic initial fields and solid masks.

This module holds no lattice Boltzmann arithmetic: it produces density and
velocity fields (FP64, [nz, ny, nx] and [3, nz, ny, nx], x fastest) and solid
masks from closed-form flow fields and a seeded PCG64 generator.  Both the
oracle and the GPU path build their own initial populations from these
fields.

Workloads (the paper's own channel and landing-gear geometries are not
available, so these stand in for them with the stated shapes):
  * Taylor-Green vortex: the 2-D mode in x-y, uniform in z.
  * Channel: walls on the y faces (halfway between the first/last row and the
    face), laminar parabola plus uniform noise, periodic in x and z -- the
    shape of the paper's turbulent-channel benchmark.
  * Obstacles: random non-overlapping solid spheres filling a volume
    fraction -- a stand-in for the landing-gear geometry.
  * Vortical perturbation: a band-limited divergence-free random field, the
    start of the closure-training runs (energy at the filter scale).
"""
from __future__ import annotations

import math

import numpy as np


def taylor_green(nx: int, ny: int, nz: int, u0: float = 0.05):
    """2-D Taylor-Green vortex, k = 2 pi / nx along x and 2 pi / ny along y.

    u = u0 cos(kx x) sin(ky y), v = -u0 sin(kx x) cos(ky y), w = 0, and the
    matching pressure field expressed as density with c_s^2 = 1/3:
    rho = 1 - (3 u0^2 / 4) (cos 2 kx x + cos 2 ky y).
    """
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    shape = (nz, ny, nx)
    u = np.zeros((3,) + shape)
    u[0] = np.broadcast_to(u0 * np.cos(kx * x) * np.sin(ky * y), shape)
    u[1] = np.broadcast_to(-u0 * np.sin(kx * x) * np.cos(ky * y), shape)
    rho = np.broadcast_to(1.0 - 0.75 * u0 * u0 * (np.cos(2 * kx * x) + np.cos(2 * ky * y)), shape).copy()
    return rho, u


def channel(nx: int, ny: int, nz: int, u_c: float = 0.05, noise: float = 0.05, seed: int = 1234):
    """Channel with walls half a cell outside rows 0 and ny-1.

    u_x = 4 u_c (y + 1/2)(ny - 1/2 - y) / ny^2 plus i.i.d. uniform noise in
    [-noise u_c, noise u_c] on every component of every cell, drawn from
    numpy's PCG64(seed) in C order (z, y, x, component); rho = 1.
    """
    y = np.arange(ny, dtype=np.float64)
    prof = 4.0 * u_c * (y + 0.5) * (ny - 0.5 - y) / (ny * ny)
    shape = (nz, ny, nx)
    u = np.zeros((3,) + shape)
    u[0] = prof[None, :, None]
    if noise > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        amp = noise * u_c
        n = rng.uniform(-amp, amp, size=shape + (3,))
        u += np.moveaxis(n, -1, 0)
    rho = np.ones(shape)
    return rho, u


def spheres(nx: int, ny: int, nz: int, fill: float = 0.10, rmin: float = 6.0, rmax: float = 20.0,
            x_margin: int = 32, seed: int = 2024, max_tries: int = 200000):
    """Random non-overlapping solid spheres; returns (mask uint8 [nz,ny,nx], list of (xc,yc,zc,r)).

    Radii are uniform reals in [rmin, rmax]; centres are uniform with
    x in [x_margin + r, nx - 1 - x_margin - r] and y, z in [r, n - 1 - r]
    (no periodic wrap).  A candidate is accepted when its centre lies at
    least r1 + r2 + 1 from every accepted centre.  Spheres are added until
    the solid voxel fraction reaches `fill`.  A cell (i, j, k) is solid iff
    (i - xc)^2 + (j - yc)^2 + (k - zc)^2 <= r^2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    acc = []
    total = nx * ny * nz
    solid = 0
    tries = 0
    while solid < fill * total:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("spheres: could not reach the requested fill fraction")
        r = rng.uniform(rmin, rmax)
        lo_x, hi_x = x_margin + r, nx - 1 - x_margin - r
        if hi_x < lo_x or ny - 1 - r < r or nz - 1 - r < r:
            raise ValueError("spheres: domain too small for the radius range")
        xc = rng.uniform(lo_x, hi_x)
        yc = rng.uniform(r, ny - 1 - r)
        zc = rng.uniform(r, nz - 1 - r)
        if any((xc - a) ** 2 + (yc - b) ** 2 + (zc - c) ** 2 < (r + s + 1.0) ** 2 for a, b, c, s in acc):
            continue
        acc.append((xc, yc, zc, r))
        x0, x1 = max(0, int(math.floor(xc - r))), min(nx - 1, int(math.ceil(xc + r)))
        y0, y1 = max(0, int(math.floor(yc - r))), min(ny - 1, int(math.ceil(yc + r)))
        z0, z1 = max(0, int(math.floor(zc - r))), min(nz - 1, int(math.ceil(zc + r)))
        zz, yy, xx = np.meshgrid(np.arange(z0, z1 + 1), np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        inside = (xx - xc) ** 2 + (yy - yc) ** 2 + (zz - zc) ** 2 <= r * r
        sub = mask[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
        solid += int(np.count_nonzero(inside & (sub == 0)))
        sub[inside] = 1
    return mask, acc


def porous(nx: int, ny: int, nz: int, solid_fraction: float = 0.7, rmin: float = 3.0, rmax: float = 8.0,
           seed: int = 77):
    """Periodic porous medium of random overlapping solid spheres; returns a
    uint8 mask [nz, ny, nx].

    Radii are uniform reals in [rmin, rmax] and centres uniform reals in the
    box; a cell (i, j, k) is solid iff its periodic distance to some centre
    is <= r.  Spheres are added until the solid voxel fraction reaches
    `solid_fraction`, so the medium wraps around every face.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    total = nx * ny * nz
    solid = 0
    while solid < solid_fraction * total:
        r = rng.uniform(rmin, rmax)
        xc, yc, zc = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        R = int(math.ceil(r))
        ix = np.arange(int(math.floor(xc)) - R, int(math.floor(xc)) + R + 2)
        iy = np.arange(int(math.floor(yc)) - R, int(math.floor(yc)) + R + 2)
        iz = np.arange(int(math.floor(zc)) - R, int(math.floor(zc)) + R + 2)
        inside = ((iz[:, None, None] - zc) ** 2 + (iy[None, :, None] - yc) ** 2 + (ix[None, None, :] - xc) ** 2
                  <= r * r)
        kz, ky, kx = np.nonzero(inside)
        cells = np.unique(((iz[kz] % nz) * ny + iy[ky] % ny) * nx + ix[kx] % nx)  # wrapped, each once
        flat = mask.reshape(-1)
        solid += int(np.count_nonzero(flat[cells] == 0))
        flat[cells] = 1
    return mask


def channel_level(nx: int, ny: int, nz: int, y0: float, h: float, height: float, u_c: float = 0.05,
                  noise: float = 0.05, seed: int = 1234):
    """One level of a channel split into refinement levels along y: cells of
    size h (in units of the coarsest cell) whose first row starts at y0, in a
    channel of total height `height` with walls at 0 and `height`.

    u_x = 4 u_c y (height - y) / height^2 at the cell centres y = y0 + (j + 1/2) h,
    plus i.i.d. uniform noise in [-noise u_c, noise u_c] on every component
    (numpy's PCG64(seed), C order (z, y, x, component)); rho = 1."""
    y = y0 + (np.arange(ny, dtype=np.float64) + 0.5) * h
    prof = 4.0 * u_c * y * (height - y) / (height * height)
    shape = (nz, ny, nx)
    u = np.zeros((3,) + shape)
    u[0] = prof[None, :, None]
    if noise > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        u += np.moveaxis(rng.uniform(-noise * u_c, noise * u_c, size=shape + (3,)), -1, 0)
    return np.ones(shape), u


def uniform_flow(nx: int, ny: int, nz: int, u=(0.04, 0.0, 0.0), rho: float = 1.0):
    shape = (nz, ny, nx)
    uu = np.zeros((3,) + shape)
    for a in range(3):
        uu[a] = u[a]
    return np.full(shape, float(rho)), uu


def perturbation(shape, scale: float, seed: int):
    """Seeded i.i.d. uniform numbers in [-scale, scale] of the given shape."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=shape)


def vortical(nx: int, ny: int, nz: int, rms: float, wavelength: float, seed: int = 7, kmax_factor: float = 3.0,
             device=None):
    """Seeded band-limited solenoidal velocity field, periodic on the box.

    Fourier modes with |k| <= kmax_factor * k_p (k_p = 2 pi / wavelength)
    get complex Gaussian amplitudes from numpy's PCG64(seed), drawn in a
    fixed order over the mode cube, shaped to the energy spectrum
    E(k) ~ k^4 exp(-2 (k/k_p)^2) and projected onto the plane normal to k
    (divergence free); the field is the real inverse transform scaled to the
    given rms velocity.  Returns float64 numpy [3, nz, ny, nx], or a float32
    torch tensor on `device` (the inverse transform then runs there).
    """
    kp = 2 * math.pi / wavelength
    kmax = kmax_factor * kp
    mx = min(nx // 2, int(math.ceil(kmax * nx / (2 * math.pi))))
    my = min(ny // 2, int(math.ceil(kmax * ny / (2 * math.pi))))
    mz = min(nz // 2, int(math.ceil(kmax * nz / (2 * math.pi))))
    ix = np.arange(0, mx + 1)                    # half spectrum along x
    iy = np.r_[np.arange(0, my + 1), np.arange(-my, 0)]
    iz = np.r_[np.arange(0, mz + 1), np.arange(-mz, 0)]
    KZ, KY, KX = np.meshgrid(2 * math.pi * iz / nz, 2 * math.pi * iy / ny, 2 * math.pi * ix / nx, indexing="ij")
    k = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.normal(size=(3,) + k.shape) + 1j * rng.normal(size=(3,) + k.shape)
    kk = np.where(k > 0, k, 1.0)
    kd = (a[0] * KX + a[1] * KY + a[2] * KZ) / kk ** 2
    a = a - np.stack([KX, KY, KZ]) * kd  # solenoidal projection
    amp = np.where((k > 0) & (k <= kmax), (k / kp) * np.exp(-(k / kp) ** 2), 0.0)  # |u_hat| ~ sqrt(E/k^2)
    a = a * amp
    zsel = np.r_[np.arange(0, mz + 1), np.arange(nz - mz, nz)]
    ysel = np.r_[np.arange(0, my + 1), np.arange(ny - my, ny)]
    if device is None:
        full = np.zeros((3, nz, ny, nx // 2 + 1), dtype=np.complex128)
        full[:, zsel[:, None, None], ysel[None, :, None], ix[None, None, :]] = a
        u = np.fft.irfftn(full, s=(nz, ny, nx), axes=(1, 2, 3))
        u *= rms / math.sqrt(np.mean(np.sum(u * u, axis=0)))
        return u
    import torch
    spec = torch.zeros((3, nz, ny, nx // 2 + 1), dtype=torch.complex64, device=device)
    zs = torch.as_tensor(zsel, device=device)
    ys = torch.as_tensor(ysel, device=device)
    xs = torch.as_tensor(ix, device=device)
    spec[:, zs[:, None, None], ys[None, :, None], xs[None, None, :]] = torch.as_tensor(a.astype(np.complex64),
                                                                                    device=device)
    u = torch.fft.irfftn(spec, s=(nz, ny, nx), dim=(1, 2, 3))
    del spec
    u *= rms / torch.sqrt(torch.mean(torch.sum(u * u, dim=0)))
    return u

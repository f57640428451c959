"""Write closure_net_oracle_trained.npz: a learned-closure network trained by
the FP64 oracle alone, and the coarse start state it is tested on.

Recipe (the learned LES closure of the turbulent channel, Section 5.1: a
per-cell relaxation-time correction for the subgrid stresses):
  * fine channel 128x64x64, D3Q19 TRT, walls on the y faces, periodic x and z,
    tau_f = 0.512 (acoustic scaling of the coarse tau_c = 0.503 by 4), force
    F_c / 4 with F_c = 1.236e-7; start: laminar parabola (centre-line 0.05)
    plus 5% uniform noise (seed 1234) plus a band-limited solenoidal field of
    rms 0.02 and peak wavelength 16 fine cells (seed 1235), damped to zero at
    the walls;
  * 200 spin-up steps, then 4 snapshots 100 steps apart: density and
    velocity -> 4^3 box filter -> six flux invariants and the target
    correction (oracle dataset builder);
  * standardisation from the data, trusted range = data range widened by a
    quarter of its width (and a relative 1e-6), seeded small weights, then 600 Adam steps (lr 2e-3)
    on minibatches of 2048 samples with the oracle's FP64 loss gradient;
  * the filtered fine state 100 steps after the last snapshot is stored as
    the coarse start state (rho, u on 32x16x16).

Only oracle/ and the seeded input generators run here; nothing comes from the
GPU path.  Run from the repository root:  python tests/golden/make_closure_net.py
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2305_09910_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closure_net_oracle_trained.npz")
FINE = (128, 64, 64)
TAU_C, FACTOR, CS = 0.503, 4, 0.1
F_C = 1.236e-7


def fine_start():
    nx, ny, nz = FINE
    rho, u = inputs.channel(nx, ny, nz, 0.05, 0.05, seed=1234)
    up = inputs.vortical(nx, ny, nz, 0.02, 16.0, seed=1235)
    y = np.arange(ny, dtype=np.float64)
    damp = (4.0 * (y + 0.5) * (ny - 0.5 - y) / (ny * ny))[None, None, :, None]
    return rho, u + up * damp


def main():
    tau_f = 0.5 + FACTOR * (TAU_C - 0.5)
    sim = oracle.Sim(19, FINE, bc=(0, 0, 1, 1, 0, 0), tau=tau_f, force=(F_C / FACTOR, 0, 0))
    rho, u = fine_start()
    sim.init_equilibrium(rho, u)
    sim.step(200)
    xs, ts = [], []
    for k in range(4):
        r, v = sim.moments()
        x, t = oracle.closure_dataset(oracle.box_filter4(r, v), (1, 0, 1), TAU_C, CS)
        xs.append(x)
        ts.append(t)
        print(f"snapshot {k}: mean target {t.mean():.3e}, nonzero {np.mean(t > 0):.2f}", flush=True)
        sim.step(100)
    r, v = sim.moments()
    filt = oracle.box_filter4(r, v)
    x, t = np.concatenate(xs), np.concatenate(ts)

    mu, sg = x.mean(0), x.std(0)
    # a feature whose spread is below a relative 1e-6 of its size is constant
    # (tau; its std is then only the roundoff of the mean): unit scale
    const = sg <= 1e-6 * np.abs(mu)
    sg = np.where(const, np.maximum(np.abs(mu), 1.0), sg)
    lo, hi = x.min(0), x.max(0)
    # widened by a quarter of the width, and by a relative 1e-6 so that a
    # constant feature (tau) keeps a range wider than its float32 rounding
    w = hi - lo
    pad = 0.25 * w + 1e-6 * np.maximum(np.abs(lo), np.abs(hi)) + 1e-30
    lo, hi = lo - pad, hi + pad
    rng = np.random.default_rng(0)
    b3 = math.log(math.expm1(max(float(t.mean()), 1e-6)))
    p = np.concatenate([rng.normal(0, 1 / math.sqrt(6), 192), np.zeros(32), rng.normal(0, 1 / math.sqrt(32), 1024),
                        np.zeros(32), rng.normal(0, 0.1 / math.sqrt(32), 32), [b3]])
    norm = np.concatenate([mu, sg, lo, hi])
    m, vv = np.zeros(1313), np.zeros(1313)
    for step in range(1, 601):
        idx = rng.integers(0, x.shape[0], 2048)
        loss, g = oracle.mlp_loss_grad(p, norm, x[idx], t[idx])
        oracle.adam(p, g, m, vv, step, 2e-3)
        if step % 100 == 0 or step == 1:
            print(f"train step {step}: loss {loss:.3e}", flush=True)
    y = oracle.mlp_forward(p, norm, x)
    print(f"mse: network {np.mean((y - t) ** 2):.3e}, smagorinsky {np.mean((x[:, 4] - t) ** 2):.3e}, "
          f"zero {np.mean(t ** 2):.3e}")
    np.savez(OUT, params=p.astype(np.float32), norm=norm.astype(np.float32), tau_c=TAU_C, force_c=F_C,
             rho=filt[0], u=filt[1:4])
    print("wrote", OUT)


if __name__ == "__main__":
    main()

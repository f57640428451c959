"""Learned LES closure: data generation, training and evaluation driver.

Workflow (every numerical step runs in the library's HIP kernels; torch
only holds device memory and selects minibatches):

1. A fine channel run (factor x finer in every direction, acoustic scaling:
   same lattice velocity, nu_fine = factor * nu_coarse, F_fine = F / factor)
   is spun up, then snapshots are taken.
2. Each snapshot: density and velocity (lbm_moments) -> 4^3 box filter
   (lbm_box_filter4) -> per coarse cell the target relaxation-time
   correction (lbm_closure_dataset), and the six flux invariants either of
   the filtered strain (lbm_closure_dataset, the default) or of a coarse
   lattice run up to the snapshot from an earlier filtered state
   (lbm_closure_features: the inputs the network meets inside the lattice).
3. The MLP 6 -> 32 -> 32 -> 1 is trained with the library's forward /
   backward (bfloat16 matrix cores) and Adam kernels.
4. Evaluation a priori (mean-squared error of the predicted correction on a
   held-out snapshot, against the Smagorinsky correction tau_smag - tau and
   against zero) and a posteriori (coarse runs started from the filtered
   fine state with no closure, Smagorinsky, and the MLP, compared with the
   filtered fine run after the same physical time).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import inputs, lbm

WALLS_Y = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")


@dataclass
class ClosureConfig:
    coarse: tuple = (64, 32, 32)     # coarse lattice (nx, ny, nz)
    factor: int = 4                  # fine / coarse resolution (the box filter is 4^3)
    tau_c: float = 0.503             # coarse molecular tau
    u_c: float = 0.05                # centre-line velocity of the start profile
    re_tau: float = 180.0            # friction Reynolds number setting the driving force
    noise: float = 0.05              # uniform velocity noise, fraction of u_c
    vortical_rms: float = 0.0        # rms of a band-limited solenoidal perturbation (0: none)
    vortical_wavelength: float = 32.0  # its peak wavelength in fine cells
    seed: int = 1234
    cs: float = 0.1                  # Smagorinsky constant (fallback and comparison)
    spinup: int = 2000               # fine steps before the first snapshot
    snapshots: int = 4               # training snapshots (+1 held out)
    every: int = 400                 # fine steps between snapshots
    train_steps: int = 400
    batch: int = 65536
    lr: float = 2e-3
    eval_coarse_steps: int = 200     # a-posteriori horizon in coarse steps
    features: str = "filtered"       # "lattice": inputs from a coarse lattice's own populations; "filtered":
                                     # inputs from the filtered strain (P = -(2/3)(tau + dtau*) S)
    lead: int = 25                   # "lattice": coarse steps from the earlier filtered state to the snapshot
    target_scale: float = 1.0        # training targets alpha * dtau* (a-posteriori calibration of the dissipation)
    extra: dict = field(default_factory=dict)

    @property
    def fine(self):
        return tuple(self.factor * n for n in self.coarse)

    @property
    def nu_c(self):
        return (self.tau_c - 0.5) / 3.0

    @property
    def force_c(self):
        # F = u_tau^2 / delta with u_tau = re_tau nu / delta, delta = half height
        delta = self.coarse[1] / 2.0
        u_tau = self.re_tau * self.nu_c / delta
        return u_tau * u_tau / delta


def _torch():
    import torch
    return torch


def fine_lattice(cfg: ClosureConfig):
    f = cfg.factor
    tau_f = 0.5 + f * (cfg.tau_c - 0.5)
    lat = lbm.Lattice(cfg.fine, q=19, tau=tau_f, force=(cfg.force_c / f, 0.0, 0.0), bc=WALLS_Y)
    rho, u = inputs.channel(*cfg.fine, u_c=cfg.u_c, noise=cfg.noise, seed=cfg.seed)
    if cfg.vortical_rms > 0:
        torch = _torch()
        nx, ny, nz = cfg.fine
        up = inputs.vortical(nx, ny, nz, cfg.vortical_rms, cfg.vortical_wavelength, seed=cfg.seed + 1,
                             device=lat.device)
        # vanish at the walls (half a cell outside rows 0 and ny - 1)
        y = torch.arange(ny, device=lat.device, dtype=torch.float32)
        damp = (4.0 * (y + 0.5) * (ny - 0.5 - y) / (ny * ny)).view(1, 1, ny, 1)
        u = torch.as_tensor(u, device=lat.device, dtype=torch.float64) + (up * damp).double()
        del up
    lat.init_equilibrium(rho, u)
    return lat


def filtered(lat):
    rho, u = lat.moments()
    return lbm.box_filter4(rho, u)


def dataset(cfg: ClosureConfig, filt):
    return lbm.closure_dataset(filt, (1, 0, 1), cfg.tau_c, cfg.cs)


def coarse_features(cfg: ClosureConfig, filt, steps):
    """The closure inputs a coarse lattice produces from its own populations
    (lbm_closure_features), `steps` coarse steps after starting from the
    filtered state `filt` with the Smagorinsky closure: the inputs the
    network meets when it runs inside the lattice, whose non-equilibrium
    flux carries the lattice's own acoustic and truncation parts that the
    filtered strain lacks."""
    c = lbm.Lattice(cfg.coarse, q=19, tau=cfg.tau_c, force=(cfg.force_c, 0, 0), bc=WALLS_Y, closure="smagorinsky",
                    cs=cfg.cs)
    c.init_equilibrium(filt[0].double(), filt[1:4].double())
    c.step(steps)
    x = c.closure_features()
    c.close()
    return x


def generate(cfg: ClosureConfig, log=print):
    """Fine run -> (training features, targets), held-out (x, t), and the
    filtered field and fine lattice at the held-out time (for a-posteriori).

    Targets come from the filtered fine field at each snapshot.  Features:
    with cfg.features == "filtered", from the same filtered field
    (lbm_closure_dataset); with "lattice", from a coarse lattice run
    cfg.lead coarse steps from the filtered state cfg.lead coarse steps
    earlier, so that it reaches the snapshot's time (coarse_features)."""
    torch = _torch()
    if cfg.features not in ("lattice", "filtered"):
        raise ValueError(f"unknown feature source {cfg.features!r}")
    lead = cfg.lead * cfg.factor if cfg.features == "lattice" else 0
    if lead > cfg.spinup or lead > cfg.every:
        raise ValueError("the lead of the lattice features must fit in the spin-up and the snapshot spacing")
    lat = fine_lattice(cfg)
    lat.step(cfg.spinup - lead)
    xs, ts = [], []
    for k in range(cfg.snapshots + 1):
        early = filtered(lat) if lead else None
        lat.step(lead)
        filt = filtered(lat)
        x, t = dataset(cfg, filt)
        if lead:
            x = coarse_features(cfg, early, cfg.lead)
        if k == cfg.snapshots:
            return torch.cat(xs), torch.cat(ts), x, t, filt, lat
        xs.append(x)
        ts.append(cfg.target_scale * t)
        log(f"[closure] snapshot {k}: mean target {float(t.mean()):.3e}, nonzero {float((t > 0).float().mean()):.2f}")
        lat.step(cfg.every - lead)


def init_params(x, t, seed=0, margin=0.25):
    """Standardisation from the data, trusted range = data range widened by
    `margin` of its width, small random weights, output bias at the mean target."""
    torch = _torch()
    xn = x.double().cpu().numpy()
    mu = xn.mean(0)
    sg = xn.std(0)
    # a feature whose spread is below a relative 1e-6 of its size is constant
    # (tau): its std is only the roundoff of the mean, so give it unit scale
    const = sg <= 1e-6 * np.abs(mu)
    sg = np.where(const, np.maximum(np.abs(mu), 1.0), sg)
    lo, hi = xn.min(0), xn.max(0)
    # widen by `margin` of the width and by a relative 1e-6, so that a
    # constant feature keeps a range wider than its float32 rounding
    w = hi - lo
    pad = margin * w + 1e-6 * np.maximum(np.abs(lo), np.abs(hi)) + 1e-30
    lo, hi = lo - pad, hi + pad
    rng = np.random.default_rng(seed)
    tm = max(float(t.mean()), 1e-6)
    b3 = math.log(math.expm1(tm))
    p = np.concatenate([rng.normal(0, 1 / math.sqrt(6), 192), np.zeros(32), rng.normal(0, 1 / math.sqrt(32), 1024),
                        np.zeros(32), rng.normal(0, 0.1 / math.sqrt(32), 32), [b3]])
    return np.concatenate([p, mu, sg, lo, hi]).astype(np.float32)


def train(cfg: ClosureConfig, x, t, params0=None, log=print):
    torch = _torch()
    P = torch.tensor(init_params(x, t) if params0 is None else params0, device=x.device)
    m = torch.zeros(lbm.MLP_NPARAM, device=x.device)
    v = torch.zeros(lbm.MLP_NPARAM, device=x.device)
    g = torch.Generator(device=x.device)
    g.manual_seed(cfg.seed)
    n = x.shape[0]
    hist = []
    for step in range(1, cfg.train_steps + 1):
        if n > cfg.batch:
            idx = torch.randint(0, n, (cfg.batch,), device=x.device, generator=g)
            xb, tb = x[idx], t[idx]
        else:
            xb, tb = x, t
        loss, grad = lbm.mlp_loss_grad(P, xb, tb)
        lbm.mlp_adam(P, grad, m, v, step, cfg.lr)
        if step == 1 or step % max(1, cfg.train_steps // 10) == 0:
            hist.append((step, float(loss)))
            log(f"[closure] train step {step}: loss {float(loss):.3e}")
    return P, hist


def a_priori(P, x, t):
    """Mean-squared error of the predicted correction against the target, for
    the MLP, for the Smagorinsky correction (feature 5) and for zero."""
    y = lbm.mlp_forward(P, x)
    return {"mse_mlp": float(((y - t) ** 2).mean()), "mse_smagorinsky": float(((x[:, 4] - t) ** 2).mean()),
            "mse_zero": float((t ** 2).mean()), "target_mean": float(t.mean())}


def a_posteriori(cfg: ClosureConfig, P, filt, fine, log=print):
    """Coarse runs from the filtered fine state versus the filtered fine run."""
    torch = _torch()
    f = cfg.factor
    rho0 = filt[0].double()
    u0 = filt[1:4].double()
    fine.step(f * cfg.eval_coarse_steps)
    ref = filtered(fine)[1:4]
    out = {}
    for name in ("none", "smagorinsky", "mlp"):
        c = lbm.Lattice(cfg.coarse, q=19, tau=cfg.tau_c, force=(cfg.force_c, 0, 0), bc=WALLS_Y, closure=name,
                        cs=cfg.cs)
        if name == "mlp":
            c.set_closure_weights(P.cpu().numpy())
        c.init_equilibrium(rho0, u0)
        c.step(cfg.eval_coarse_steps)
        rc, _, _ = c.totals(check=False)
        _, u = c.moments()
        err = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))
        fb = c.closure_fallbacks() if name == "mlp" else 0
        out[name] = {"l2_velocity_error": err if rc == 0 else float("nan"), "finite": rc == 0,
                     "fallback_fraction": fb / (cfg.eval_coarse_steps * c.n) if name == "mlp" else None}
        log(f"[closure] a posteriori {name}: L2 {out[name]['l2_velocity_error']:.4e}")
    return out


def study(cfg: ClosureConfig, log=print):
    x, t, xh, th, filt, fine = generate(cfg, log)
    P, hist = train(cfg, x, t, log=log)
    res = {"a_priori_train": a_priori(P, x, t), "a_priori_heldout": a_priori(P, xh, th), "loss_history": hist}
    res["a_posteriori"] = a_posteriori(cfg, P, filt, fine, log)
    return res, P


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="learned LES closure study (fine run -> filter -> train -> compare)")
    ap.add_argument("--coarse", type=int, nargs=3, default=[256, 128, 128])
    ap.add_argument("--tau-c", type=float, default=0.503)
    ap.add_argument("--noise", type=float, default=0.3)
    ap.add_argument("--vortical-rms", type=float, default=0.0)
    ap.add_argument("--vortical-wavelength", type=float, default=32.0)
    ap.add_argument("--spinup", type=int, default=1000)
    ap.add_argument("--snapshots", type=int, default=4)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-coarse-steps", type=int, default=500)
    ap.add_argument("--seed", type=int, default=1234, help="seed of the start state and of minibatch sampling")
    ap.add_argument("--features", choices=["lattice", "filtered"], default="filtered",
                    help="training inputs from a coarse lattice's populations or from the filtered strain")
    ap.add_argument("--lead", type=int, default=25, help="coarse steps of the lattice run behind each snapshot")
    ap.add_argument("--target-scale", type=float, default=1.0,
                    help="train on target_scale * dtau* (a-posteriori calibration of the dissipation)")
    ap.add_argument("--out", default=None, help="write the JSON result here")
    a = ap.parse_args(argv)
    cfg = ClosureConfig(coarse=tuple(a.coarse), tau_c=a.tau_c, noise=a.noise, vortical_rms=a.vortical_rms,
                        vortical_wavelength=a.vortical_wavelength, spinup=a.spinup,
                        snapshots=a.snapshots, every=a.every, train_steps=a.train_steps, batch=a.batch, lr=a.lr,
                        eval_coarse_steps=a.eval_coarse_steps, seed=a.seed, features=a.features, lead=a.lead,
                        target_scale=a.target_scale)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    log(f"[closure] fine {cfg.fine}, coarse {cfg.coarse}, tau_c {cfg.tau_c}, F_c {cfg.force_c:.3e}")
    res, P = study(cfg, log)
    res["config"] = {k: getattr(cfg, k) for k in ("coarse", "factor", "tau_c", "u_c", "re_tau", "noise",
                                                   "vortical_rms", "vortical_wavelength", "seed", "cs",
                                                   "spinup", "snapshots", "every", "train_steps", "batch", "lr",
                                                   "eval_coarse_steps", "features", "lead", "target_scale")}
    res["config"]["fine"] = cfg.fine
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
        np.save(a.out.replace(".json", "_weights.npy"), P.cpu().numpy())


if __name__ == "__main__":
    main()

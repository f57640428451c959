#!/usr/bin/env python3
"""Benchmark of the fused stream-collide hot path on one MI355X.

Headline workload: obstacle flow, D3Q27 TRT, 384x384x384 cells, velocity
inflow u = (0.04, 0, 0) at -x, pressure outflow rho = 1 at +x, periodic y and
z faces, seeded random non-overlapping solid spheres (radius 6-20) filling
10% of the volume as bounce-back cells, FP32 storage: the largest workload
of the set that fits one GPU (6.1 GB of populations, far beyond the 256 MB
last-level cache).  One step is one fused stream-collide kernel over every
cell; the FP64 mass/momentum diagnostics run every 1000 steps inside the
timed region.  The metric is MLUPS (million lattice-cell updates per second)
and the fraction of the HBM roofline P_max = b_s / n_b of the paper (LAGOON
scalability section, Eq. (3)), with n_b = 2 q s bytes per cell update (each
population read once and written once, s bytes per population) plus one
byte of solid flag.

The JSON line on stdout also carries the other storage forms and
workloads (FP16/BF16 deviation storage, the channels, closures, MRT, the
Esoteric Twist and sparse addressing) as `forms`, the measured device copy
bandwidth, the paper's own CPU figures as context, and the FP64 oracle timed
on the host cores (`cpu_baseline`).  The same oracle runs, on stated smaller
copies of each workload, give the velocity L2 error of every form against
FP64 (`velocity_l2_vs_oracle`).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WALLS_Y = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")
INOUT_X = ("velocity", "pressure", "periodic", "periodic", "periodic", "periodic")
BYTES = {"f32": 4, "f16": 2, "bf16": 2}


def bytes_per_cell(q, value_bytes, mask=False, hrr=False):
    """Algorithmic HBM bytes of one cell update (the paper's n_b, Section 5.2):
    each of the q populations is read once and written once, plus the solid
    flag of the cell when the domain has one; the HRR collision also reads the
    previous step's velocity (3 FP32) and writes its own."""
    return 2 * q * value_bytes + (1 if mask else 0) + (24 if hrr else 0)


def sparse_bytes_per_fluid_cell(q, value_bytes, table_every_step=False):
    """Algorithmic HBM bytes of one fluid-cell update with sparse addressing:
    every population read once and written once, plus the q - 1 four-byte
    neighbour-table entries, read on odd steps (half the updates), or on
    every step when the domain has velocity or pressure faces."""
    return 2 * q * value_bytes + (4 if table_every_step else 2) * (q - 1)


def roofline_mlups(bandwidth_bytes_per_s, nb):
    """Bandwidth bound P_max = b_s / n_b in lattice updates per second, as MLUPS."""
    return bandwidth_bytes_per_s / nb / 1e6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def channel_cfg(nx, ny, nz, storage="f32", closure="none", collision="trt"):
    F = 8 * (1 / 300) * 0.05 / ny ** 2  # centre-line u ~ 0.05 at tau = 0.51
    return dict(name=f"channel_{nx}x{ny}x{nz}", shape=(nx, ny, nz), q=19, tau=0.51, force=(F, 0, 0), bc=WALLS_Y,
                storage=storage, closure=closure, solid=None, u_bc=None, collision=collision, hrr_sigma=0.995)


def obstacle_cfg(n=384, collision="trt"):
    """D3Q27 obstacle flow on n^3 cells: velocity inflow 0.04 at -x, pressure
    outflow at +x, periodic y and z, random spheres (radius 6-20) filling 10%,
    seed 2024, sphere centres 32 cells from the x faces at n = 384 (scaled
    with n for smaller copies: 11 cells at n = 128)."""
    from paper_2305_09910_amd import inputs
    solid, _ = inputs.spheres(n, n, n, fill=0.10, x_margin=round(32 * n / 384), seed=2024)
    uw = np.zeros((6, 3))
    uw[0] = (0.04, 0, 0)
    # ghost rates >= 1.5 keep the D3Q27 tensor-product MRT stable at low viscosity
    return dict(name=f"obstacles_{n}^3_d3q27", shape=(n, n, n), q=27, tau=0.56, force=(0, 0, 0), bc=INOUT_X,
                storage="f32", closure="none", solid=solid, u_bc=uw, collision=collision,
                mrt_rates=(1.6, 1.75, 1.55, 1.65, 1.7))


def porous_cfg(n=256, storage="f32", streaming="aa"):
    """Force-driven flow through a periodic porous medium, 70% solid (random
    overlapping spheres of radius 3-8), D3Q19 TRT: the solid-heavy case
    sparse addressing is for."""
    from paper_2305_09910_amd import inputs
    solid = inputs.porous(n, n, n, solid_fraction=0.7, rmin=3.0, rmax=8.0, seed=77)
    return dict(name=f"porous_{n}^3_d3q19", shape=(n, n, n), q=19, tau=0.6, force=(1e-5, 0, 0),
                bc=("periodic",) * 6, storage=storage, closure="none", solid=solid, u_bc=None, collision="trt",
                streaming=streaming)


def demo_closure_weights(seed=9):
    """Seeded network weights for timing the fused closure (the kernel's cost
    does not depend on their values); the trusted input range is unbounded."""
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.normal(0, 0.3, 192), rng.normal(0, 0.1, 32), rng.normal(0, 0.15, 1024),
                        rng.normal(0, 0.1, 32), rng.normal(0, 0.1, 32), [-5.0]])
    norm = np.concatenate([np.zeros(6), [1e-3, 1e-3, 1e-3, 1e-2, 1e-2, 1.0], np.full(6, -1e30), np.full(6, 1e30)])
    return np.concatenate([p, norm]).astype(np.float32)


KERNEL_SOURCES = ["paper_2305_09910_amd/csrc/lbm_kernels.hip", "paper_2305_09910_amd/csrc/lbm_et.hip",
                  "paper_2305_09910_amd/csrc/lbm_sparse.hip",
                  "paper_2305_09910_amd/csrc/lattice.h",
                  "paper_2305_09910_amd/csrc/stencil.h", "paper_2305_09910_amd/csrc/internal.h",
                  "paper_2305_09910_amd/csrc/mlp_wave.h"]
PROFILE = "profiles/stream_collide_obstacles_384x384x384_d3q27.md"


def kernel_source_hash():
    """Hash of the step kernels' code: comments and whitespace are dropped,
    so that editing a comment does not invalidate a profile."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(os.path.join(ROOT, f)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    import re
    path = os.path.join(ROOT, PROFILE)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel source sha256\[:16\]: `([0-9a-f]+)`", txt, re.I)
    t = re.search(r"HBM traffic per launch \(scaled\): ([0-9.]+) MB", txt)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1)) * 1e6


def make_lattice(cfg):
    from paper_2305_09910_amd import lbm
    lat = lbm.Lattice(cfg["shape"], q=cfg["q"], tau=cfg["tau"], force=cfg["force"], bc=cfg["bc"],
                      u_bc=cfg["u_bc"], solid=cfg["solid"], storage=cfg["storage"], closure=cfg["closure"],
                      collision=cfg.get("collision", "trt"), mrt_rates=cfg.get("mrt_rates"),
                      streaming=cfg.get("streaming", "aa"), hrr_sigma=cfg.get("hrr_sigma"))
    if cfg["closure"] == "mlp":
        lat.set_closure_weights(demo_closure_weights())
    rho, u = initial_fields(cfg)
    lat.init_equilibrium(rho, u)
    return lat


def time_lattice(cfg, steps, warmup, diag_every=1000):
    """Run warmup steps, then time `steps` steps.  Returns timing details.

    Whole-step time comes from host-synchronised wall clock around the timed
    region (diagnostics included); the stream-collide kernel's average
    duration comes from HIP events bracketing each run of step launches on
    the lattice's stream (diagnostics excluded)."""
    import torch
    lat = make_lattice(cfg)
    stream = lat.stream
    lat.step(warmup)
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    done = 0
    diag = []
    while done < steps:
        k = min(diag_every, steps - done) if diag_every > 0 else steps - done
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step(k)
        b.record(stream)
        ev.append((a, b, k))
        done += k
        if diag_every and done % diag_every == 0:
            rc, m, p = lat.totals(check=False)
            diag.append((rc, m))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    n = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    nfluid = n - (int(cfg["solid"].sum()) if cfg["solid"] is not None else 0)
    mass_ok = all(rc == 0 for rc, _ in diag)
    res = dict(cells=n, fluid_cells=nfluid, steps=steps, warmup=warmup, wall_s=wall,
               ms_per_step=1e3 * wall / steps, kernel_ms=kern_ms / steps,
               mlups=n * steps / wall / 1e6, kernel_mlups=n * steps / (kern_ms * 1e-3) / 1e6,
               mflups=nfluid * steps / wall / 1e6, finite=mass_ok)
    if cfg.get("streaming") == "sparse":
        vp = any(b in ("velocity", "pressure") for b in cfg["bc"])
        nb = sparse_bytes_per_fluid_cell(cfg["q"], BYTES[cfg["storage"]], vp)
        res["bytes_per_fluid_cell"] = nb
        moved = nb * nfluid
    else:
        nb = bytes_per_cell(cfg["q"], BYTES[cfg["storage"]], cfg["solid"] is not None,
                            cfg.get("collision") == "hrr")
        moved = nb * n
    res["bytes_per_cell"] = nb if moved == nb * n else moved / n
    res["achieved_gbs"] = moved / (res["kernel_ms"] * 1e-3) / 1e9
    res["roofline_frac"] = res["achieved_gbs"] / HBM_PEAK_GBS
    del lat
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(nbytes=2 << 30, reps=20):
    """Device copy bandwidth (read + write bytes per second), the STREAM analogue."""
    import torch
    from paper_2305_09910_amd import lbm
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    lbm.stream_copy(src, dst)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        lbm.stream_copy(src, dst)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


# ---------------------------------------------------------------------------
# FP64 oracle leg: the CPU baseline (the oracle timed on the host cores on a
# bounded copy of the headline workload) and, from the same kind of oracle
# runs on smaller copies of every workload, the velocity L2 error of each GPU
# form against FP64.
# ---------------------------------------------------------------------------
# name -> (workload config at the copy size, steps); which forms use it below
L2_REFS = {
    "obstacles_128^3_d3q27": (lambda: obstacle_cfg(128), 200),
    "channel_128x64x64": (lambda: channel_cfg(128, 64, 64), 1000),
    "channel_64x32x32_smagorinsky": (lambda: channel_cfg(64, 32, 32, closure="smagorinsky"), 1000),
    "channel_64x32x32_mlp_closure": (lambda: channel_cfg(64, 32, 32, closure="mlp"), 200),
    "channel_64x32x32_mrt": (lambda: channel_cfg(64, 32, 32, collision="mrt"), 1000),
    "channel_64x32x32_hrr": (lambda: channel_cfg(64, 32, 32, collision="hrr"), 1000),
    "obstacles_64^3_d3q27_mrt": (lambda: obstacle_cfg(64, collision="mrt"), 200),
    "porous_64^3_d3q19": (lambda: porous_cfg(64), 500),
}
HEADLINE = "obstacles_384^3_d3q27_f32"
CPU_BASELINE_REF = "obstacles_128^3_d3q27"


def l2_ref_of(form):
    """The oracle copy and GPU storage/streaming under which a form's velocity
    L2 error is measured: the same workload, collision, closure, storage and
    streaming scheme on a smaller copy (same recipe and seed)."""
    if form.startswith("obstacles"):
        return "obstacles_64^3_d3q27_mrt" if form.endswith("_mrt") else "obstacles_128^3_d3q27"
    if form.startswith("porous"):
        return "porous_64^3_d3q19"
    if "smagorinsky" in form:
        return "channel_64x32x32_smagorinsky"
    if "mlp_closure" in form:
        return "channel_64x32x32_mlp_closure"
    if form.endswith("_mrt"):
        return "channel_64x32x32_mrt"
    if form.endswith("_hrr"):
        return "channel_64x32x32_hrr"
    return "channel_128x64x64"


def run_oracle(cfg, steps):
    """FP64 two-lattice oracle on one workload from the same initial fields
    as the GPU run; returns (u [3][nz][ny][nx], seconds, threads)."""
    import oracle
    from paper_2305_09910_amd import inputs
    bcs = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "velocity": oracle.BC_VELOCITY,
           "pressure": oracle.BC_PRESSURE}
    cl = {"none": oracle.CL_NONE, "smagorinsky": oracle.CL_SMAG, "mlp": oracle.CL_MLP}[cfg["closure"]]
    o = oracle.Sim(cfg["q"], cfg["shape"], bc=tuple(bcs[b] for b in cfg["bc"]), tau=cfg["tau"], force=cfg["force"],
                   u_bc=cfg["u_bc"], solid=cfg["solid"], closure=cl, cs=0.1)
    if cfg.get("collision") == "mrt":
        o.set_mrt(cfg["mrt_rates"] if cfg["q"] == 27 else oracle.MRT_DHUMIERES)
    if cfg.get("collision") == "hrr":
        o.set_hrr(cfg["hrr_sigma"])
    if cl == oracle.CL_MLP:
        w = demo_closure_weights().astype(np.float64)
        o.set_mlp(w[:1313], w[1313:])
    rho, u = initial_fields(cfg)
    o.init_equilibrium(rho, u)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    _, uo = o.moments()
    return uo, dt


def initial_fields(cfg):
    from paper_2305_09910_amd import inputs
    nx, ny, nz = cfg["shape"]
    if cfg["name"].startswith("channel"):
        return inputs.channel(nx, ny, nz, 0.05, 0.05, seed=1234)
    if cfg["name"].startswith("porous"):
        return inputs.uniform_flow(nx, ny, nz, (0.0, 0, 0))
    rho, u = inputs.uniform_flow(nx, ny, nz, (0.04, 0, 0))
    if cfg["solid"] is not None:
        u[:, cfg["solid"] == 1] = 0.0
    return rho, u


def velocity_l2(u_gpu, u_orc, solid=None):
    """||u_gpu - u_orc||_2 / ||u_orc||_2 over the fluid cells, in FP64."""
    a = np.asarray(u_gpu, dtype=np.float64).reshape(3, -1)
    b = np.asarray(u_orc, dtype=np.float64).reshape(3, -1)
    if solid is not None:
        keep = np.asarray(solid).reshape(-1) == 0
        a, b = a[:, keep], b[:, keep]
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def oracle_leg(forms):
    """The oracle on the host cores: the CPU baseline, and the references for
    the velocity L2 error of every form (GPU run of the same copy, its
    storage, streaming, collision and closure, against the oracle's FP64)."""
    need = sorted({l2_ref_of(f) for f in forms} | {CPU_BASELINE_REF})
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    refs, cpu = {}, None
    for name in need:
        mk, steps = L2_REFS[name]
        cfg = mk()
        log(f"[bench] oracle {name}, {steps} steps")
        uo, dt = run_oracle(cfg, steps)
        refs[name] = (cfg, steps, uo)
        n = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
        log(f"[bench]   {n * steps / dt / 1e6:.1f} MLUPS, {dt:.1f} s")
        if name == CPU_BASELINE_REF:
            cpu = {"value": round(n * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                   "sample": f"{name} (the 128^3 copy of the headline obstacle flow: same recipe, seed and "
                             f"parameters), D3Q27 FP64 two-lattice oracle, {steps} steps from the initial state, "
                             f"{dt:.1f} s, OpenMP over z on {cores} threads",
                   "cpu_model": cpu_model()}
    return cpu, refs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gpu_l2(form, refs):
    """Velocity L2 error of a form: the GPU run of the form's copy against the
    oracle's FP64 run of the same copy."""
    from paper_2305_09910_amd import lbm
    name = l2_ref_of(form)
    cfg, steps, uo = refs[name]
    fcfg = form_cfg(form, sized=False)
    cfg = dict(cfg, storage=fcfg["storage"], streaming=fcfg.get("streaming", "aa"))
    lat = make_lattice(cfg)
    lat.step(steps)
    _, ug = lat.moments()
    err = velocity_l2(ug.cpu().numpy(), uo, cfg["solid"])
    del lat
    return {"value": float(f"{err:.3g}"), "copy": name, "steps": steps, "storage": cfg["storage"],
            "streaming": cfg["streaming"]}


# ---------------------------------------------------------------------------
# 2:1 refinement: a wall-refined channel (a coarse core between stacks of ever
# finer levels at both walls); each level at depth d takes 2^d steps per
# coarsest step (lbm_refine_tree_step)
# ---------------------------------------------------------------------------
REFINED = "refined_channel_512x128x256_d3q19_f32"
REFINED_TREE = "refined_tree_channel_256x64x128_d3q19_f32"
REFINED_FORMS = {  # coarse nx, ny, nz; ny of the levels at depth 1, 2, ...
    REFINED: (512, 128, 256, (64,)),
    REFINED_TREE: (256, 64, 128, (32, 32)),
}
REFINED_L2_COPY = {  # the same stacks scaled down, and the coarsest steps they run against the oracle
    REFINED: (64, 16, 32, (8,), 100),
    REFINED_TREE: (32, 16, 16, (8, 8), 100),
}
REFINED_NOTES = {
    REFINED: "2:1 refinement: fine levels at both walls, coarse core; MLUPS count every level's cell updates "
             "(fine cells twice per coarse step)",
    REFINED_TREE: "hierarchy of 2:1 levels: fine (4x) / medium (2x) / coarse / medium / fine along y; MLUPS count "
                  "every level's cell updates (2^depth per coarsest step)",
}


def refined_nodes(nxc, nyc, nzc, nys, storage="f32"):
    """A coarse core (nxc, nyc, nzc) between stacks of finer levels at both
    walls: the level at depth d (1, 2, ...) has (2^d nxc, nys[d-1], 2^d nzc)
    cells of size 2^-d coarse cells, tau_d = 1/2 + 2^d (tau_c - 1/2) and force
    F_c / 2^d, with tau_c = 0.51 and the body force of a centreline velocity of
    0.05.  Returned in tree order (coarse, then the lower and upper level of
    each depth), each with the indices of its finer neighbours below / above."""
    D = len(nys)
    H = nyc + sum(2 * ny / 2 ** d for d, ny in enumerate(nys, 1))
    tau = 0.51
    F = 8 * ((tau - 0.5) / 3) * 0.05 / H ** 2
    per, I = ("periodic", "periodic"), "interface"

    def mk(name, depth, shape, faces, lo, hi):
        return dict(name=name, depth=depth, shape=shape, q=19, tau=0.5 + 2 ** depth * (tau - 0.5),
                    force=(F / 2 ** depth, 0.0, 0.0), bc=per + faces + per, storage=storage, lo=lo, hi=hi, height=H,
                    h=2.0 ** -depth)

    nodes = [mk("c", 0, (nxc, nyc, nzc), (I, I) if D else ("noslip", "noslip"), 1 if D else None, 2 if D else None)]
    for d, ny in enumerate(nys, 1):
        shape, deeper = (2 ** d * nxc, ny, 2 ** d * nzc), d < D
        nodes.append(mk(f"lo{d}", d, shape, (I if deeper else "noslip", I), 2 * d + 1 if deeper else None, None))
        nodes.append(mk(f"hi{d}", d, shape, (I, I if deeper else "noslip"), None, 2 * d + 2 if deeper else None))
    # first rows and seeds from the bottom wall up
    order = [2 * d - 1 for d in range(D, 0, -1)] + [0] + [2 * d for d in range(1, D + 1)]
    y = 0.0
    for k, i in enumerate(order):
        nodes[i]["y0"], nodes[i]["seed"] = y, 1234 + k
        y += nodes[i]["shape"][1] * nodes[i]["h"]
    return nodes


def refined_fields(cfg):
    from paper_2305_09910_amd import inputs
    nx, ny, nz = cfg["shape"]
    return inputs.channel_level(nx, ny, nz, cfg["y0"], cfg["h"], cfg["height"], 0.05, 0.05, seed=cfg["seed"])


def make_refined(nodes):
    """GPU lattices in tree order as (Lattice, lo, hi) for refine_tree_step."""
    from paper_2305_09910_amd import lbm
    tree = []
    for cfg in nodes:
        lat = lbm.Lattice(cfg["shape"], q=19, tau=cfg["tau"], force=cfg["force"], bc=cfg["bc"], storage=cfg["storage"])
        lat.init_equilibrium(*refined_fields(cfg))
        tree.append((lat, cfg["lo"], cfg["hi"]))
    return tree


def time_refined(key, steps, warmup):
    """Cell updates per second over all levels (a level at depth d 2^d times
    per coarsest step), and the share of the time spent outside the levels'
    own step kernels (the exchange kernels and their launches)."""
    import torch
    from paper_2305_09910_amd import lbm
    nodes = refined_nodes(*REFINED_FORMS[key])
    tree = make_refined(nodes)
    stream = tree[0][0].stream
    lbm.refine_tree_step(tree, warmup)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    lbm.refine_tree_step(tree, steps)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = a.elapsed_time(b)
    # the same level steps without the exchange (their states advance further; timing only)
    a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a2.record(stream)
    for _ in range(steps):
        for (lat, _, _), cfg in zip(tree, nodes):
            lat.step(2 ** cfg["depth"])
    b2.record(stream)
    torch.cuda.synchronize()
    ms_levels = a2.elapsed_time(b2)
    updates = sum(cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2] * 2 ** cfg["depth"] for cfg in nodes)
    nb = bytes_per_cell(19, BYTES["f32"])
    # per child and parent step, 5 crossing directions, two exchanges per parent interface cell and
    # direction: 4 fine slots read and written and the parent's slot read (36 B) in each, then the
    # sum written (4 B) or read with the parent's slot written (8 B)
    xbytes = sum(2 ** cfg["depth"] * 5 * cfg["shape"][0] * cfg["shape"][2] * (36 + 4 + 36 + 8)
                 for cfg in nodes for child in (cfg["lo"], cfg["hi"]) if child is not None)
    moved = updates * nb + xbytes
    del tree
    torch.cuda.empty_cache()
    return {"mlups": round(updates * steps / wall / 1e6, 1), "kernel_mlups": round(updates * steps / (ms * 1e-3) / 1e6, 1),
            "cell_updates_per_coarse_step": updates, "levels": {cfg["name"]: cfg["shape"] for cfg in nodes},
            "bytes_per_coarse_step": moved, "achieved_gbs": round(moved * steps / (ms * 1e-3) / 1e9, 1),
            "roofline_frac": round(moved * steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "exchange_share": round(max(0.0, 1 - ms_levels / ms), 4), "us_per_coarse_step": round(1e3 * ms / steps, 1)}


def refined_l2(key):
    """Velocity L2 error of a refined form's scaled-down copy against the
    oracle after its coarsest steps, per level."""
    import oracle
    from paper_2305_09910_amd import lbm
    nxc, nyc, nzc, nys, steps = REFINED_L2_COPY[key]
    nodes = refined_nodes(nxc, nyc, nzc, nys)
    bcs = {"periodic": oracle.BC_PERIODIC, "noslip": oracle.BC_NOSLIP, "interface": oracle.BC_INTERFACE}
    orc = []
    for cfg in nodes:
        o = oracle.Sim(19, cfg["shape"], bc=tuple(bcs[b] for b in cfg["bc"]), tau=cfg["tau"], force=cfg["force"])
        o.init_equilibrium(*refined_fields(cfg))
        orc.append((o, cfg["lo"], cfg["hi"]))
    oracle.refine_tree_step(orc, steps)
    tree = make_refined(nodes)
    lbm.refine_tree_step(tree, steps)
    out = {}
    for (g, _, _), (o, _, _), cfg in zip(tree, orc, nodes):
        out[cfg["name"]] = float(f"{velocity_l2(g.moments()[1].cpu().numpy(), o.moments()[1]):.3g}")
    levels = ", ".join(f"{c['name']} {c['shape'][0]}x{c['shape'][1]}x{c['shape'][2]}" for c in nodes)
    return {"value": max(out.values()), "per_level": out, "copy": levels, "steps": steps}


PAPER_CONTEXT = {
    "kernel_mlups_per_node": 874, "roofline_mlups_per_node": 977, "bandwidth_gbs": 297.9, "bytes_per_cell": 304,
    "hardware": "one HAWK node, 2x AMD EPYC 7742 (128 cores), STREAM bandwidth",
    "workload": "D3Q19 MRT, FP64, Esoteric Twist in place, SoA, generated C kernels (LAGOON blocks of 24^3)",
    "source": "Section 5.2, Eq. (3)",
    "note": "another machine and precision: context, not the target",
}

FORMS = ["channel_256x128x128_f32", "channel_512x256x256_f32", "channel_512x256x256_f16",
         "channel_512x256x256_bf16", "channel_256x128x128_smagorinsky", "channel_256x128x128_mlp_closure",
         "channel_512x256x256_mlp_closure", "channel_512x256x256_mrt", "channel_512x256x256_hrr",
         "obstacles_384^3_d3q27_mrt",
         "channel_256x128x128_et", "channel_512x256x256_f32_et", "channel_512x256x256_f16_et",
         "obstacles_384^3_d3q27_et", "porous_256^3_d3q19_f32", "porous_256^3_d3q19_f32_sparse",
         "porous_256^3_d3q19_f16", "porous_256^3_d3q19_f16_sparse", "channel_256x128x128_mlp_closure_et"]

NOTES = {
    "channel_256x128x128_f32": "319 MB of populations, partly resident in the 256 MB last-level cache: "
                               "cache-assisted, not an HBM roofline figure",
    "channel_256x128x128_smagorinsky": "cache-assisted (319 MB state)",
    "channel_256x128x128_mlp_closure": "cache-assisted (319 MB state); bound by the vector ALU",
    "channel_256x128x128_et": "cache-assisted (319 MB state)",
    "channel_256x128x128_mlp_closure_et": "cache-assisted (319 MB state)",
}


def form_cfg(key, sized=True):
    table = {
        HEADLINE: lambda: obstacle_cfg(),
        "channel_256x128x128_f32": lambda: channel_cfg(256, 128, 128, "f32"),
        "channel_512x256x256_f32": lambda: channel_cfg(512, 256, 256, "f32"),
        "channel_512x256x256_f16": lambda: channel_cfg(512, 256, 256, "f16"),
        "channel_512x256x256_bf16": lambda: channel_cfg(512, 256, 256, "bf16"),
        "channel_256x128x128_smagorinsky": lambda: channel_cfg(256, 128, 128, "f32", "smagorinsky"),
        "channel_256x128x128_mlp_closure": lambda: channel_cfg(256, 128, 128, "f32", "mlp"),
        "channel_512x256x256_mlp_closure": lambda: channel_cfg(512, 256, 256, "f32", "mlp"),
        "channel_512x256x256_mrt": lambda: channel_cfg(512, 256, 256, "f32", collision="mrt"),
        "channel_512x256x256_hrr": lambda: channel_cfg(512, 256, 256, "f32", collision="hrr"),
        "obstacles_384^3_d3q27_mrt": lambda: obstacle_cfg(collision="mrt"),
        "channel_256x128x128_et": lambda: dict(channel_cfg(256, 128, 128, "f32"), streaming="et"),
        "channel_512x256x256_f32_et": lambda: dict(channel_cfg(512, 256, 256, "f32"), streaming="et"),
        "channel_512x256x256_f16_et": lambda: dict(channel_cfg(512, 256, 256, "f16"), streaming="et"),
        "obstacles_384^3_d3q27_et": lambda: dict(obstacle_cfg(), streaming="et"),
        "porous_256^3_d3q19_f32": lambda: porous_cfg(256, "f32"),
        "porous_256^3_d3q19_f32_sparse": lambda: porous_cfg(256, "f32", "sparse"),
        "porous_256^3_d3q19_f16": lambda: porous_cfg(256, "f16"),
        "porous_256^3_d3q19_f16_sparse": lambda: porous_cfg(256, "f16", "sparse"),
        "channel_256x128x128_mlp_closure_et": lambda: dict(channel_cfg(256, 128, 128, "f32", "mlp"),
                                                           streaming="et"),
    }
    if sized:
        return table[key]()
    # storage and streaming only (no full-size geometry): for the L2 copies
    st = "f16" if "_f16" in key else ("bf16" if "_bf16" in key else "f32")
    streaming = "et" if key.endswith("_et") else ("sparse" if key.endswith("_sparse") else "aa")
    return {"storage": st, "streaming": streaming}


def form_plan():
    for key in FORMS:
        yield key, form_cfg(key)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and velocity L2 errors)")
    ap.add_argument("--no-forms", action="store_true", help="headline workload only")
    ap.add_argument("--form-steps", type=int, default=300)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB once with the library's copy kernel (counter calibration)")
    ap.add_argument("--only-form", choices=[HEADLINE] + FORMS + list(REFINED_FORMS), default=None,
                    help="time only this form for --form-steps steps (for profiling); prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on exactly one GPU (asked for {args.gpus}); the multi-GPU halo "
              f"exchange is a design only.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2305_09910_amd import lbm
    lbm.lib()

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        lbm.stream_copy(src, dst)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
        torch.cuda.empty_cache()

    if args.only_form in REFINED_FORMS:
        log(f"[bench] form {args.only_form}, {args.form_steps} coarse steps")
        log(f"[bench]   {time_refined(args.only_form, args.form_steps, 20)}")
        return
    if args.only_form:
        log(f"[bench] form {args.only_form}, {args.form_steps} steps")
        fr = time_lattice(form_cfg(args.only_form), args.form_steps, 50, diag_every=0)
        log(f"[bench]   {fr['kernel_mlups']:.0f} MLUPS (kernel), {fr['achieved_gbs']:.0f} GB/s, "
            f"kernel {fr['kernel_ms'] * 1e3:.1f} us")
        return

    head = form_cfg(HEADLINE)
    log(f"[bench] headline {HEADLINE}, warmup {args.warmup}, steps {args.steps}")
    r = time_lattice(head, args.steps, args.warmup)
    log(f"[bench] headline: {r['mlups']:.0f} MLUPS, kernel {r['kernel_ms']*1e3:.1f} us, "
        f"{r['achieved_gbs']:.0f} GB/s ({100*r['roofline_frac']:.1f}% of 8 TB/s)")

    forms = {}
    bs = None
    if not args.no_forms:
        bs = copy_bandwidth()
        log(f"[bench] device copy bandwidth {bs:.0f} GB/s")
        fs = args.form_steps
        for key, cfg in form_plan():
            log(f"[bench] form {key}, {fs} steps")
            fr = time_lattice(cfg, fs, 50, diag_every=0)
            forms[key] = {"mlups": round(fr["mlups"], 1), "kernel_mlups": round(fr["kernel_mlups"], 1),
                          "mflups": round(fr["mflups"], 1), "fluid_cells": fr["fluid_cells"],
                          "bytes_per_cell": round(fr["bytes_per_cell"], 2),
                          "achieved_gbs": round(fr["achieved_gbs"], 1),
                          "roofline_frac": round(fr["roofline_frac"], 4),
                          "frac_of_copy": round(fr["achieved_gbs"] / bs, 4) if bs else None}
            if key in NOTES:
                forms[key]["note"] = NOTES[key]
            log(f"[bench]   {forms[key]}")
        for key in REFINED_FORMS:
            log(f"[bench] form {key}, {fs} coarse steps")
            forms[key] = time_refined(key, fs, 20)
            forms[key]["frac_of_copy"] = round(forms[key]["achieved_gbs"] / bs, 4) if bs else None
            forms[key]["note"] = REFINED_NOTES[key]
            log(f"[bench]   {forms[key]}")

    cpu, l2 = None, {}
    if not args.no_cpu_baseline:
        log("[bench] oracle leg: cpu baseline and velocity L2 references (oracle on host cores)")
        cpu, refs = oracle_leg([HEADLINE] + [f for f in forms if f not in REFINED_FORMS])
        log(f"[bench]   {cpu}")
        for key in REFINED_FORMS:
            if key in forms:
                forms[key]["velocity_l2_vs_oracle"] = refined_l2(key)
                log(f"[bench]   velocity L2 {key}: {forms[key]['velocity_l2_vs_oracle']}")
        for key in [HEADLINE] + [f for f in forms if f not in REFINED_FORMS]:
            l2[key] = gpu_l2(key, refs)
            log(f"[bench]   velocity L2 {key}: {l2[key]}")
            if key in forms:
                forms[key]["velocity_l2_vs_oracle"] = l2[key]
        torch.cuda.empty_cache()

    traffic = profiled_traffic()
    algo = r["bytes_per_cell"] * r["cells"]
    out = {
        "metric": "MLUPS and % HBM roofline, FP32 vs FP16-storage vs learned-closure",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "obstacle flow 384x384x384 D3Q27 TRT, velocity inflow 0.04 at -x, pressure "
                               "outflow at +x, periodic y/z, seeded solid spheres (radius 6-20) filling 10%, "
                               "FP32 storage",
                   "cells": r["cells"], "fluid_cells": r["fluid_cells"], "stencil": "D3Q27", "storage": "f32",
                   "tau": head["tau"], "diagnostics_every": 1000, "mflups": round(r["mflups"], 1)},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["roofline_frac"], 4),
                     "traffic": (round(traffic / 1e6, 1) if traffic else None),
                     "traffic_unit": "MB per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_mb_per_launch": round(algo / 1e6, 1),
                     "kernel": "k_stream_collide<27,f32,none,mask,TRT> (one launch per step)",
                     "bytes_per_cell": r["bytes_per_cell"], "kernel_us": round(r["kernel_ms"] * 1e3, 2),
                     "frac_of_copy": round(r["achieved_gbs"] / bs, 4) if bs else None},
        "velocity_l2_vs_oracle": l2.get(HEADLINE),
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "copy_bandwidth_gbs": round(bs, 1) if bs else None,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput benchmark of the D3Q19 hot path on one MI355X.

Headline workload: dense D3Q19 lid-driven cavity, 256^3 voxels, FP32
populations, bounce-back walls, lid velocity 0.1 along x, tau = 0.55, in the
disaggregated layout (shell blocks and interior blocks, one kernel each).
A step is one lbm_step: every group's fused collide-and-stream kernel over
the whole grid.  Inputs are synthetic and already resident in HBM when the
timed region starts.

Printed: one JSON line with MLUPS (million fluid-voxel updates per second),
the roofline of the dominant kernel (the interior-group kernel; 152 bytes
per FP32 update = 19 population reads + 19 writes, against 8 TB/s HBM), the
other arms (lexicographic single kernel, FP16/BF16-shifted storage, the
block-sparse wind tunnel with naive vs grouped kernels, the regularized
operator) and the FP64 CPU oracle timed on the host on a bounded sample of
the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--arms all|none]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM roofline, FP32 plain vs FP16-storage vs MLP closure"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {0: 152, 1: 76, 2: 76}  # FP32, FP16-shifted, BF16-shifted


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cavity(lbm, n=256, storage=0, schedule=1, tau=0.55, uw=0.1):
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (uw, 0.0, 0.0))
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, periodic=(False,) * 3, faces=faces, tau=tau,
                 storage=storage, schedule=schedule).bind()
    N = g.n
    g.init_equilibrium(np.ones(N), np.zeros((3, N)))
    return g


def tunnel(lbm, workloads, storage=0, schedule=1, tau=0.6, n=(512, 256, 256)):
    fluid, _ = workloads.sphere_packing(*n, seed=7898)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
        faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
    g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3, fluid=fluid, faces=faces,
                 tau=tau, storage=storage, schedule=schedule).bind()
    N = g.n
    u = np.zeros((3, N))
    u[0] = 0.05
    g.init_equilibrium(np.ones(N), u)
    return g, fluid


def taylor_green(lbm, workloads, n=256, collision=1, storage=0):
    k = 2 * math.pi / n
    rho, u = workloads.taylor_green_3d(n, 0.05)
    tau = workloads.tau_for_reynolds(1600.0, 0.05, k)
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, collision=collision, storage=storage).bind()
    g.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
    return g


def multires_sphere(lbm, workloads, storage=0, schedule=1, scale=1):
    """Flow past a sphere, 3 levels, coarsest 128x64x64 (finest 512x256x256),
    sphere radius 16 finest cells at (128, 128, 128), finest level within 24
    cells of the sphere, level 1 within a further 48; regularized inlet and
    outlet on x, periodic y and z, tau_coarsest = 0.52.  scale=2 doubles
    every length (the same shape at 8x the voxels)."""
    n = (512 * scale, 256 * scale, 256 * scale)
    lm, fluid = workloads.multires_sphere(*n, levels=3, center=(128.0 * scale,) * 3,
                                          radius=16.0 * scale, bands=(24.0 * scale, 48.0 * scale))
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    g = lbm.Grid(*n, kind=lbm.MULTIRES, levels=3, level_map=lm, fluid=fluid, periodic=(False, True, True),
                 faces=faces, tau=0.52, storage=storage, schedule=schedule).bind()
    for l in range(3):
        N = g.n_level(l)
        u = np.zeros((3, N))
        u[0] = 0.05
        g.init_equilibrium(np.ones(N), u, level=l)
    # updates per coarse step: every level-l voxel updates 2^(L-1-l) times
    g.updates_per_step = sum(g.n_level(l) * 2 ** (2 - l) for l in range(3))
    return g


def time_steps(torch, g, steps: int, warmup: int) -> float:
    """Seconds for `steps` lbm_step calls, after `warmup` untimed ones."""
    g.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(e0.elapsed_time(e1) / 1e3, 1e-9), wall


def time_launch(torch, lbm, g, k: int, reps: int) -> float:
    """Average duration (s) of launch k of the step, timed with HIP events on
    the stream the library launches on (torch's current stream)."""
    for _ in range(3):
        lbm.lbm_launch_group(g.h, k)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.lbm_launch_group(g.h, k)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("device_common.h", "step_kernels.hip", "launch.h", "lattice.h"):
        with open(os.path.join(ROOT, "paper_2503_07898_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(workloads, budget_s: float = 15.0):
    """The FP64 oracle on the same cavity (256^3, full box) for as many whole
    steps as fit in about budget_s seconds (at least 1)."""
    from oracle import oracle as orc
    orc.build()
    n = 256
    bc = [(orc.BB, (0, 0, 0))] * 5 + [(orc.MOVING, (0.1, 0.0, 0.0))]
    g = orc.Grid(n, n, n, periodic=(False,) * 3, bc=bc, tau=0.55)
    f = g.init_equilibrium(1.0, np.zeros(3))
    t0 = time.perf_counter()
    f = g.run(f, 1)
    t1 = time.perf_counter() - t0
    extra = max(0, min(9, int(budget_s / t1) - 1))
    t0 = time.perf_counter()
    if extra:
        f = g.run(f, extra)
    dt = t1 + (time.perf_counter() - t0)
    steps = 1 + extra
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        threads = min(threads, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    return {"value": round(n ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle, dense lid-driven cavity 256^3 (full box), {steps} step(s), "
                      f"{dt:.1f} s, OpenMP threads={threads}"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--arms", default="all", choices=["all", "none"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (torch) 5 times, the reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2503_07898_amd import lbm, workloads
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    lbm.lib()

    if args.copy_calibration:
        src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": src.numel() * 4, "launches": 5}))
        return 0

    # ---------------- headline: cavity 256^3, FP32, disaggregated ----------
    log("cavity 256^3 FP32 disaggregated")
    g = cavity(lbm)
    N = g.n
    dt, wall = time_steps(torch, g, args.steps, args.warmup)
    mlups = N * args.steps / dt / 1e6
    launches = g.launches()
    _, gb, gm, gf, tot = g.index_map(lbm.MAP_GROUPS)
    k_full = launches.index(int(gf))
    t_full = time_launch(torch, lbm, g, k_full, 50)
    upd_full = int(gf) * 64
    alg_bytes = upd_full * BYTES_PER_UPDATE[0]
    achieved = alg_bytes / t_full / 1e9
    kname = "k_block_interior<StoreF32, 0, false>"
    traffic = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "launch_blocks": int(gf), "updates_per_launch": upd_full,
                "bytes_per_update": BYTES_PER_UPDATE[0], "avg_launch_us": round(t_full * 1e6, 2)}
    step_frac = mlups * 1e6 * BYTES_PER_UPDATE[0] / 1e9 / HBM_PEAK_GBS
    g.close()
    del g
    torch.cuda.empty_cache()

    arms = {}
    if args.arms == "all":
        def arm(name, make, steps, bytes_per_update):
            log(name)
            gg = make()
            n_up = getattr(gg, "updates_per_step", None) or gg.n
            d, _ = time_steps(torch, gg, steps, 10)
            m = n_up * steps / d / 1e6
            arms[name] = {"MLUPS": round(m, 1),
                          "hbm_frac_alg": round(m * 1e6 * bytes_per_update / 1e9 / HBM_PEAK_GBS, 4),
                          "fluid_voxels": n_up, "launch_blocks": gg.launches()}
            gg.close()
            torch.cuda.empty_cache()

        arm("cavity256_f32_plain_lexicographic", lambda: cavity(lbm, schedule=0), 100, 152)
        arm("cavity256_f16_disagg", lambda: cavity(lbm, storage=1), 100, 76)
        arm("cavity256_bf16_disagg", lambda: cavity(lbm, storage=2), 100, 76)
        for st, bpu in ((0, 152), (1, 76)):
            for sch, nm in ((0, "naive_single_kernel"), (1, "disagg_grouped")):
                arm(f"tunnel512x256x256_{['f32', 'f16'][st]}_{nm}",
                    lambda st=st, sch=sch: tunnel(lbm, workloads, storage=st, schedule=sch)[0], 50, bpu)
        for st, bpu in ((0, 152), (1, 76)):
            for sch, nm in ((0, "unfused_baseline"), (1, "disagg_fused")):
                arm(f"multires_sphere_c128_{['f32', 'f16'][st]}_{nm}",
                    lambda st=st, sch=sch: multires_sphere(lbm, workloads, storage=st, schedule=sch), 50, bpu)
        for sch, nm in ((0, "unfused_baseline"), (1, "disagg_fused")):
            arm(f"multires_sphere_c256_f32_{nm}",
                lambda sch=sch: multires_sphere(lbm, workloads, schedule=sch, scale=2), 20, 152)
        arm("taylor_green256_re1600_f32_regularized", lambda: taylor_green(lbm, workloads, collision=1), 100, 152)
        arm("taylor_green256_re1600_f32_bgk", lambda: taylor_green(lbm, workloads, collision=0), 100, 152)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(workloads)

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense D3Q19 lid-driven cavity 256^3, FP32 shifted storage, "
                               "bounce-back walls, lid u=0.1, tau=0.55, disaggregated shell/interior kernels",
                   "fluid_voxels": N, "groups": {"shell": int(gb), "interior": int(gf)},
                   "step_hbm_frac_alg": round(step_frac, 4), "wall_s": round(wall, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "arms": arms,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

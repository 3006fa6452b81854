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
per FP32 update = 19 population reads + 19 writes, against 8 TB/s HBM, with
the measured HBM traffic when a counter summary of the same kernel source is
committed), the FP64 CPU oracle timed on the host on a bounded sample of the
same workload, and the other arms: lexicographic single kernel, FP16/BF16-
shifted storage, the block-sparse wind tunnel with the naive kernel against
memory-based and bitmask-based grouping (D3Q19 and D3Q27), the multires
sphere and the multires lid-driven cavity (unfused baseline against fused),
the regularized operator and the learned closure (with the share of HBM and
matrix-core peak of its interior launch).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--arms all|none|closure|storage|table]
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
# closure network per update on the matrix cores: 2 x (32x64 + 64x64 + 64x32)
# multiply-adds with the 19-wide layers padded to 32
MLP_MFMA_FLOPS = 2 * (32 * 64 + 64 * 64 + 64 * 32)
MFMA_BF16_PEAK_TFLOPS = 2500.0
# vector ALU issue without packed FP32 (which this library never emits): a
# wave64 instruction occupies one of a CU's 4 SIMDs (16 lanes) for 4 cycles,
# so 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
STORE_NAME = {0: "StoreF32", 1: "StoreF16", 2: "StoreBF16"}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def closure_net(torch, lbm, workloads, cases):
    """The learned closure for the MLP arms: the trained weights shipped with
    the package when present, else He-uniform weights standardized on
    samples of a regularized Taylor-Green run (same cost per update)."""
    from paper_2503_07898_amd import train_closure
    net = lbm.Mlp()
    w = train_closure.load()
    if w is not None:
        net.set_params(w[0])
        net.set_standardization(w[1])
        return net, "trained"
    net.set_params(lbm.flatten_params(workloads.mlp_he_uniform(7898)))
    g = cases.taylor_green(n=64, re=400.0, collision=lbm.REGULARIZED)
    g.step(50)
    net.fit_standardization(g.sample(1, 200_000))
    g.close()
    return net, "untrained"


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
    for f in ("device_common.h", "step_kernels.hip", "launch.h", "lattice.h", "mlp_device.h", "api.cpp"):
        with open(os.path.join(ROOT, "paper_2503_07898_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """Bytes per launch of `kernel` that left the L2 (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's readings) from the committed
    rocprofv3 counter summary, or None if absent or taken on a different
    kernel source.  An upper bound on the HBM bytes: reads that the Infinity
    Cache serves count too, and no counter on this stack separates them."""
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


def measured_valu(kernel: str):
    """Vector instructions per wave of `kernel` (SQ_INSTS_VALU / SQ_WAVES)
    from the committed rocprofv3 counter summary, or None if absent or taken
    on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "valu.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("valu_insts_per_wave")


def cpu_baseline(workloads, budget_s: float = 15.0):
    """The FP64 oracle on the same cavity (256^3, full box): as many whole
    steps as fit in about budget_s seconds (at least 1) on every OpenMP
    thread, plus one step on a single thread."""
    import ctypes
    from oracle import oracle as orc
    orc.build()
    L = orc.lib()
    omp_max = L.omp_get_max_threads
    omp_max.restype = ctypes.c_int
    omp_set = L.omp_set_num_threads
    omp_set.argtypes = [ctypes.c_int]
    threads = int(omp_max())
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
    omp_set(1)
    t0 = time.perf_counter()
    g.run(f, 1)
    dt1 = time.perf_counter() - t0
    omp_set(threads)
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(n ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "value_1_thread": round(n ** 3 / dt1 / 1e6, 3), "cpu": cpu,
            "sample": f"FP64 oracle, dense lid-driven cavity 256^3 (full box), {steps} step(s) in "
                      f"{dt:.1f} s on {threads} OpenMP threads; 1 step in {dt1:.1f} s on 1 thread"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--arms", default="all", choices=["all", "none", "closure", "storage", "tunnel", "table"],
                    help="closure: only the learned-closure arms; storage: only the 16-bit cavity "
                         "arms; tunnel: only the D3Q19 wind-tunnel arms (these three for counter "
                         "runs); table: the 320^3 and 480^3 multires cavity rows of table multiResLbm")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (torch) 5 times, the reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(one process drives one GPU); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2503_07898_amd import cases, lbm, workloads
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
    g = cases.cavity()
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
    kname = "lbm::k19::k_block_interior<lbm::k19::StoreF32, 0, false, true>"
    traffic = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "launch_blocks": int(gf), "updates_per_launch": upd_full,
                "bytes_per_update": BYTES_PER_UPDATE[0], "avg_launch_us": round(t_full * 1e6, 2)}
    step_frac = mlups * 1e6 * BYTES_PER_UPDATE[0] / 1e9 / HBM_PEAK_GBS
    # off the timed loop: FP64 reductions and the macroscopic read-out
    aux = {}
    for name, fn in (("reduce_fp64_ms", g.reduce), ("read_macroscopic_fp32_ms", lambda: g.macroscopic(f64=False))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        aux[name] = round(e0.elapsed_time(e1) / 10, 3)
    g.close()
    del g
    torch.cuda.empty_cache()

    arms = {}
    if args.arms in ("all", "closure", "storage", "tunnel", "table"):
        def arm(name, make, steps, bytes_per_update, interior=None):
            log(name)
            gg = make()
            n_up = getattr(gg, "updates_per_step", None) or gg.n
            d, _ = time_steps(torch, gg, steps, 10)
            m = n_up * steps / d / 1e6
            arms[name] = {"MLUPS": round(m, 1),
                          "hbm_frac_alg": round(m * 1e6 * bytes_per_update / 1e9 / HBM_PEAK_GBS, 4),
                          "fluid_voxels": n_up, "launch_blocks": gg.launches()}
            if getattr(gg, "kind", None) == lbm.BLOCK_SPARSE:
                # per-slot reading: every slot of an active block moves its bytes,
                # solid or fluid
                slots = int(gg.index_map(lbm.MAP_GROUPS)[4]) * 64
                arms[name]["slots"] = slots
                arms[name]["hbm_frac_slot"] = round(m * 1e6 * slots / n_up * bytes_per_update / 1e9
                                                    / HBM_PEAK_GBS, 4)
            if interior is not None:
                # the interior (full-group) launch alone: HBM and matrix-core shares
                _, _, _, nf, _ = gg.index_map(lbm.MAP_GROUPS)
                t = time_launch(torch, lbm, gg, gg.launches().index(int(nf)), 20)
                ups = int(nf) * 64
                arms[name]["interior_launch"] = {
                    "avg_launch_us": round(t * 1e6, 2), "updates": ups,
                    "hbm_GBs": round(ups * bytes_per_update / t / 1e9, 1),
                    "hbm_frac": round(ups * bytes_per_update / t / 1e9 / HBM_PEAK_GBS, 4),
                    "mfma_TFLOPs_bf16": round(ups * MLP_MFMA_FLOPS / t / 1e12, 1),
                    "mfma_frac": round(ups * MLP_MFMA_FLOPS / t / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)}
                # the binding resource of the closure: vector-instruction issue,
                # from the counted instructions per wave (a wave takes one block
                # with FP32 storage, two with 16-bit storage)
                pb = 1 if interior == lbm.F32 else 2
                kname = f"lbm::k19::k_block_interior_mlp<lbm::k19::{STORE_NAME[interior]}, false, true, {pb}>"
                vpw = measured_valu(kname)
                waves = (int(nf) + pb - 1) // pb
                il = arms[name]["interior_launch"]
                il["valu_insts_per_wave"] = vpw
                il["blocks_per_wave"] = pb
                il["valu_lane_Tops"] = None if vpw is None else round(vpw * 64 * waves / t / 1e12, 2)
                il["valu_frac"] = None if vpw is None else round(vpw * 64 * waves / t / VALU_LANE_PEAK, 4)
                il["bound"] = "valu"
            gg.close()
            torch.cuda.empty_cache()

    if args.arms == "storage":
        arm("cavity256_f16_disagg", lambda: cases.cavity(storage=lbm.F16_SHIFTED), 20, 76)
        arm("cavity256_bf16_disagg", lambda: cases.cavity(storage=lbm.BF16_SHIFTED), 20, 76)
    if args.arms == "all":
        arm("cavity256_f32_plain_lexicographic", lambda: cases.cavity(schedule=lbm.PLAIN_SINGLE_KERNEL), 100, 152)
        arm("cavity256_f16_disagg", lambda: cases.cavity(storage=lbm.F16_SHIFTED), 100, 76)
        arm("cavity256_bf16_disagg", lambda: cases.cavity(storage=lbm.BF16_SHIFTED), 100, 76)
    if args.arms in ("all", "tunnel"):
        for st, bpu in ((lbm.F32, 152), (lbm.F16_SHIFTED, 76)):
            for sch, nm in ((lbm.PLAIN_SINGLE_KERNEL, "naive_single_kernel"), (lbm.DISAGG, "disagg_grouped"),
                            (lbm.DISAGG_BITMASK, "disagg_bitmask")):
                arm(f"tunnel512x256x256_{['f32', 'f16'][st]}_{nm}",
                    lambda st=st, sch=sch: cases.tunnel(storage=st, schedule=sch), 50, bpu)
    if args.arms == "all":
        # multires schedules: the unfused baseline, the paper's own (uniform
        # blocks fused, jump blocks unfused) and every group fused
        mr_schedules = ((lbm.PLAIN_SINGLE_KERNEL, "unfused_baseline"),
                        (lbm.DISAGG_UNIFORM_FUSED, "paper_uniform_fused"), (lbm.DISAGG, "disagg_fused"))
        for st, bpu in ((lbm.F32, 152), (lbm.F16_SHIFTED, 76)):
            for sch, nm in mr_schedules:
                arm(f"multires_sphere_c128_{['f32', 'f16'][st]}_{nm}",
                    lambda st=st, sch=sch: cases.multires_sphere(storage=st, schedule=sch), 50, bpu)
        for sch, nm in mr_schedules:
            arm(f"multires_sphere_c256_f32_{nm}",
                lambda sch=sch: cases.multires_sphere(schedule=sch, scale=2), 20, 152)
        # D3Q27 (the lattice of the paper's block-sparse register study):
        # 27 reads + 27 writes per update
        for st, bpu in ((lbm.F32, 216), (lbm.F16_SHIFTED, 108)):
            for sch, nm in ((lbm.PLAIN_SINGLE_KERNEL, "naive_single_kernel"), (lbm.DISAGG, "disagg_grouped"),
                            (lbm.DISAGG_BITMASK, "disagg_bitmask")):
                arm(f"tunnel512x256x256_d3q27_{['f32', 'f16'][st]}_{nm}",
                    lambda st=st, sch=sch: cases.tunnel(storage=st, schedule=sch, q=27), 50, bpu)
        arm("cavity256_d3q27_f32_disagg", lambda: cases.cavity(q=27), 50, 216)
        # the paper's own multires benchmark shape: lid-driven cavity, 512^3
        # finest box, 77.6M / 4.09M / 0.37M voxels on levels 0 / 1 / 2
        for sch, nm in mr_schedules:
            arm(f"multires_cavity512_f32_{nm}", lambda sch=sch: cases.multires_cavity(schedule=sch), 10, 152)
        # the 4-level rows of table multiResLbm (77.6M / 2.98M / 0.48M / 0.004M voxels)
        for sch, nm in mr_schedules:
            arm(f"multires_cavity512_4lvl_f32_{nm}",
                lambda sch=sch: cases.multires_cavity(schedule=sch, levels=4), 10, 152)
        arm("taylor_green256_re1600_f32_regularized",
            lambda: cases.taylor_green(collision=lbm.REGULARIZED), 100, 152)
        arm("taylor_green256_re1600_f32_bgk", lambda: cases.taylor_green(collision=lbm.BGK), 100, 152)

    if args.arms == "table":
        # the other sizes of table multiResLbm (320^3 and 480^3, 3 and 4
        # levels), each schedule; not in the default run (every grid takes
        # some seconds to build on the host)
        mr_schedules = ((lbm.PLAIN_SINGLE_KERNEL, "unfused_baseline"),
                        (lbm.DISAGG_UNIFORM_FUSED, "paper_uniform_fused"), (lbm.DISAGG, "disagg_fused"))
        for n in (320, 480):
            for levels in (3, 4):
                for sch, nm in mr_schedules:
                    arm(f"multires_cavity{n}_{levels}lvl_f32_{nm}",
                        lambda n=n, levels=levels, sch=sch: cases.multires_cavity(n=n, schedule=sch, levels=levels),
                        10, 152)

    if args.arms in ("all", "closure"):
        # the learned closure in place of the collision operator
        net, which = closure_net(torch, lbm, workloads, cases)

        def with_net(g):
            g.set_collision(lbm.MLP, net)
            return g

        for name, make in (("taylor_green256_re1600_f32_mlp", lambda: cases.taylor_green()),
                           ("taylor_green256_re1600_f16_mlp",
                            lambda: cases.taylor_green(storage=lbm.F16_SHIFTED)),
                           ("cavity256_f32_mlp", lambda: cases.cavity()),
                           ("cavity256_f16_mlp", lambda: cases.cavity(storage=lbm.F16_SHIFTED))):
            net.fallbacks(reset=True)
            arm(name, lambda make=make: with_net(make()), 50, 76 if "f16" in name else 152,
                interior=lbm.F16_SHIFTED if "f16" in name else lbm.F32)
            arms[name]["closure"] = which
            arms[name]["fallbacks"] = net.fallbacks()
        net.close()

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
                   "step_hbm_frac_alg": round(step_frac, 4), "wall_s": round(wall, 3), **aux},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "arms": arms,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Train the learned collision closure on the solver's own regularized runs.

Data: pre-collision populations of non-boundary fluid voxels sampled at 20
evenly spaced times from regularized-operator runs of the three benchmark
geometries (dense cavity 256^3 over 2000 steps, block-sparse wind tunnel
512x256x256 over 1000 steps, multires sphere over 1000 coarse steps), one
third of the samples from each.  Rows that are not finite are dropped.
Training: the
library's own kernels (matrix-core forward, backward, Adam), batch 4096,
learning rate cosine-decayed from 1e-3 to 1e-5, He-uniform initialization.

Usage (on the GPU):
    python -m paper_2503_07898_amd.train_closure --samples 10000000 --epochs 20 \\
        --out paper_2503_07898_amd/closure_weights.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import cases, lbm, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "closure_weights.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def dataset(n_total: int, seed: int = 2025, times: int = 20):
    """n_total pre-collision samples [n][19] (FP32 device tensor)."""
    import torch
    per_case = n_total // 3
    parts = []
    # dense cavity, 2000 steps
    g = cases.cavity(collision=lbm.REGULARIZED)
    for k in range(times):
        g.step(2000 // times)
        parts.append(g.sample(seed + k, per_case // times))
    g.close()
    log(f"  cavity samples done")
    # block-sparse wind tunnel, 1000 steps
    g = cases.tunnel(collision=lbm.REGULARIZED)
    for k in range(times):
        g.step(1000 // times)
        parts.append(g.sample(seed + 100 + k, per_case // times))
    g.close()
    log(f"  tunnel samples done")
    # multires sphere, 1000 coarse steps; levels sampled by their share of updates
    g = cases.multires_sphere(collision=lbm.REGULARIZED)
    w = np.array([g.n_level(l) * 2 ** (2 - l) for l in range(3)], np.float64)
    share = w / w.sum()
    rest = n_total - 2 * (per_case // times) * times
    for k in range(times):
        g.step(1000 // times)
        for l in range(3):
            parts.append(g.sample(seed + 200 + 3 * k + l, int(rest / times * share[l]), level=l))
    g.close()
    log(f"  multires samples done")
    data = torch.cat(parts)
    ok = torch.isfinite(data).all(1)
    if not bool(ok.all()):
        log(f"  dropping {int((~ok).sum())} non-finite rows")
        data = data[ok].contiguous()
    return data


def train(data, epochs: float, batch: int = 4096, lr0: float = 1e-3, lr_min: float = 1e-5, seed: int = 0,
          init_seed: int = 7898, net=None, log_every: int = 200):
    """Train a closure on `data` (device tensor [n][19]); returns (Mlp, losses)."""
    import torch
    m = net or lbm.Mlp()
    if net is None:
        m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(init_seed)))
        m.fit_standardization(data)
    n = data.shape[0]
    iters = max(1, int(epochs * n / batch))
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float64, device=data.device)
    hist = []
    t0 = time.perf_counter()
    for t in range(1, iters + 1):
        idx = torch.as_tensor(rng.integers(0, n, batch), device=data.device)
        lr = lr_min + 0.5 * (lr0 - lr_min) * (1 + math.cos(math.pi * (t - 1) / iters))
        m.train_step(data, lr, t, loss, idx=idx)
        if t == 1 or t % log_every == 0 or t == iters:
            hist.append((t, loss.item()))
            log(f"  iter {t}/{iters} loss {hist[-1][1]:.3e} ({time.perf_counter() - t0:.1f} s)")
    return m, hist


def save(m, path: str, meta: dict | None = None) -> None:
    with open(path, "w") as fh:
        json.dump({"params": [float(x) for x in m.params()],
                   "standardization": [float(x) for x in m.standardization()],
                   "meta": meta or {}}, fh)


def load(path: str = DEFAULT_WEIGHTS):
    """(params [6675] float32, standardization [128] float32, meta) or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    return np.asarray(d["params"], np.float32), np.asarray(d["standardization"], np.float32), d.get("meta", {})


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=float, default=20.0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    t0 = time.perf_counter()
    log(f"generating {args.samples} samples")
    data = dataset(args.samples)
    t1 = time.perf_counter()
    log(f"training {args.epochs} epochs")
    m, hist = train(data, args.epochs)
    t2 = time.perf_counter()
    meta = {"samples": int(data.shape[0]), "epochs": args.epochs, "batch": 4096, "loss_history": hist,
            "data_s": round(t1 - t0, 1), "train_s": round(t2 - t1, 1)}
    save(m, args.out, meta)
    print(json.dumps({"loss_first": hist[0][1], "loss_last": hist[-1][1], **{k: v for k, v in meta.items()
                                                                             if k != "loss_history"}}))
    return 0


if __name__ == "__main__":
    sys.exit(main())

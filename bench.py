#!/usr/bin/env python3
"""Benchmark of the superquadric renderer hot path on one MI355X.

A step is one pass of the whole hot path over one synthetic batch: index build
(sq_build_index), differentiable forward with transmittance checkpoints
(sq_render_fwd) and backward (sq_render_bwd) for fixed random upstream
gradients.  Default workload: 6 cameras x 900 x 1600 rays, 25,600
superquadrics (40% in 64 dense blobs), 200 samples per ray in [0.1, 50] m,
17 classes, 200x200x16 grid at 0.4 m, N_v = 5.

Prints ONE JSON line.  `value` is forward+backward ray-samples/s (R*L per
step time) with all inputs resident in HBM.  The roofline object describes the
dominant kernel (the backward); its FLOP count per launch is the per-unit
algorithmic FLOPs times the unit counts a counting run of the same kernels
reports (pairs listed / evaluated, samples)."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-samples/s fwd & fwd+bwd at 6×900×1600, 25.6k SQs; % HBM/VALU roofline"

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# FP32 vector without packed math: 256 CU x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic FLOPs per unit (each FMA = 2, add/mul/compare = 1, transcendental = 1)
#   listed pair (transform + cull test):                 3 sub + 9 FMA + 3 abs/max/cmp = 24
#   evaluated pair, forward:      24 + 9 trans + 5 mul + 2 add + FMA(a) + C FMA(s) = 40 + 2 + 2C
#   evaluated pair, backward recompute: 40 + FMA(a) + C FMA(gamma) + FMA(G)     = 44 + 2C
#   evaluated pair, backward adjoint: 40 + C FMA(gamma) + derivatives (~81)
#                                    + one add per summed contribution (15 + C)   = 136 + 3C
#   sample visited (pinned point + voxel): 6 + 6 + 6 compares + 5 int            = 23
#   live sample compositing: min, 2 mul, FMA(D), C FMA(S), 2 (T)                  = 7 + 2C
# The backward's algorithmic recompute is the forward's work (its unit counts);
# evaluations the kernel spends past a ray's saturation inside its last chunk
# are overhead and are not counted.


def api_cp(C):
    """class count padded to the compiled kernel widths"""
    return 4 if C <= 4 else 8 if C <= 8 else 17 if C <= 17 else 32


def flops_fwd(st, C):
    samples, listed, evaluated = st["samples"], st["listed"], st["evaluated"]
    return 24 * listed + (16 + 2 * C) * evaluated + (23 + 7 + 2 * C) * samples


def flops_bwd(fst, bst, C):
    recompute = 24 * fst["listed"] + (20 + 2 * C) * fst["evaluated"] + (23 + 7 + 2 * C) * fst["samples"]
    adjoint = 24 * bst["listed2"] + (112 + 3 * C) * bst["eval2"] + (23 + 10) * bst["samples2"]
    return recompute + adjoint


def recorded_traffic(kernel_name):
    """Calibrated HBM bytes per launch of `kernel_name` from the committed counter
    runs (profiles/hbm_traffic.json), or None when the kernel sources changed
    since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, "paper_2511_17361_amd", "csrc", f), "rb").read()
                   for f in ("render.hip", "sqr_device.h"))
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    k = rec["kernels"].get(kernel_name)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4, help="workload config (4 = 6x900x1600, 25.6k SQs)")
    ap.add_argument("--ckpt-every", type=int, default=4)
    ap.add_argument("--tile-w", type=int, default=8)
    ap.add_argument("--wpb", type=int, default=4)
    ap.add_argument("--bwd-mode", type=int, default=0, help="0 auto, 1 sample-major, 2 primitive-major")
    ap.add_argument("--cpu-rays", type=int, default=8192, help="rays in the oracle's CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-stats", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB once (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(sc, n_rays, seed=0):
    """The FP64 oracle (forward + adjoint) on a seeded ray sample of the same
    workload, single process."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(sc.rays.n_rays, n_rays, replace=False))
    C = sc.prims.n_classes
    g_d = rng.standard_normal(n_rays)
    g_s = rng.standard_normal((n_rays, C))
    index = oracle.build_index(sc.prims.means, sc.grid)[:3]      # untimed: the index is shared
    t0 = time.perf_counter()
    oracle.render(sc.grid, sc.prims, sc.rays, sc.march, index=index, ray_ids=ids)
    oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s, index=index, ray_ids=ids)
    dt = time.perf_counter() - t0
    rs = n_rays * sc.march.n_samples / dt
    return dict(value=rs, unit="ray-samples/s", cores=1, kind="oracle",
                sample=f"{n_rays} seeded rays of the same workload, forward + adjoint, FP64 NumPy, "
                       f"one process ({dt:.1f} s); index build excluded")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2511_17361_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    sc = synth.config(args.config)
    grid, march = api.Grid.of(sc.grid), api.March.of(sc.march)
    prims = api.Prims.from_numpy(sc.prims, dev)
    rays = api.Rays.from_numpy(sc.rays, dev)
    C = sc.prims.n_classes
    K = args.ckpt_every
    tune = api.Tuning(args.tile_w, args.wpb, args.bwd_mode)
    rng = np.random.default_rng(1)
    g_d_np, g_s_np = synth.upstream_grads(rng, sc.rays, C)
    g_d = torch.from_numpy(g_d_np).to(dev)
    g_s = torch.from_numpy(g_s_np).to(dev)
    ws_i, ws_r = api.Workspace(dev), api.Workspace(dev)
    R = sc.rays.n_rays
    Ls = sc.march.n_samples
    stream = torch.cuda.current_stream()

    idx = api.build_index(grid, prims, ws=ws_i)
    fwd_out = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=K, tuning=tune, ws=ws_r)
    bwd_out = api.render_bwd(grid, idx, prims, rays, march, fwd_out["ckpt"], K, g_d, g_s, tuning=tune, ws=ws_r)
    torch.cuda.synchronize()
    E = idx.checked_total()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        api.build_index(grid, prims, ws=ws_i, out=idx)
        if ev:
            ev[1].record(stream)
        api.render_fwd(grid, idx, prims, rays, march, ckpt_every=K, tuning=tune, ws=ws_r, out=fwd_out)
        if ev:
            ev[2].record(stream)
        api.render_bwd(grid, idx, prims, rays, march, fwd_out["ckpt"], K, g_d, g_s, tuning=tune, ws=ws_r,
                       out=bwd_out)
        if ev:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_idx = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_fwd = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    t_bwd = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    ms_step = wall * 1e3 / args.steps

    # plain forward (no checkpoints) beside the differentiable one
    plain = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=0, tuning=tune, ws=ws_r)
    torch.cuda.synchronize()
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    pe[0].record(stream)
    for _ in range(args.steps):
        api.render_fwd(grid, idx, prims, rays, march, ckpt_every=0, tuning=tune, ws=ws_r, out=plain)
    pe[1].record(stream)
    torch.cuda.synchronize()
    t_plain = pe[0].elapsed_time(pe[1]) / args.steps

    result = {
        "metric": METRIC,
        "value": R * Ls / (ms_step / 1e3),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"config {args.config}: {sc.rays.shape[0]} cameras x {sc.rays.shape[1]}x"
                                f"{sc.rays.shape[2]} rays, {sc.prims.n} superquadrics, L={Ls} in "
                                f"[{sc.march.t_near}, {sc.march.t_far}] m, C={C}, grid "
                                f"{'x'.join(map(str, sc.grid.dims))} at {sc.grid.voxel} m, N_v={sc.grid.nv}; "
                                "step = index + forward(ckpt) + backward"),
                   "rays": R, "samples_per_ray": Ls, "superquadrics": sc.prims.n, "classes": C,
                   "ckpt_every": K, "tile_w": args.tile_w, "waves_per_block": args.wpb,
                   "bwd_mode": args.bwd_mode},
        "fwd_ray_samples_per_s": R * Ls / (t_fwd / 1e3),
        "plain_fwd_ray_samples_per_s": R * Ls / (t_plain / 1e3),
        "rays_per_s_fwd_bwd": R / (ms_step / 1e3),
        "index_ms": t_idx, "fwd_ms": t_fwd, "bwd_ms": t_bwd, "plain_fwd_ms": t_plain,
        "index_entries": E,
    }

    if not args.no_stats:
        st = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=0, tuning=tune, ws=ws_r, stats=True)
        bst = api.render_bwd_stats(grid, idx, prims, rays, march, fwd_out["ckpt"], K, g_d, g_s, tuning=tune,
                                   ws=ws_r) if hasattr(api, "render_bwd_stats") else None
        torch.cuda.synchronize()
        s = st["stats"].cpu().numpy()
        fst = dict(samples=int(s[0]), listed=int(s[1]), evaluated=int(s[2]))
        result["units_fwd"] = fst
        f_fwd = flops_fwd(fst, C)
        result["fwd_tflops"] = f_fwd / (t_plain / 1e3) / 1e12
        if bst is not None:
            b = {k: int(v) for k, v in bst.items()}
            result["units_bwd"] = b
            f_bwd = flops_bwd(fst, b, C)
            ach = f_bwd / (t_bwd / 1e3) / 1e12
            kname = f"sqr::k_render_bwd_km<{api_cp(C)}, {K}, false>"
            result["roofline"] = {"bound": "alu", "kernel": kname, "achieved": ach,
                                  "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / VALU_PEAK_TFLOPS,
                                  "traffic": recorded_traffic(kname), "flop_per_launch": f_bwd,
                                  "kernel_ms": t_bwd}
        result["fwd_roofline_frac"] = result["fwd_tflops"] / VALU_PEAK_TFLOPS

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = 4 * n

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_rays)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the superquadric renderer hot path on one MI355X.

A step is one pass of the whole hot path over one synthetic batch: index build
(sq_build_index), differentiable forward with transmittance checkpoints and
the per-sample stash (sq_batch_io.stash; --no-stash leaves it out) and backward
(sq_render_bwd) for fixed random upstream gradients.  Default workload: 6 cameras x 900 x 1600 rays, 25,600
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

# MI355X published peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s
# (256 CUs x 4 SIMDs x 2.4 GHz x 64 FLOP per SIMD and clock, which needs packed
# FP32).  These kernels are built without packed FP32, so one FP32 instruction
# occupies a SIMD for 4 clocks (16 lanes per clock): 78.6 TFLOP/s with FMAs.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 157.3
VALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

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


def flops_bwd(fst, C, stash=False):
    """Algorithmic FLOPs of the backward over the method's own (sample,
    primitive) pairs, the forward's counts: the recompute and the adjoint each
    cover every listed pair of every live sample once.  Work the kernel skips
    because it is provably zero (samples past a ray's end in pass 1, primitives
    with p = 0 throughout a chunk in pass 2) is neither added nor removed.
    With the stash there is no recompute: each live sample's G_j = <g_S, s_j>
    (C FMAs) takes its place."""
    adjoint = 24 * fst["listed"] + (112 + 3 * C) * fst["evaluated"] + (23 + 10) * fst["samples"]
    if stash:
        return adjoint + 2 * C * fst["samples"]
    recompute = 24 * fst["listed"] + (20 + 2 * C) * fst["evaluated"] + (23 + 7 + 2 * C) * fst["samples"]
    return recompute + adjoint


def _source_hash():
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_2511_17361_amd", "csrc", f), "rb").read()
                   for f in ("render.hip", "sqr_device.h", "index.hip"))
    return hashlib.sha256(src).hexdigest()[:16]


def recorded_profile():
    """Per-kernel counter figures of the committed profile runs
    (profiles/render_counters.json: calibrated HBM bytes, VALU issue
    utilisation, lane occupancy, LDS bank-conflict rate, instruction counts),
    with `current` telling whether the kernel sources still hash to the
    profiled version.  None when the file is absent."""
    path = os.path.join(ROOT, "profiles", "render_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    rec["current"] = rec.get("source_sha256_16") == _source_hash()
    return rec


def stage_bytes(R, C, L, K, N, V, E, probs=True, ckpt=True, stash_samples=0):
    """Algorithmic HBM bytes of each stage (inputs read once, outputs written
    once; lists, records and per-sample state that stay on chip are not
    counted):
      index:    means 12 N, counts and offsets 4 V each, ids 4 E;
      forward:  rays 24 R, primitives 120 N, depth and t_final 4 R each, sem
                4 C R, probs 4 C R, checkpoints 4 ceil(L/K) R, and with the
                stash 4 (Q + 2) per live sample (Q: C padded to 4, 8, 16, 32);
      backward: rays 24 R, primitives 120 N, g_D 4 R, g_S 4 C R, checkpoints
                4 ceil(L/K) R, gradients 4 (13 + C) N, and the stash read back."""
    nck = -(-L // K)
    cp = api_cp(C)
    q = cp // 16 * 16 if cp >= 16 else cp
    st = 4 * (q + 2) * stash_samples
    idx = 12 * N + 8 * V + 4 * E
    fwd = 24 * R + 120 * N + 8 * R + 4 * C * R * (2 if probs else 1) + (4 * nck * R if ckpt else 0) + st
    bwd = 24 * R + 120 * N + 4 * R + 4 * C * R + 4 * nck * R + 4 * (13 + C) * N + st
    return dict(index=idx, fwd=fwd, bwd=bwd)


def form(ms, rays, L, listed, hbm_bytes=None):
    """Rates of one form of the path over `ms` milliseconds."""
    t = ms / 1e3
    d = dict(ms=ms, rays_per_s=rays / t, ray_samples_per_s=rays * L / t, pairs_per_s=listed / t)
    if hbm_bytes is not None:
        d["hbm_gb_per_s"] = hbm_bytes / t / 1e9
        d["hbm_frac"] = hbm_bytes / t / 1e9 / HBM_PEAK_GBS
    return d


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4, help="workload config (4 = 6x900x1600, 25.6k SQs)")
    ap.add_argument("--ckpt-every", type=int, default=8)
    ap.add_argument("--tile-w", type=int, default=8)
    ap.add_argument("--wpb", type=int, default=2)
    ap.add_argument("--bwd-mode", type=int, default=0, help="0 auto, 1 sample-major, 2 primitive-major")
    ap.add_argument("--cpu-rays", type=int, default=6 * 8192, help="rays in the oracle's CPU sample")
    ap.add_argument("--cpu-procs", type=int, default=0, help="CPU-baseline worker processes (0: every core, <= 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-stats", action="store_true")
    ap.add_argument("--no-stash", action="store_true",
                    help="no per-sample stash: the backward recomputes each chunk's a_j and G_j")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the tuning given by --tile-w/--wpb/--ckpt-every instead of timing the default "
                         "candidates first and running the fastest")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB once (HBM counter calibration)")
    return ap.parse_args()


_CPU = {}


def _cpu_tile(span):
    """One worker's share of the CPU baseline: the oracle's forward and adjoint
    over rays [s, e) of the seeded sample (one NumPy thread per process)."""
    import oracle
    from threadpoolctl import threadpool_limits
    s, e = span
    c = _CPU
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.render(c["sc"].grid, c["sc"].prims, c["sc"].rays, c["sc"].march, index=c["index"],
                      ray_ids=c["ids"][s:e])
        oracle.render_grad(c["sc"].grid, c["sc"].prims, c["sc"].rays, c["sc"].march, c["gd"][s:e], c["gs"][s:e],
                           index=c["index"], ray_ids=c["ids"][s:e])
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_procs_default():
    """Worker processes of the CPU baseline: every core this process may run
    on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(sc, n_rays, procs, seed=0, tile=512):
    """The FP64 oracle (forward + adjoint) on a seeded ray sample of the same
    workload, split into tiles of `tile` rays over `procs` forked worker
    processes.  Runs before anything initialises the GPU (the workers are
    forks of this process).  The index is built once, untimed, and shared."""
    import multiprocessing as mp

    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(sc.rays.n_rays, n_rays, replace=False))
    C = sc.prims.n_classes
    _CPU.update(sc=sc, ids=ids, gd=rng.standard_normal(n_rays), gs=rng.standard_normal((n_rays, C)),
                index=oracle.build_index(sc.prims, sc.grid)[:3])
    spans = [(s, min(n_rays, s + tile)) for s in range(0, n_rays, tile)]
    with mp.get_context("fork").Pool(procs) as pool:
        t0 = time.perf_counter()
        busy = pool.map(_cpu_tile, spans, chunksize=1)
        wall = time.perf_counter() - t0
    _CPU.clear()
    rs = n_rays * sc.march.n_samples / wall
    return dict(value=rs, unit="ray-samples/s", cores=procs, kind="oracle",
                cpu_model=_cpu_model(), os_cpu_count=os.cpu_count(),
                sample=(f"{n_rays} seeded rays of the same workload (a subset: {n_rays / sc.rays.n_rays:.2%} of its "
                        f"rays), forward + adjoint, FP64 NumPy, {len(spans)} tiles of {tile} rays over {procs} "
                        f"processes ({wall:.1f} s wall, {sum(busy):.1f} s of worker time); index build excluded"))


def sq_major_ab(dev, steps, K=4):
    """A/B of the two backward strategies on the 6,400-superquadric workload
    (6 cameras x 352x200 rays, L = 100): the default wavefront-reduced
    atomics against the superquadric-major grouping of interactions."""
    import numpy as np
    import torch

    import synth
    from paper_2511_17361_amd import api
    sc = synth.config(1)
    grid, march = api.Grid.of(sc.grid), api.March(sc.march.n_samples, sc.march.t_near, sc.march.t_far, K)
    prims, rays = api.Prims.from_numpy(sc.prims, dev), api.Rays.from_numpy(sc.rays, dev)
    idx = api.build_index(grid, prims)
    out = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=K)
    gd, gs = synth.upstream_grads(np.random.default_rng(4), sc.rays, sc.prims.n_classes)
    gd, gs = torch.from_numpy(gd).to(dev), torch.from_numpy(gs).to(dev)
    probe = api.render_bwd_sq_major(grid, idx, prims, rays, march, out["ckpt"], K, gd, gs, 0)
    torch.cuda.synchronize()
    E = int(probe["interactions"].item())
    iws = None

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    lib_ws = {}
    t_atomic = timed(lambda: api.render_bwd(grid, idx, prims, rays, march, out["ckpt"], K, gd, gs))
    t_sqm = timed(lambda: lib_ws.__setitem__("g", api.render_bwd_sq_major(grid, idx, prims, rays, march,
                                                                          out["ckpt"], K, gd, gs, E)))
    return dict(workload="6,400 superquadrics, 6 cameras x 352x200 rays, L=100, K=4", interactions=E,
                atomics_ms=t_atomic, sq_major_ms=t_sqm)


def size_stash(batch, tune, stream, headroom=1.25):
    """Give `batch` a per-sample stash: a forward with only the header and
    slot table counts the slots it asks for, and the pool gets that many
    times `headroom` (for every tiling the autotuner may pick; a chunk left
    without a slot is recomputed)."""
    import torch
    batch.set_stash(0)
    with torch.cuda.stream(stream):
        batch.build_index(stream=stream)
        batch.render_fwd(tune, stream=stream)
    torch.cuda.synchronize()
    demand = batch.stash_demand()
    slots = int(demand * headroom) + 64
    batch.set_stash(slots)
    return dict(demand=demand, slots=slots, gib=batch.buf["stash"].numel() * 4 / 2 ** 30)


def batched_8_scenes(dev, steps, warmup, use_stash=True):
    """The batched training step over the 8 scenes of uneven size (2k .. 25.6k
    superquadrics, 94k in all; 6 cameras x 352x200 rays each, L = 100), with the
    tuning chosen by the autotuner, captured once and replayed."""
    import numpy as np
    import torch

    import synth
    from paper_2511_17361_amd import api
    scenes = [synth.config(3, s) for s in range(8)]
    sc0 = scenes[0]
    grid = api.Grid.of(sc0.grid)
    march = api.March(sc0.march.n_samples, sc0.march.t_near, sc0.march.t_far, 4)
    dprims = [(api.Prims.from_numpy(s.prims, dev), api.Rays.from_numpy(s.rays, dev)) for s in scenes]
    batch = api.Batch(grid, march, dprims, device=dev, min_chunk=4)
    rng = np.random.default_rng(3)
    for i, s in enumerate(scenes):
        gd, gs = synth.upstream_grads(rng, s.rays, s.prims.n_classes)
        batch.set_upstream(i, torch.from_numpy(gd).to(dev), torch.from_numpy(gs).to(dev))
    stream = torch.cuda.Stream(device=dev)
    stash = size_stash(batch, api.Tuning(8, 2, 0, 1, 4), stream) if use_stash else None
    with torch.cuda.stream(stream):
        tune, _ = batch.autotune(api.default_candidates(), reps=1, stream=stream)
    torch.cuda.synchronize()
    batch.capture(tune, stream=stream)
    for _ in range(warmup):
        batch.replay(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.replay(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    batch.release_graph()
    st = torch.zeros(4, dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        batch.render_fwd(tune, stats=st, stream=stream)
    torch.cuda.synchronize()
    listed = int(st[1].item())
    samples = batch.n_rays * sc0.march.n_samples
    return dict(workload="8 scenes, 2k..25.6k superquadrics (94k), 6 cameras x 352x200 rays each, L=100, "
                         "step = index + forward(checkpoints) + backward, autotuned, one hipGraph replay",
                superquadrics=sum(s.prims.n for s in scenes), rays=batch.n_rays, step_ms=ms,
                ray_samples_per_s=samples / (ms / 1e3), listed_pairs=listed,
                rays_per_s=batch.n_rays / (ms / 1e3), pairs_per_s=listed / (ms / 1e3),
                tuning=dict(tile_w=tune.tile_w, waves_per_block=tune.waves_per_block, bwd_mode=tune.bwd_mode,
                            persistent=tune.persistent, chunk=tune.chunk), stash=stash)


def paper_setting(dev, steps):
    """The paper's render setting: 6 cameras x 704x256 rays, 1,600 superquadrics,
    L = 100 in [0.1, 40] m, N_v = 5.  Timed: the index build and the plain
    forward (depth, semantics and probabilities, no checkpoints), the render the
    paper times per frame of six views in Table tab:ablation_render_occ.  The
    primitives are synthetic, so the paper's figure is context only."""
    import torch

    import synth
    from paper_2511_17361_amd import api
    sc = synth.paper_render_scene()
    grid, march = api.Grid.of(sc.grid), api.March.of(sc.march)
    prims, rays = api.Prims.from_numpy(sc.prims, dev), api.Rays.from_numpy(sc.rays, dev)
    wi, wf = api.Workspace(dev), api.Workspace(dev)
    idx = api.build_index(grid, prims, ws=wi)
    out = api.render_fwd(grid, idx, prims, rays, march, ws=wf)
    torch.cuda.synchronize()
    E = idx.checked_total()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    t_idx = timed(lambda: api.build_index(grid, prims, ws=wi, out=idx))
    t_fwd = timed(lambda: api.render_fwd(grid, idx, prims, rays, march, ws=wf, out=out))
    R = sc.rays.n_rays
    return dict(workload=("6 cameras x 704x256 rays, 1600 superquadrics, L=100 in [0.1, 40] m, N_v=5, C=17, "
                          "grid 200x200x16 at 0.4 m; synthetic primitives; index + plain forward"),
                index_entries=E, index_ms=t_idx, fwd_ms=t_fwd, render_ms=t_idx + t_fwd,
                ray_samples_per_s=R * sc.march.n_samples / ((t_idx + t_fwd) / 1e3),
                paper=dict(render_ms=17.2, hardware="1x NVIDIA A100",
                           source="Table tab:ablation_render_occ, six views, trained primitives"))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 (sharding over several GPUs is a design, not code)"}))
        sys.exit(2)
    import numpy as np

    import synth
    scenes = [synth.config(3, s) for s in range(8)] if args.config == 3 else [synth.config(args.config)]
    sc0 = scenes[0]
    # the CPU baseline forks its workers before anything touches the GPU
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc0, args.cpu_rays, args.cpu_procs or cpu_procs_default())

    import torch

    from paper_2511_17361_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    grid = api.Grid.of(sc0.grid)
    march = api.March(sc0.march.n_samples, sc0.march.t_near, sc0.march.t_far, args.ckpt_every)
    C = sc0.prims.n_classes
    dprims = [(api.Prims.from_numpy(s.prims, dev), api.Rays.from_numpy(s.rays, dev)) for s in scenes]
    batch = api.Batch(grid, march, dprims, device=dev, min_chunk=4)
    rng = np.random.default_rng(1)
    ups = []
    for i, s in enumerate(scenes):
        gd, gs = synth.upstream_grads(rng, s.rays, C)
        ups.append((torch.from_numpy(gd).to(dev), torch.from_numpy(gs).to(dev)))
        batch.set_upstream(i, *ups[i])
    R = batch.n_rays
    Ls = sc0.march.n_samples
    stream = torch.cuda.Stream(device=dev)

    tune = api.Tuning(args.tile_w, args.wpb, args.bwd_mode, 1, args.ckpt_every)
    # the per-sample stash, sized by the slots a first forward asks for
    stash = None if args.no_stash else size_stash(batch, tune, stream)
    tuned_ms = None
    cands = api.default_candidates()
    if not args.no_autotune:
        with torch.cuda.stream(stream):
            tune, tuned_ms = batch.autotune(cands, reps=2, stream=stream)
    torch.cuda.synchronize()

    # the step: index + forward with checkpoints + backward, captured once and replayed
    with torch.cuda.stream(stream):
        batch.step(tune, stream=stream)
    torch.cuda.synchronize()
    E = [int(x) for x in batch.buf["totals"].cpu().tolist()]
    for e, cap in zip(E, batch.caps):
        assert e <= cap, "index capacity exceeded"
    batch.capture(tune, stream=stream)
    for _ in range(args.warmup):
        batch.replay(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.replay(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    batch.release_graph()
    if stash is not None:
        # the slots the timed step's forward (the chosen tuning) asked for, against the pool
        hdr = batch.buf["stash"][:16].view(torch.int32).cpu().tolist()
        stash["covered"] = hdr[4] <= hdr[5]
        stash["demand_step"] = hdr[4]

    # per-stage kernel time (HIP events on the launch stream), eager
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        for i in range(args.steps):
            evs[i][0].record(stream)
            batch.build_index(stream=stream)
            evs[i][1].record(stream)
            batch.render_fwd(tune, stream=stream)
            evs[i][2].record(stream)
            batch.render_bwd(tune, stream=stream)
            evs[i][3].record(stream)
    torch.cuda.synchronize()
    t_idx = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_fwd = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    t_bwd = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    ref_out = [{k: batch.scene_outputs(i)[k].clone() for k in ("depth", "probs")} for i in range(len(scenes))]

    # the plain per-scene forward (no checkpoints) beside the differentiable and batched forms
    plain = []
    for s, (p, r) in zip(scenes, dprims):
        idx = api.build_index(grid, p)
        plain.append((p, r, idx, api.render_fwd(grid, idx, p, r, march, ckpt_every=0,
                                                 tuning=api.Tuning(tune.tile_w, tune.waves_per_block))))
    torch.cuda.synchronize()
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    pe[0].record()
    for _ in range(args.steps):
        for p, r, idx, out in plain:
            api.render_fwd(grid, idx, p, r, march, ckpt_every=0, out=out,
                           tuning=api.Tuning(tune.tile_w, tune.waves_per_block))
    pe[1].record()
    torch.cuda.synchronize()
    t_plain = pe[0].elapsed_time(pe[1]) / args.steps

    # training step with the loss of Eq. eq:loss fused into the forward (synthetic pseudo-labels)
    lrng = np.random.default_rng(2)
    for i, s in enumerate(scenes):
        sl, dl = synth.pseudo_labels(lrng, s.rays, C, s.march.t_near, s.march.t_far)
        batch.set_labels(i, torch.from_numpy(sl).to(dev), torch.from_numpy(dl).to(dev))
    batch.capture(tune, stream=stream, loss=api.PAPER_LOSS)
    for _ in range(args.warmup):
        batch.replay(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.replay(stream)
    torch.cuda.synchronize()
    ms_train = (time.perf_counter() - t0) * 1e3 / args.steps
    batch.release_graph()
    train_loss = [float(x) for x in batch.buf["loss"].cpu().tolist()]

    # early ray termination (Supplement "Ray Termination"): the step and the forward at kappa = 1e-4, 1e-2
    kappa_ms = {}
    for kappa in (1e-4, 1e-2):
        batch.set_kappa(kappa)
        batch.capture(tune, stream=stream)
        for _ in range(args.warmup):
            batch.replay(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.replay(stream)
        torch.cuda.synchronize()
        step_k = (time.perf_counter() - t0) * 1e3 / args.steps
        batch.release_graph()
        ke = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        with torch.cuda.stream(stream):
            ke[0].record(stream)
            for _ in range(args.steps):
                batch.render_fwd(tune, stream=stream)
            ke[1].record(stream)
        torch.cuda.synchronize()
        kappa_ms[f"{kappa:g}"] = dict(step_ms=step_k, fwd_ms=ke[0].elapsed_time(ke[1]) / args.steps)
    batch.set_kappa(0.0)

    # influence-thresholded index (grid.theta): index size, step time and the change of the renders
    theta_ab = {}
    for theta in (1e-3, 1e-2):
        gt = api.Grid(grid.lo, grid.voxel, grid.dims, grid.nv, theta)
        bt = api.Batch(gt, march, dprims, device=dev, min_chunk=4)
        for i in range(len(scenes)):
            bt.set_upstream(i, *ups[i])
        with torch.cuda.stream(stream):
            bt.step(tune, stream=stream)
        torch.cuda.synchronize()
        et = sum(int(x) for x in bt.buf["totals"].cpu().tolist())
        bt.capture(tune, stream=stream)
        for _ in range(args.warmup):
            bt.replay(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bt.replay(stream)
        torch.cuda.synchronize()
        step_t = (time.perf_counter() - t0) * 1e3 / args.steps
        bt.release_graph()
        dd, dp = 0.0, 0.0
        for i in range(len(scenes)):
            o = bt.scene_outputs(i)
            d0 = ref_out[i]["depth"]
            dd = max(dd, float(((o["depth"] - d0).abs() / d0.clamp_min(0.1)).max()))
            dp = max(dp, float((o["probs"] - ref_out[i]["probs"]).abs().max()))
        theta_ab[f"{theta:g}"] = dict(index_entries=et, step_ms=step_t, max_rel_depth_change=dd,
                                      max_prob_change=dp)
        del bt
    torch.cuda.synchronize()

    # voxelisation of each scene's grid (Eq. eq:voxelisation, tau = 0.05) from the same index
    vox = [api.voxelise(grid, idx, p, tau=0.05) for p, r, idx, out in plain]
    torch.cuda.synchronize()
    ve = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ve[0].record()
    for _ in range(args.steps):
        for (p, r, idx, out), vo in zip(plain, vox):
            api.voxelise(grid, idx, p, tau=0.05, out=vo)
    ve[1].record()
    torch.cuda.synchronize()
    t_vox = ve[0].elapsed_time(ve[1]) / args.steps

    workload = (f"{len(scenes)} scene(s), {sum(s.prims.n for s in scenes)} superquadrics "
                f"({'/'.join(str(s.prims.n) for s in scenes)}), {sc0.rays.shape[0]} cameras x "
                f"{sc0.rays.shape[2]}x{sc0.rays.shape[1]} rays per scene, L={Ls} in [{sc0.march.t_near}, "
                f"{sc0.march.t_far}] m, C={C}, grid {'x'.join(map(str, sc0.grid.dims))} at {sc0.grid.voxel} m, "
                f"N_v={sc0.grid.nv}; step = index + forward(checkpoints"
                f"{', per-sample stash' if stash else ''}) + backward, one hipGraph replay")

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
        "config": {"workload": workload, "scenes": len(scenes), "rays": R, "samples_per_ray": Ls,
                   "superquadrics": sum(s.prims.n for s in scenes), "classes": C,
                   "tuning": dict(tile_w=tune.tile_w, waves_per_block=tune.waves_per_block,
                                  bwd_mode=tune.bwd_mode, persistent=tune.persistent,
                                  chunk=tune.chunk or args.ckpt_every),
                   "autotuned": not args.no_autotune, "stash": stash},
        "fwd_ray_samples_per_s": R * Ls / (t_fwd / 1e3),
        "plain_fwd_ray_samples_per_s": R * Ls / (t_plain / 1e3),
        "rays_per_s_fwd_bwd": R / (ms_step / 1e3),
        "index_ms": t_idx, "fwd_ms": t_fwd, "bwd_ms": t_bwd, "plain_fwd_ms": t_plain,
        "index_entries": sum(E),
        "kappa_ms": kappa_ms,
        "theta_index": theta_ab,
        "train_step_ms": ms_train,
        "train_ray_samples_per_s": R * Ls / (ms_train / 1e3),
        "train_loss": train_loss,
        "voxelise_ms": t_vox,
        "voxelise_voxels_per_s": len(scenes) * grid.n_voxels / (t_vox / 1e3),
        "voxelise_pairs_per_s": sum(E) / (t_vox / 1e3),
    }
    if tuned_ms is not None:
        result["autotune"] = [dict(tile_w=c.tile_w, waves_per_block=c.waves_per_block, chunk=c.chunk,
                                   persistent=c.persistent, step_ms=round(m, 3)) for c, m in zip(cands, tuned_ms)]

    K = tune.chunk or args.ckpt_every
    if not args.no_stats:
        st = torch.zeros(4, dtype=torch.int64, device=dev)
        bst = torch.zeros(6, dtype=torch.int64, device=dev)
        with torch.cuda.stream(stream):
            batch.render_fwd(tune, stats=st, stream=stream)
            batch.render_bwd(tune, stats=bst, stream=stream)
        torch.cuda.synchronize()
        s = st.cpu().numpy()
        fst = dict(samples=int(s[0]), listed=int(s[1]), evaluated=int(s[2]))
        b = dict(zip(api.BWD_STAT_NAMES, [int(v) for v in bst.cpu().numpy()]))
        result["units_fwd"] = fst
        result["units_bwd"] = b
        result["fwd_tflops"] = flops_fwd(fst, C) / (t_fwd / 1e3) / 1e12
        result["fwd_roofline_frac"] = result["fwd_tflops"] / VALU_PEAK_TFLOPS
        result["fwd_roofline_frac_nonpacked"] = result["fwd_tflops"] / VALU_NONPACKED_TFLOPS
        stashed = stash is not None and stash["covered"]
        f_bwd = flops_bwd(fst, C, stash=stashed)
        ach = f_bwd / (t_bwd / 1e3) / 1e12
        kname = f"sqr::k_render_bwd_km<{api_cp(C)}, {K}, false, {'true' if tune.persistent else 'false'}>"
        prof = recorded_profile()
        kprof = (prof or {}).get("kernels", {}).get(kname) if prof and prof["current"] else None
        traffic = None if kprof is None else kprof["read_bytes"] + kprof["write_bytes"]
        result["roofline"] = {"bound": "alu", "kernel": kname, "achieved": ach, "peak": VALU_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": ach / VALU_PEAK_TFLOPS,
                              "traffic": traffic, "flop_per_launch": f_bwd, "kernel_ms": t_bwd,
                              "peak_nonpacked": VALU_NONPACKED_TFLOPS,
                              "frac_nonpacked": ach / VALU_NONPACKED_TFLOPS}
        # every form of the path at this workload: rays/s, ray-samples/s, pairs/s (the
        # method's listed (sample, primitive) pairs), algorithmic HBM GB/s and its fraction
        N = sum(s_.prims.n for s_ in scenes)
        sb = stage_bytes(R, C, Ls, K, N, grid.n_voxels * len(scenes), sum(E),
                         stash_samples=fst["samples"] if stashed else 0)
        sbp = stage_bytes(R, C, Ls, K, N, grid.n_voxels * len(scenes), sum(E), ckpt=False)
        P = fst["listed"]
        result["forms"] = {
            "plain_fwd": form(t_plain, R, Ls, P, sbp["fwd"]),
            "differentiable_fwd": form(t_fwd, R, Ls, P, sb["fwd"]),
            "bwd": form(t_bwd, R, Ls, P, sb["bwd"]),
            "fwd_bwd_step": form(ms_step, R, Ls, P, sb["index"] + sb["fwd"] + sb["bwd"]),
            "index": dict(ms=t_idx, entries=sum(E), hbm_gb_per_s=sb["index"] / (t_idx / 1e3) / 1e9,
                          hbm_frac=sb["index"] / (t_idx / 1e3) / 1e9 / HBM_PEAK_GBS),
        }
        if prof is not None:
            keep = ("valu_issue_util", "valu_lane_occupancy", "lds_bank_conflict_rate", "valu_insts",
                    "valu_trans_insts", "read_bytes", "write_bytes")
            result["profile"] = {
                "source": "profiles/render_counters.json (rocprofv3 counter runs of this bench, committed)",
                "current": prof["current"], "tuning": prof.get("tuning"),
                "kernels": {k: {f: v[f] for f in keep if f in v} for k, v in prof["kernels"].items()
                            if k.startswith("sqr::k_render") or k.startswith("sqr::k_tile_lists")}}

    result["sq_major_ab"] = sq_major_ab(dev, args.steps)
    result["batched_8_scenes"] = batched_8_scenes(dev, args.steps, args.warmup, use_stash=not args.no_stash)
    result["paper_setting"] = paper_setting(dev, args.steps)

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = 4 * n

    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Torch-facing binding of the renderer's C ABI.

PyTorch only provides device memory (tensors) and the current HIP stream;
every step of the method runs in libsqr.so.  Each function below fills the
ctypes structs of include/sqr.h from tensors, allocates outputs and the
workspace with torch, and calls one C entry point.
"""
from __future__ import annotations

import ctypes as ct
import os
import dataclasses
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return t


@dataclass
class Grid:
    lo: tuple
    voxel: float
    dims: tuple
    nv: int
    theta: float = 0.0      # influence threshold of the index (0: the N_v cube)

    def c(self) -> L.SqGrid:
        g = L.SqGrid()
        for i in range(3):
            g.lo[i] = float(self.lo[i])
            g.dims[i] = int(self.dims[i])
        g.voxel = float(self.voxel)
        g.nv = int(self.nv)
        g.theta = float(self.theta)
        return g

    @property
    def n_voxels(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    @staticmethod
    def of(obj) -> "Grid":
        return obj if isinstance(obj, Grid) else Grid(tuple(obj.lo), float(obj.voxel), tuple(obj.dims), int(obj.nv),
                                                      float(getattr(obj, "theta", 0.0)))


@dataclass
class March:
    n_samples: int
    t_near: float
    t_far: float
    ckpt_every: int = 0
    kappa: float = 0.0      # early ray termination threshold (0 = none)

    def c(self, ckpt_every: Optional[int] = None) -> L.SqMarch:
        m = L.SqMarch()
        m.n_samples = int(self.n_samples)
        m.t_near = float(self.t_near)
        m.t_far = float(self.t_far)
        m.ckpt_every = int(self.ckpt_every if ckpt_every is None else ckpt_every)
        m.kappa = float(self.kappa)
        return m

    @staticmethod
    def of(obj) -> "March":
        return obj if isinstance(obj, March) else March(int(obj.n_samples), float(obj.t_near), float(obj.t_far),
                                                        int(getattr(obj, "ckpt_every", 0)),
                                                        float(getattr(obj, "kappa", 0.0)))


@dataclass
class Prims:
    """Device copies of the primitive parameters (float32, contiguous)."""
    means: torch.Tensor
    quats: torch.Tensor
    scales: torch.Tensor
    eps: torch.Tensor
    opacity: torch.Tensor
    logits: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_classes(self) -> int:
        return int(self.logits.shape[1])

    def c(self) -> L.SqPrims:
        p = L.SqPrims()
        p.n = self.n
        p.n_classes = self.n_classes
        for name in ("means", "quats", "scales", "eps", "opacity", "logits"):
            setattr(p, name, _ptr(_f32(getattr(self, name), name)))
        return p

    @staticmethod
    def from_numpy(pr, device="cuda") -> "Prims":
        f = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return Prims(f(pr.means), f(pr.quats), f(pr.scales), f(pr.eps), f(pr.opacity), f(pr.logits))


@dataclass
class Rays:
    origins: torch.Tensor   # [cams,H,W,3]
    dirs: torch.Tensor      # [cams,H,W,3]

    @property
    def shape(self):
        return tuple(self.origins.shape[:3])

    def c(self) -> L.SqRays:
        r = L.SqRays()
        r.n_cams, r.height, r.width = self.shape
        r.origins = _ptr(_f32(self.origins, "origins"))
        r.dirs = _ptr(_f32(self.dirs, "dirs"))
        return r

    @staticmethod
    def from_numpy(rays, device="cuda") -> "Rays":
        f = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return Rays(f(rays.origins), f(rays.dirs))


@dataclass
class Tuning:
    tile_w: int = 8
    waves_per_block: int = 4
    bwd_mode: int = L.SQ_BWD_AUTO
    persistent: int = 1
    chunk: int = 0

    def c(self) -> L.SqTuning:
        t = L.SqTuning()
        t.tile_w = int(self.tile_w)
        t.waves_per_block = int(self.waves_per_block)
        t.bwd_mode = int(self.bwd_mode)
        t.persistent = int(self.persistent)
        t.chunk = int(self.chunk)
        return t


@dataclass
class Index:
    counts: torch.Tensor
    offsets: torch.Tensor
    ids: torch.Tensor
    total: torch.Tensor      # one int64 on the device
    capacity: int

    def c(self) -> L.SqIndex:
        i = L.SqIndex()
        i.counts = _ptr(self.counts)
        i.offsets = _ptr(self.offsets)
        i.ids = _ptr(self.ids)
        i.capacity = int(self.capacity)
        i.total = _ptr(self.total)
        return i

    def checked_total(self) -> int:
        """Synchronise and return E; raise if the capacity was too small."""
        e = int(self.total.item())
        if e > self.capacity:
            raise L.SqrError(L.SQ_ERR_CAPACITY, f"index needs {e} entries, capacity {self.capacity}")
        return e


def capacity_bound(grid: Grid, n: int) -> int:
    g = grid.c()
    return int(L.load().sq_index_capacity_bound(ct.byref(g), int(n)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Workspace:
    """Reusable device scratch buffer (grown on demand, never shrunk)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = _workspace(nbytes, self.device)
        return self.buf


def build_index(grid, prims: Prims, capacity: Optional[int] = None, stream=None, ws: Optional[Workspace] = None,
                out: Optional[Index] = None) -> Index:
    """sq_build_index: superquadric -> voxel CSR lists."""
    lib = L.load()
    grid = Grid.of(grid)
    dev = prims.means.device
    g = grid.c()
    if out is None:
        cap = capacity_bound(grid, prims.n) if capacity is None else int(capacity)
        out = Index(torch.empty(grid.n_voxels, dtype=torch.int32, device=dev),
                    torch.empty(grid.n_voxels, dtype=torch.int32, device=dev),
                    torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                    torch.zeros(1, dtype=torch.int64, device=dev), cap)
    need = lib.sq_build_index_workspace(ct.byref(g), prims.n)
    wbuf = ws.get(need) if ws is not None else _workspace(need, dev)
    p = prims.c()
    ix = out.c()
    L.check(lib.sq_build_index(ct.byref(g), ct.byref(p), ct.byref(ix), _ptr(wbuf), wbuf.numel(),
                               _stream_handle(stream)))
    return out


def render_fwd(grid, index: Index, prims: Prims, rays: Rays, march, ckpt_every: int = 0, probs: bool = True,
               stats: bool = False, tuning: Optional[Tuning] = None, stream=None,
               ws: Optional[Workspace] = None, out: Optional[dict] = None) -> dict:
    """sq_render_fwd.  Returns depth [cams,H,W], sem [cams,C,H,W], probs, t_final,
    ckpt ([ceil(L/K), R] when ckpt_every > 0) and stats (4 int64) when asked."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    cams, H, W = rays.shape
    C = prims.n_classes
    R = cams * H * W
    if out is None:
        out = dict(depth=torch.empty((cams, H, W), device=dev), sem=torch.empty((cams, C, H, W), device=dev),
                   t_final=torch.empty((cams, H, W), device=dev))
        if probs:
            out["probs"] = torch.empty((cams, C, H, W), device=dev)
        if ckpt_every > 0:
            nck = -(-march.n_samples // ckpt_every)
            out["ckpt"] = torch.empty((nck, R), device=dev)
        if stats:
            out["stats"] = torch.zeros(4, dtype=torch.int64, device=dev)
    g, p, r, m = grid.c(), prims.c(), rays.c(), march.c(ckpt_every)
    ix = index.c()
    t = (tuning or Tuning()).c()
    need = lib.sq_render_workspace(ct.byref(g), ct.byref(p), ct.byref(r), ct.byref(m))
    wbuf = ws.get(need) if ws is not None else _workspace(need, dev)
    L.check(lib.sq_render_fwd(ct.byref(g), ct.byref(ix), ct.byref(p), ct.byref(r), ct.byref(m),
                              _ptr(out["depth"]), _ptr(out["sem"]), _ptr(out.get("probs")), _ptr(out["t_final"]),
                              _ptr(out.get("ckpt")), _ptr(out.get("stats")), ct.byref(t), _ptr(wbuf),
                              wbuf.numel(), _stream_handle(stream)))
    return out


class StashPool:
    """The per-sample stash (sq_batch_io.stash) of the one-scene training
    path (render_train_fwd): sized on first use for a workload (scene shape,
    classes, march, tiling) by the slots its forward asks for, times
    `headroom`, and reused by later calls of that workload.  Chunks beyond
    the pool are recomputed by the backward, so a workload that grows stays
    correct."""

    def __init__(self, headroom: float = 1.25):
        self.headroom = float(headroom)
        self.buf: Optional[torch.Tensor] = None
        self.key = None

    def demand(self) -> int:
        """Slots the last forward asked for (synchronises)."""
        return 0 if self.buf is None else int(self.buf[:L.SQ_STASH_HEAD].view(torch.int32)[4].item())


def _one_scene_io(st, g_depth=None, g_sem=None, grads=None) -> L.SqBatchIO:
    io = L.SqBatchIO()
    p, r, ix = st["prims"], st["rays"], st["index"]
    for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
        setattr(io, k, _ptr(getattr(p, k)))
    io.origins, io.dirs = _ptr(r.origins), _ptr(r.dirs)
    io.counts, io.offsets, io.ids, io.totals = _ptr(ix.counts), _ptr(ix.offsets), _ptr(ix.ids), _ptr(ix.total)
    for k in ("depth", "sem", "t_final", "ckpt", "tile_stop"):
        setattr(io, k, _ptr(st[k]))
    io.tile_stop_len = int(st["tile_stop"].numel())
    io.ckpt_len = int(st["ckpt"].numel())
    pool = st["stash"]
    if pool is not None and pool.buf is not None:
        io.stash, io.stash_len = _ptr(pool.buf), int(pool.buf.numel())
    io.g_depth, io.g_sem = _ptr(g_depth), _ptr(g_sem)
    if grads is not None:
        for k, v in grads.items():
            setattr(io, "g_" + k, _ptr(v))
    return io


def render_train_fwd(grid, index: Index, prims: Prims, rays: Rays, march, ckpt_every: int = 8,
                     tuning: Optional[Tuning] = None, stash: Optional[StashPool] = None, stream=None) -> dict:
    """The differentiable forward of one scene through the batched ABI, on the
    caller's tensors (no copies): depth [cams,H,W], sem [cams,C,H,W], t_final,
    the checkpoints and the per-tile stops, and with a StashPool the
    per-sample stash.  Returns the state render_train_bwd takes."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    t = (tuning or Tuning()).c()
    b = L.SqBatch()
    b.n_scenes, b.n_classes = 1, prims.n_classes
    b.grid, b.march = grid.c(), march.c(ckpt_every)
    cams, H, W = rays.shape
    C, R = prims.n_classes, cams * H * W
    sc = b.scenes[0]
    sc.n_prims, sc.n_cams, sc.height, sc.width, sc.index_capacity = prims.n, cams, H, W, index.capacity
    nck = -(-march.n_samples // ckpt_every)
    st = dict(batch=b, tuning=t, index=index, prims=prims, rays=rays, stash=stash,
              depth=torch.empty((cams, H, W), device=dev), sem=torch.empty((cams, C, H, W), device=dev),
              t_final=torch.empty((cams, H, W), device=dev), ckpt=torch.empty((nck, R), device=dev),
              tile_stop=torch.empty(int(lib.sq_batch_tile_stop_len(ct.byref(b), ct.byref(t))), dtype=torch.int32,
                                    device=dev),
              ws=_workspace(lib.sq_batch_workspace(ct.byref(b)), dev), stream=stream)

    def run():
        L.check(lib.sq_batch_render_fwd(ct.byref(b), ct.byref(_one_scene_io(st)), None, ct.byref(t),
                                        _ptr(st["ws"]), st["ws"].numel(), _stream_handle(stream)))

    if stash is not None:
        key = (cams, H, W, C, march.n_samples, ckpt_every, t.tile_w)
        if stash.buf is None or stash.key != key:
            # size the pool: a forward against the header and slot table alone counts the slots
            n0 = int(lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), 0))
            if n0 <= 0:
                raise ValueError("no stash layout for this call (chunk must be 4, 8 or 16)")
            stash.buf, stash.key = torch.zeros(n0, dtype=torch.float32, device=dev), key
            run()
            slots = int(stash.demand() * stash.headroom) + 16
            stash.buf = torch.zeros(int(lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), slots)),
                                    dtype=torch.float32, device=dev)
    run()
    return st


def render_train_bwd(st: dict, g_depth: Optional[torch.Tensor], g_sem: Optional[torch.Tensor]) -> dict:
    """The backward of render_train_fwd's render (same checkpoints, stops and
    stash): gradients of sum(g_depth*depth) + sum(g_sem*sem) w.r.t. the
    primitives."""
    lib = L.load()
    prims = st["prims"]
    out = {k: torch.empty_like(getattr(prims, k)) for k in ("means", "quats", "scales", "eps", "opacity", "logits")}
    gd = None if g_depth is None else _f32(g_depth, "g_depth")
    gs = None if g_sem is None else _f32(g_sem, "g_sem")
    L.check(lib.sq_batch_render_bwd(ct.byref(st["batch"]), ct.byref(_one_scene_io(st, gd, gs, out)), None,
                                    ct.byref(st["tuning"]), _ptr(st["ws"]), st["ws"].numel(),
                                    _stream_handle(st["stream"])))
    return out


def render_fwd_noalloc(grid, index: Index, prims: Prims, rays: Rays, march, ckpt_every: int = 0,
                       probs: bool = True, tuning: Optional[Tuning] = None, stream=None,
                       out: Optional[dict] = None) -> dict:
    """sq_render_fwd_noalloc: sq_render_fwd with its scratch in the library's
    fixed per-GPU array (no workspace).  The library allocates nothing; this
    binding allocates the outputs unless `out` (same keys as render_fwd's)
    is given."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    cams, H, W = rays.shape
    C = prims.n_classes
    R = cams * H * W
    if out is None:
        out = dict(depth=torch.empty((cams, H, W), device=dev), sem=torch.empty((cams, C, H, W), device=dev),
                   t_final=torch.empty((cams, H, W), device=dev))
        if probs:
            out["probs"] = torch.empty((cams, C, H, W), device=dev)
        if ckpt_every > 0:
            out["ckpt"] = torch.empty((-(-march.n_samples // ckpt_every), R), device=dev)
    g, p, r, m = grid.c(), prims.c(), rays.c(), march.c(ckpt_every)
    ix = index.c()
    t = (tuning or Tuning()).c()
    L.check(lib.sq_render_fwd_noalloc(ct.byref(g), ct.byref(ix), ct.byref(p), ct.byref(r), ct.byref(m),
                                      _ptr(out["depth"]), _ptr(out["sem"]), _ptr(out.get("probs")),
                                      _ptr(out["t_final"]), _ptr(out.get("ckpt")), None, ct.byref(t),
                                      _stream_handle(stream)))
    return out


def render_bwd(grid, index: Index, prims: Prims, rays: Rays, march, ckpt: torch.Tensor, ckpt_every: int,
               g_depth: Optional[torch.Tensor], g_sem: Optional[torch.Tensor], tuning: Optional[Tuning] = None,
               stream=None, ws: Optional[Workspace] = None, out: Optional[dict] = None,
               stats: Optional[torch.Tensor] = None) -> dict:
    """sq_render_bwd: gradients of sum(g_depth*depth) + sum(g_sem*sem) w.r.t. the primitives.
    `stats` (6 int64 on the device, accumulated) selects the counting variant."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    if out is None:
        out = {name: torch.empty_like(getattr(prims, name))
               for name in ("means", "quats", "scales", "eps", "opacity", "logits")}
    gr = L.SqGrads(*(_ptr(out[name]) for name in ("means", "quats", "scales", "eps", "opacity", "logits")))
    g, p, r, m = grid.c(), prims.c(), rays.c(), march.c(ckpt_every)
    ix = index.c()
    t = (tuning or Tuning()).c()
    need = lib.sq_render_workspace(ct.byref(g), ct.byref(p), ct.byref(r), ct.byref(m))
    wbuf = ws.get(need) if ws is not None else _workspace(need, dev)
    gd = None if g_depth is None else _f32(g_depth, "g_depth")
    gs = None if g_sem is None else _f32(g_sem, "g_sem")
    L.check(lib.sq_render_bwd(ct.byref(g), ct.byref(ix), ct.byref(p), ct.byref(r), ct.byref(m),
                              _ptr(ckpt), _ptr(gd), _ptr(gs), ct.byref(gr), _ptr(stats), ct.byref(t), _ptr(wbuf),
                              wbuf.numel(), _stream_handle(stream)))
    return out


def render_bwd_sq_major(grid, index: Index, prims: Prims, rays: Rays, march, ckpt: torch.Tensor, ckpt_every: int,
                        g_depth: Optional[torch.Tensor], g_sem: Optional[torch.Tensor], capacity: int,
                        tuning: Optional[Tuning] = None, stream=None, iws: Optional[torch.Tensor] = None,
                        out: Optional[dict] = None) -> dict:
    """sq_render_bwd_sq_major: the superquadric-major backward (interactions
    grouped by primitive).  Returns the gradients and `interactions` (device
    int64: the number of interactions; results are valid when it is <=
    capacity)."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    if out is None:
        out = {name: torch.empty_like(getattr(prims, name))
               for name in ("means", "quats", "scales", "eps", "opacity", "logits")}
    out["interactions"] = torch.zeros(1, dtype=torch.int64, device=dev)
    gr = L.SqGrads(*(_ptr(out[name]) for name in ("means", "quats", "scales", "eps", "opacity", "logits")))
    g, p, r, m = grid.c(), prims.c(), rays.c(), march.c(ckpt_every)
    ix = index.c()
    t = (tuning or Tuning()).c()
    need = lib.sq_render_workspace(ct.byref(g), ct.byref(p), ct.byref(r), ct.byref(m))
    wbuf = _workspace(need, dev)
    ineed = lib.sq_sq_major_workspace(ct.byref(g), ct.byref(p), ct.byref(r), ct.byref(m), int(capacity))
    if iws is None or iws.numel() < ineed:
        iws = _workspace(ineed, dev)
    gd = None if g_depth is None else _f32(g_depth, "g_depth")
    gs = None if g_sem is None else _f32(g_sem, "g_sem")
    L.check(lib.sq_render_bwd_sq_major(ct.byref(g), ct.byref(ix), ct.byref(p), ct.byref(r), ct.byref(m),
                                       _ptr(ckpt), _ptr(gd), _ptr(gs), ct.byref(gr), int(capacity),
                                       _ptr(out["interactions"]), _ptr(iws), iws.numel(), ct.byref(t), _ptr(wbuf),
                                       wbuf.numel(), _stream_handle(stream)))
    return out


BWD_STAT_NAMES = ("samples1", "listed1", "eval1", "samples2", "listed2", "eval2")


def render_bwd_stats(grid, index: Index, prims: Prims, rays: Rays, march, ckpt, ckpt_every, g_depth, g_sem,
                     tuning: Optional[Tuning] = None, stream=None, ws: Optional[Workspace] = None) -> dict:
    """Unit counts of the backward (counting variant of sq_render_bwd)."""
    st = torch.zeros(6, dtype=torch.int64, device=prims.means.device)
    render_bwd(grid, index, prims, rays, march, ckpt, ckpt_every, g_depth, g_sem, tuning=tuning, stream=stream,
               ws=ws, stats=st)
    vals = st.cpu().tolist()
    return dict(zip(BWD_STAT_NAMES, vals))


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------

_IO_FIELDS = ("means", "quats", "scales", "eps", "opacity", "logits", "origins", "dirs", "counts", "offsets", "ids",
              "totals", "depth", "sem", "probs", "t_final", "ckpt", "g_depth", "g_sem", "g_means", "g_quats",
              "g_scales", "g_eps", "g_opacity", "g_logits", "vox_density", "vox_sem", "vox_labels", "sem_label",
              "depth_label", "loss", "tile_stop", "stash")

# Loss weights of the paper (Supplement "Loss Formulation"): lambda_s = 2, lambda_d = 0.05.
PAPER_LOSS = (2.0, 0.05)


def _weights(loss) -> L.SqLossWeights:
    w = L.SqLossWeights()
    w.lambda_sem, w.lambda_depth = (float(loss[0]), float(loss[1]))
    return w


def _fwd_outputs(grid, prims, rays, march, ckpt_every, probs):
    dev = prims.means.device
    cams, H, W = rays.shape
    C = prims.n_classes
    out = dict(depth=torch.empty((cams, H, W), device=dev), sem=torch.empty((cams, C, H, W), device=dev),
               t_final=torch.empty((cams, H, W), device=dev), g_depth=torch.empty((cams, H, W), device=dev),
               g_sem=torch.empty((cams, C, H, W), device=dev), loss=torch.zeros(3, device=dev))
    if probs:
        out["probs"] = torch.empty((cams, C, H, W), device=dev)
    if ckpt_every > 0:
        out["ckpt"] = torch.empty((-(-march.n_samples // ckpt_every), cams * H * W), device=dev)
    return out


def render_fwd_loss(grid, index: Index, prims: Prims, rays: Rays, march, sem_label: torch.Tensor,
                    depth_label: torch.Tensor, loss=PAPER_LOSS, ckpt_every: int = 0, probs: bool = True,
                    tuning: Optional[Tuning] = None, stream=None, ws: Optional[Workspace] = None,
                    out: Optional[dict] = None) -> dict:
    """sq_render_fwd_loss: render_fwd plus the fused loss of Eq. eq:loss.
    sem_label int32 [cams,H,W] (outside [0,C) = no label), depth_label
    [cams,H,W] (> 0 = labelled).  Adds g_depth, g_sem (the upstream gradients
    for render_bwd) and loss (3 floats: total, semantic, depth) to the outputs."""
    lib = L.load()
    grid, march = Grid.of(grid), March.of(march)
    dev = prims.means.device
    cams, H, W = rays.shape
    C = prims.n_classes
    if out is None:
        out = _fwd_outputs(grid, prims, rays, march, ckpt_every, probs)
    if sem_label.dtype != torch.int32 or not sem_label.is_contiguous():
        raise ValueError("sem_label must be contiguous int32")
    depth_label = _f32(depth_label, "depth_label")
    g, p, r, m = grid.c(), prims.c(), rays.c(), march.c(ckpt_every)
    ix = index.c()
    t = (tuning or Tuning()).c()
    w = _weights(loss)
    need = lib.sq_render_workspace(ct.byref(g), ct.byref(p), ct.byref(r), ct.byref(m))
    wbuf = ws.get(need) if ws is not None else _workspace(need, dev)
    L.check(lib.sq_render_fwd_loss(ct.byref(g), ct.byref(ix), ct.byref(p), ct.byref(r), ct.byref(m), ct.byref(w),
                                   _ptr(sem_label), _ptr(depth_label), _ptr(out["depth"]), _ptr(out["sem"]),
                                   _ptr(out.get("probs")), _ptr(out["t_final"]), _ptr(out.get("ckpt")),
                                   _ptr(out["g_depth"]), _ptr(out["g_sem"]), _ptr(out["loss"]), ct.byref(t),
                                   _ptr(wbuf), wbuf.numel(), _stream_handle(stream)))
    return out


def voxelise(grid, index: Index, prims: Prims, tau: float = 0.05, sem: bool = True, labels: bool = True,
             stream=None, ws: Optional[Workspace] = None, out: Optional[dict] = None) -> dict:
    """sq_voxelise (Eq. eq:voxelisation).  Returns density [X,Y,Z], sem
    [C,X,Y,Z] and labels [X,Y,Z] (int32, n_classes = free) on the device."""
    lib = L.load()
    grid = Grid.of(grid)
    dev = prims.means.device
    X, Y, Z = grid.dims
    C = prims.n_classes
    if out is None:
        out = dict(density=torch.empty((X, Y, Z), device=dev))
        if sem:
            out["sem"] = torch.empty((C, X, Y, Z), device=dev)
        if labels:
            out["labels"] = torch.empty((X, Y, Z), dtype=torch.int32, device=dev)
    g, p, ix = grid.c(), prims.c(), index.c()
    need = lib.sq_voxelise_workspace(ct.byref(g), ct.byref(p))
    wbuf = ws.get(need) if ws is not None else _workspace(need, dev)
    L.check(lib.sq_voxelise(ct.byref(g), ct.byref(ix), ct.byref(p), ct.c_float(tau), _ptr(out["density"]),
                            _ptr(out.get("sem")), _ptr(out.get("labels")), _ptr(wbuf), wbuf.numel(),
                            _stream_handle(stream)))
    return out


class Batch:
    """Several scenes sharing one grid, march and class count, concatenated
    scene-major in device memory (the layout of sq_batch_io in include/sqr.h).

    Owns every device buffer of a training step (inputs, index, outputs,
    checkpoints, upstream and parameter gradients) and one workspace, so a
    captured step graph stays valid for the lifetime of the object."""

    def __init__(self, grid, march, scenes, device="cuda", min_chunk: int = 4, probs: bool = True):
        """scenes: list of (Prims, Rays) with device tensors; march.ckpt_every is
        the default chunk (4, 8 or 16)."""
        lib = L.load()
        self.grid, self.march = Grid.of(grid), March.of(march)
        if not 1 <= len(scenes) <= L.SQ_MAX_SCENES:
            raise ValueError("1..32 scenes")
        C = scenes[0][0].n_classes
        if any(p.n_classes != C for p, _ in scenes):
            raise ValueError("all scenes need the same class count")
        self.n_classes = C
        self.device = device
        b = L.SqBatch()
        b.n_scenes = len(scenes)
        b.n_classes = C
        b.grid = self.grid.c()
        b.march = self.march.c()
        self.caps = []
        for i, (p, r) in enumerate(scenes):
            cams, H, W = r.shape
            cap = capacity_bound(self.grid, p.n)
            self.caps.append(cap)
            b.scenes[i].n_prims = p.n
            b.scenes[i].n_cams, b.scenes[i].height, b.scenes[i].width = cams, H, W
            b.scenes[i].index_capacity = cap
        self.c_batch = b
        self.scene_shapes = [(p.n,) + tuple(r.shape) for p, r in scenes]
        cat = lambda ts: torch.cat([t.reshape(-1) for t in ts]).contiguous()
        self.prims = Prims(*(cat([getattr(p, k) for p, _ in scenes]).view(-1, *getattr(scenes[0][0], k).shape[1:])
                             for k in ("means", "quats", "scales", "eps", "opacity", "logits")))
        self.origins = cat([r.origins for _, r in scenes]).view(-1, 3)
        self.dirs = cat([r.dirs for _, r in scenes]).view(-1, 3)
        R = self.origins.shape[0]
        V = self.grid.n_voxels
        S = len(scenes)
        nck = -(-self.march.n_samples // min_chunk)
        z = lambda *shape, dt=torch.float32: torch.zeros(shape, dtype=dt, device=device)
        self.buf = dict(counts=z(S * V, dt=torch.int32), offsets=z(S * V, dt=torch.int32),
                        ids=z(max(sum(self.caps), 1), dt=torch.int32), totals=z(S, dt=torch.int64),
                        depth=z(R), sem=z(R * C), probs=z(R * C) if probs else None, t_final=z(R), ckpt=z(nck * R),
                        g_depth=z(R), g_sem=z(R * C))
        for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
            self.buf["g_" + k] = torch.zeros_like(getattr(self.prims, k))
        # where each ray tile's forward stopped, sized for every tile width
        n_stop = max(int(lib.sq_batch_tile_stop_len(ct.byref(b), ct.byref(Tuning(tile_w=tw).c())))
                     for tw in (4, 8, 16))
        self.buf["tile_stop"] = torch.zeros(n_stop, dtype=torch.int32, device=device)
        self.ws = _workspace(lib.sq_batch_workspace(ct.byref(b)), device)
        self.graph = None

    @property
    def n_rays(self) -> int:
        return int(self.origins.shape[0])

    def io(self) -> L.SqBatchIO:
        io = L.SqBatchIO()
        vals = dict(self.buf)
        for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
            vals[k] = getattr(self.prims, k)
        vals["origins"], vals["dirs"] = self.origins, self.dirs
        for name in _IO_FIELDS:
            setattr(io, name, _ptr(vals.get(name)))
        if vals.get("tile_stop") is not None:
            io.tile_stop_len = int(vals["tile_stop"].numel())
        if vals.get("ckpt") is not None:
            io.ckpt_len = int(vals["ckpt"].numel())
        if vals.get("stash") is not None:
            io.stash_len = int(vals["stash"].numel())
        return io

    def set_stash(self, slots: Optional[int], tuning: Optional[Tuning] = None):
        """Give the batch a per-sample stash (sq_batch_io.stash) whose pool
        holds `slots` slots for `tuning` (its tile width and chunk), or, with
        no tuning, at least `slots` for every tile width and primitive-major
        chunk (4 or 8); 0 keeps only the header and slot table, which still
        count the slots a forward asks for (stash_demand); None removes it.  A
        captured graph keeps the buffer it was captured with: capture again."""
        self.release_graph()
        if slots is None:
            self.buf.pop("stash", None)
            return
        lib = L.load()
        tunings = [tuning] if tuning is not None else [Tuning(tile_w=tw, chunk=k) for tw in (4, 8, 16) for k in (4, 8)]
        n = max(int(lib.sq_batch_stash_len(ct.byref(self.c_batch), ct.byref(t.c()), int(slots))) for t in tunings)
        if n <= 0:
            raise ValueError(f"no stash layout for {slots} slots")
        self.buf["stash"] = torch.zeros(n, dtype=torch.float32, device=self.device)

    def stash_demand(self) -> int:
        """Slots the last forward with checkpoints asked for (one per chunk a
        ray tile entered); reads the device, so it synchronises."""
        st = self.buf.get("stash")
        return 0 if st is None else int(st[:L.SQ_STASH_HEAD].view(torch.int32)[4].item())

    def _call(self, fn, *args):
        L.check(fn(ct.byref(self.c_batch), ct.byref(self.io()), *args))

    def build_index(self, stream=None):
        lib = L.load()
        self._call(lib.sq_batch_build_index, _ptr(self.ws), self.ws.numel(), _stream_handle(stream))

    def render_fwd(self, tuning: Optional[Tuning] = None, stats=None, stream=None):
        lib = L.load()
        t = (tuning or Tuning()).c()
        self._call(lib.sq_batch_render_fwd, _ptr(stats), ct.byref(t), _ptr(self.ws), self.ws.numel(),
                   _stream_handle(stream))

    def render_bwd(self, tuning: Optional[Tuning] = None, stats=None, stream=None):
        lib = L.load()
        t = (tuning or Tuning()).c()
        self._call(lib.sq_batch_render_bwd, _ptr(stats), ct.byref(t), _ptr(self.ws), self.ws.numel(),
                   _stream_handle(stream))

    def voxelise(self, tau: float = 0.05, stream=None):
        """sq_batch_voxelise into vox_density [S*V], vox_sem [S*C*V], vox_labels [S*V]."""
        lib = L.load()
        if self.buf.get("vox_density") is None:
            S, V, C = len(self.scene_shapes), self.grid.n_voxels, self.n_classes
            self.buf["vox_density"] = torch.zeros(S * V, device=self.device)
            self.buf["vox_sem"] = torch.zeros(S * C * V, device=self.device)
            self.buf["vox_labels"] = torch.zeros(S * V, dtype=torch.int32, device=self.device)
        self._call(lib.sq_batch_voxelise, ct.c_float(tau), _ptr(self.ws), self.ws.numel(), _stream_handle(stream))

    def scene_voxels(self, i):
        """Scene i's voxelisation outputs shaped [X,Y,Z] / [C,X,Y,Z]."""
        V, C = self.grid.n_voxels, self.n_classes
        X, Y, Z = self.grid.dims
        return dict(density=self.buf["vox_density"][i * V:(i + 1) * V].view(X, Y, Z),
                    sem=self.buf["vox_sem"][i * C * V:(i + 1) * C * V].view(C, X, Y, Z),
                    labels=self.buf["vox_labels"][i * V:(i + 1) * V].view(X, Y, Z))

    def set_kappa(self, kappa: float):
        """Early ray termination threshold of later calls (captured graphs keep theirs)."""
        self.march = dataclasses.replace(self.march, kappa=float(kappa))
        self.c_batch.march.kappa = float(kappa)

    def set_labels(self, i, sem_label, depth_label):
        """Scene i's pseudo-labels for the fused loss: sem_label int32 and
        depth_label float, each [cams, H, W]."""
        if self.buf.get("sem_label") is None:
            R = self.n_rays
            self.buf["sem_label"] = torch.full((R,), -1, dtype=torch.int32, device=self.device)
            self.buf["depth_label"] = torch.zeros(R, device=self.device)
            self.buf["loss"] = torch.zeros(3, device=self.device)
        n0, n, r0, cams, H, W = self.scene_slices(i)
        R = cams * H * W
        self.buf["sem_label"][r0:r0 + R] = sem_label.reshape(-1).to(torch.int32)
        self.buf["depth_label"][r0:r0 + R] = depth_label.reshape(-1)

    def render_fwd_loss(self, loss=PAPER_LOSS, tuning: Optional[Tuning] = None, stream=None):
        lib = L.load()
        t = (tuning or Tuning()).c()
        self._call(lib.sq_batch_render_fwd_loss, ct.byref(_weights(loss)), ct.byref(t), _ptr(self.ws),
                   self.ws.numel(), _stream_handle(stream))

    def train_step(self, loss=PAPER_LOSS, tuning: Optional[Tuning] = None, stream=None):
        lib = L.load()
        t = (tuning or Tuning()).c()
        self._call(lib.sq_batch_train_step, ct.byref(_weights(loss)), ct.byref(t), _ptr(self.ws),
                   self.ws.numel(), _stream_handle(stream))

    def step(self, tuning: Optional[Tuning] = None, stream=None):
        lib = L.load()
        t = (tuning or Tuning()).c()
        self._call(lib.sq_batch_step, ct.byref(t), _ptr(self.ws), self.ws.numel(), _stream_handle(stream))

    def capture(self, tuning: Optional[Tuning] = None, stream=None, loss=None):
        """Capture one step into a hipGraph on `stream` (a non-default torch
        stream); with `loss` weights, the training step with the fused loss."""
        lib = L.load()
        self.release_graph()
        t = (tuning or Tuning()).c()
        h = ct.c_void_p()
        stream = stream or torch.cuda.Stream(device=self.device)
        if loss is None:
            L.check(lib.sq_batch_step_graph_create(ct.byref(self.c_batch), ct.byref(self.io()), ct.byref(t),
                                                   _ptr(self.ws), self.ws.numel(), _stream_handle(stream),
                                                   ct.byref(h)))
        else:
            L.check(lib.sq_batch_train_graph_create(ct.byref(self.c_batch), ct.byref(self.io()),
                                                    ct.byref(_weights(loss)), ct.byref(t), _ptr(self.ws),
                                                    self.ws.numel(), _stream_handle(stream), ct.byref(h)))
        self.graph = h
        self.graph_stream = stream
        return stream

    def replay(self, stream=None):
        lib = L.load()
        if self.graph is None:
            raise RuntimeError("no captured graph")
        L.check(lib.sq_graph_launch(self.graph, _stream_handle(stream or self.graph_stream)))

    def release_graph(self):
        if getattr(self, "graph", None) is not None:
            L.load().sq_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.release_graph()
        except Exception:
            pass

    def autotune(self, candidates, reps: int = 2, stream=None):
        """Time a step for every candidate Tuning; returns (best Tuning, ms list). Synchronous."""
        lib = L.load()
        n = len(candidates)
        arr = (L.SqTuning * n)(*[c.c() for c in candidates])
        best = ct.c_int32(-1)
        ms = (ct.c_float * n)()
        L.check(lib.sq_batch_autotune(ct.byref(self.c_batch), ct.byref(self.io()), arr, n, int(reps),
                                      ct.byref(best), ms, _ptr(self.ws), self.ws.numel(), _stream_handle(stream)))
        return candidates[best.value], list(ms)

    def autotune_cached(self, candidates, cache_path, reps: int = 2, stream=None):
        """sq_batch_autotune_cached: the tuning stored under this batch's key in
        cache_path, else the fastest candidate (timed, then appended to the
        file).  Returns (best Tuning, from_cache)."""
        lib = L.load()
        n = len(candidates)
        arr = (L.SqTuning * n)(*[c.c() for c in candidates])
        best = L.SqTuning()
        hit = ct.c_int32(0)
        path = None if cache_path is None else os.fsencode(cache_path)
        L.check(lib.sq_batch_autotune_cached(ct.byref(self.c_batch), ct.byref(self.io()), arr, n, int(reps), path,
                                             ct.byref(best), ct.byref(hit), _ptr(self.ws), self.ws.numel(),
                                             _stream_handle(stream)))
        return Tuning(best.tile_w, best.waves_per_block, best.bwd_mode, best.persistent, best.chunk), bool(hit.value)

    def tuning_key(self) -> str:
        """The autotune cache key of this batch on the current device."""
        lib = L.load()
        n = lib.sq_batch_tuning_key(ct.byref(self.c_batch), None, 0)
        buf = ct.create_string_buffer(n + 1)
        lib.sq_batch_tuning_key(ct.byref(self.c_batch), buf, n + 1)
        return buf.value.decode()

    # ---- views of one scene's slice of the concatenated outputs ----
    def scene_slices(self, i):
        n_before = sum(s[0] for s in self.scene_shapes[:i])
        r_before = sum(s[1] * s[2] * s[3] for s in self.scene_shapes[:i])
        n, cams, H, W = self.scene_shapes[i]
        return n_before, n, r_before, cams, H, W

    def scene_outputs(self, i):
        n0, n, r0, cams, H, W = self.scene_slices(i)
        R = cams * H * W
        C = self.n_classes
        out = dict(depth=self.buf["depth"][r0:r0 + R].view(cams, H, W),
                   t_final=self.buf["t_final"][r0:r0 + R].view(cams, H, W),
                   sem=self.buf["sem"][r0 * C:(r0 + R) * C].view(cams, C, H, W))
        if self.buf.get("probs") is not None:
            out["probs"] = self.buf["probs"][r0 * C:(r0 + R) * C].view(cams, C, H, W)
        for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
            out["g_" + k] = self.buf["g_" + k][n0:n0 + n]
        return out

    def set_upstream(self, i, g_depth, g_sem):
        n0, n, r0, cams, H, W = self.scene_slices(i)
        R = cams * H * W
        C = self.n_classes
        self.buf["g_depth"][r0:r0 + R] = g_depth.reshape(-1)
        self.buf["g_sem"][r0 * C:(r0 + R) * C] = g_sem.reshape(-1)


def default_candidates():
    """Tile width x waves per block x chunk x persistent waves."""
    out = []
    for tw in (8, 16, 4):
        for wpb in (4, 2):
            for chunk in (4, 8):
                for pers in (0, 1):
                    out.append(Tuning(tile_w=tw, waves_per_block=wpb, chunk=chunk, persistent=pers))
    return out

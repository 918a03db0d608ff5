"""Torch-facing binding of the renderer's C ABI.

PyTorch only provides device memory (tensors) and the current HIP stream;
every step of the method runs in libsqr.so.  Each function below fills the
ctypes structs of include/sqr.h from tensors, allocates outputs and the
workspace with torch, and calls one C entry point.
"""
from __future__ import annotations

import ctypes as ct
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

    def c(self) -> L.SqGrid:
        g = L.SqGrid()
        for i in range(3):
            g.lo[i] = float(self.lo[i])
            g.dims[i] = int(self.dims[i])
        g.voxel = float(self.voxel)
        g.nv = int(self.nv)
        return g

    @property
    def n_voxels(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    @staticmethod
    def of(obj) -> "Grid":
        return obj if isinstance(obj, Grid) else Grid(tuple(obj.lo), float(obj.voxel), tuple(obj.dims), int(obj.nv))


@dataclass
class March:
    n_samples: int
    t_near: float
    t_far: float
    ckpt_every: int = 0

    def c(self, ckpt_every: Optional[int] = None) -> L.SqMarch:
        m = L.SqMarch()
        m.n_samples = int(self.n_samples)
        m.t_near = float(self.t_near)
        m.t_far = float(self.t_far)
        m.ckpt_every = int(self.ckpt_every if ckpt_every is None else ckpt_every)
        return m

    @staticmethod
    def of(obj) -> "March":
        return obj if isinstance(obj, March) else March(int(obj.n_samples), float(obj.t_near), float(obj.t_far),
                                                        int(getattr(obj, "ckpt_every", 0)))


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

    def c(self) -> L.SqTuning:
        t = L.SqTuning()
        t.tile_w = int(self.tile_w)
        t.waves_per_block = int(self.waves_per_block)
        t.bwd_mode = int(self.bwd_mode)
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


BWD_STAT_NAMES = ("samples1", "listed1", "eval1", "samples2", "listed2", "eval2")


def render_bwd_stats(grid, index: Index, prims: Prims, rays: Rays, march, ckpt, ckpt_every, g_depth, g_sem,
                     tuning: Optional[Tuning] = None, stream=None, ws: Optional[Workspace] = None) -> dict:
    """Unit counts of the backward (counting variant of sq_render_bwd)."""
    st = torch.zeros(6, dtype=torch.int64, device=prims.means.device)
    render_bwd(grid, index, prims, rays, march, ckpt, ckpt_every, g_depth, g_sem, tuning=tuning, stream=stream,
               ws=ws, stats=st)
    vals = st.cpu().tolist()
    return dict(zip(BWD_STAT_NAMES, vals))

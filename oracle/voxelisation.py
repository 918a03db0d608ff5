"""FP64 oracle of superquadric voxelisation (Supplement "SuperQuadric
Voxelisation", Eq. eq:voxelisation).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For every voxel v with centre p the density and semantic voxels are the sums
over the superquadrics of the cubic neighbourhood N_v:
    v_d(p) = sum_i p_o(p, S_i) sigma_i,   v_s(p) = sum_i p_o(p, S_i) c_i,
and a voxel whose density is below tau is free in the semantic prediction.
The neighbourhood is the same one the renderer's index uses (reading R4): S_i
takes part at voxel v exactly when v lies in the clipped cube of half-width
N_v around the voxel containing m_i, i.e. when i is listed in V_sq(v).

Readings (listed with the others in the design notes):
R18 Voxel centres are float32, per axis p = fl(lo + fl(fl(i + 0.5) * voxel))
    (each op correctly rounded, no FMA); the evaluation downstream is FP64.
R19 The final prediction is the class index argmax_c v_s (first maximum)
    where v_d >= tau, and the label n_classes ("free") where v_d < tau.
"""
from __future__ import annotations

import numpy as np

from .sqr_oracle import F32, _eval_pairs, _Prep, build_index, centre_boxes, influence_boxes

__all__ = ["voxel_centres", "voxelise", "labels_from"]


def voxel_centres(grid):
    """Per-axis FP32 voxel centres (reading R18): three arrays of length dims[a]."""
    out = []
    for a in range(3):
        i = np.arange(grid.dims[a]).astype(F32)
        half = (i + F32(0.5)).astype(F32)
        out.append((F32(grid.lo[a]) + (half * F32(grid.voxel)).astype(F32)).astype(F32))
    return out


def _voxel_coords(grid, v):
    Y, Z = grid.dims[1], grid.dims[2]
    return v // (Y * Z), (v // Z) % Y, v % Z


def labels_from(density, sem, tau):
    """Reading R19: class argmax (first maximum) where density >= tau, else C."""
    C = sem.shape[-1]
    lab = np.argmax(sem, axis=-1).astype(np.int64)
    return np.where(density < tau, C, lab)


def voxelise(grid, prims, index=None, brute=False, tau=0.05, voxel_ids=None, chunk=1 << 20):
    """Density, semantic voxels and labels (Eq. eq:voxelisation).

    Returns FP64 density [V], sem [V, C] and int64 labels [V] (V = voxels of the
    grid, linear id (ix*Y + iy)*Z + iz), or, with `voxel_ids`, the same for
    those voxels only.  `brute` takes the neighbourhood from the boxes directly
    instead of the index lists."""
    P = _Prep(prims)
    n_vox = int(np.prod(grid.dims))
    vids = np.arange(n_vox) if voxel_ids is None else np.asarray(voxel_ids, np.int64)
    C = prims.logits.shape[1]
    cx, cy, cz = voxel_centres(grid)
    ix, iy, iz = _voxel_coords(grid, vids)
    centre = np.stack([cx[ix], cy[iy], cz[iz]], axis=1).astype(np.float64)

    if brute:
        blo, bhi = influence_boxes(prims, grid)
        vi = np.stack([ix, iy, iz], axis=1)
        inside = np.all((vi[:, None, :] >= blo[None]) & (vi[:, None, :] <= bhi[None]), axis=2)
        pv, pk = np.nonzero(inside)                  # pairs (voxel row, primitive), ascending k per voxel
    else:
        counts, offsets, ids = (build_index(prims, grid)[:3] if index is None else index[:3])
        n = counts[vids].astype(np.int64)
        pv = np.repeat(np.arange(vids.size), n)
        start = np.repeat(offsets[vids].astype(np.int64), n)
        within = np.arange(pv.size) - np.repeat(np.cumsum(n) - n, n)
        pk = ids[start + within].astype(np.int64)

    density = np.zeros(vids.size)
    sem = np.zeros((vids.size, C))
    for s in range(0, pv.size, chunk):
        v, k = pv[s:s + chunk], pk[s:s + chunk]
        p, _, _ = _eval_pairs(P, centre[v], k)
        density += np.bincount(v, weights=p * P.sigma[k], minlength=vids.size)
        for c in range(C):
            sem[:, c] += np.bincount(v, weights=p * P.logits[k, c], minlength=vids.size)
    return dict(density=density, sem=sem, labels=labels_from(density, sem, tau))

"""FP64 CPU oracle for the superquadric volume renderer (SQOcc-R).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path (the two meet only in
the seeded input arrays of `synth`).

The renderer is exact by construction (no approximation beyond its own
definition), so this oracle is the plain definition written out, evaluated in
FP64 on FP32 inputs.  Section/equation names refer to the paper
(arXiv 2511.17361):

* "SuperQuadrics": primitive S = {m, s, r, eps, sigma, c}; the canonical
  inside-outside function f and the occupancy p_o = exp(-f(x_S)) with
  x_S = R(x - m)  (Eq. eq:sq_occupancy_prob).
* "Preliminary Construction": per-primitive cubic neighbourhood of half-width
  N_v, hashed into the per-voxel tensors V_sq, V_f, V_n; uniformly spaced ray
  samples x = o + t d in [t_near, t_far].
* "Forward Pass": skip samples outside the grid or with V_n = 0; per-sample
  alpha (upper-bounded by 1) and semantics (Eq. eq:alpha_sem_sq); front-to-back
  compositing (Eq. eq:alpha_composite); depth and semantic render
  (Eq. eq:depth_sem).
* "Backward Pass": gradients of the renders w.r.t. every primitive parameter.
  The oracle computes them with the plain reverse-mode chain rule of the
  equations above (no interaction sort, no tiling).

Readings where the paper is silent or ambiguous (all listed in the design
notes of the repository):

R1  |.| inside the fractional powers of f (signed-power convention of Barr).
R2  R = R(r/|r|), Hamilton convention, quaternion stored (w, x, y, z);
    x_S = R (x - m) taken literally.
R3  "Hashing" = dense linear voxel id v = (ix*Y + iy)*Z + iz.
R4  Neighbourhood of S_k = the cube of half-width N_v around the voxel that
    contains m_k, clipped to the grid.  Lists are ascending in primitive id.
R5  Samples: t_j = t_near + j*(t_far - t_near)/(L-1), endpoints included
    (t_0 = t_near when L = 1).  The sample depths and points are defined in
    FP32 by the op sequence below (each op correctly rounded, no FMA):
      delta = fl(fl(t_far - t_near) / fl(L - 1)),  t_j = fl(t_near + fl(j*delta)),
      x_j = fl(o + fl(t_j * d)),  i = floor(fl(fl(x_j - lo) * inv_vs)),
      inv_vs = fl(1/voxel).
    The same FP32 sequence gives each centre's voxel.  Every continuous
    quantity downstream of x_j, t_j is evaluated in FP64.
R6  Voxel cells are half-open; a point on a face belongs to the higher cell;
    the upper grid face is outside.
R7  alpha = min(1, a) with a = sum p*sigma; d alpha/d a = 0 where a >= 1.
R8  s_j = sum p*c (no sigma factor), as printed.
R9  Depth is range along the unit ray, no normalisation by sum(w); an empty
    ray renders depth 0, semantics 0, transmittance 1.
R10 "Class probabilities" = softmax over classes of the rendered semantic
    vector S_hat (max-subtracted).
R21 Influence threshold of the index (the Supplement's future work on
    occupancy-aware indexing): with theta > 0 a primitive is listed only in
    the voxels of its N_v cube that meet the world box of
    max(|u|,|v|,|w|) <= ln(sigma/theta)^(eps1/2), a box that holds every point
    where p_o sigma >= theta (see influence_boxes).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "pinned_inv_voxel", "sample_depths", "voxel_of_points", "centre_boxes", "influence_boxes",
    "build_index", "rotation_matrix", "inside_outside", "occupancy",
    "render", "render_grad", "box_volume_total", "pair_records",
]

F32 = np.float32


# ---------------------------------------------------------------------------
# FP32-pinned discrete decisions (reading R5)
# ---------------------------------------------------------------------------

def pinned_inv_voxel(voxel) -> np.float32:
    """inv_vs = fl32(1 / voxel)."""
    return F32(1.0) / F32(voxel)


def sample_depths(n_samples: int, t_near, t_far) -> np.ndarray:
    """t_j in FP32: delta = fl((t_far - t_near) / (L - 1)), t_j = fl(t_near + fl(j*delta)).

    "Preliminary Construction": L uniformly spaced samples in [t_near, t_far]."""
    tn, tf = F32(t_near), F32(t_far)
    if n_samples == 1:
        return np.array([tn], dtype=F32)
    delta = (tf - tn) / F32(n_samples - 1)
    j = np.arange(n_samples).astype(F32)
    return (tn + (j * delta)).astype(F32)


def voxel_of_points(x32: np.ndarray, grid):
    """Voxel of FP32 points [..., 3]: q = fl(fl(x - lo) * inv_vs); inside iff
    0 <= q < dims on every axis (reading R6); returns (inside, linear id)."""
    lo = np.asarray(grid.lo, dtype=F32)
    inv = pinned_inv_voxel(grid.voxel)
    q = ((x32.astype(F32) - lo) * inv).astype(F32)
    dims = np.asarray(grid.dims)
    inside = np.all((q >= 0) & (q < dims.astype(F32)), axis=-1)
    idx = np.floor(np.where(inside[..., None], q, 0)).astype(np.int64)
    v = (idx[..., 0] * dims[1] + idx[..., 1]) * dims[2] + idx[..., 2]
    return inside, v


def centre_boxes(means: np.ndarray, grid):
    """Clipped neighbourhood box of each primitive (reading R4).

    c_k = floor(fl(fl(m_k - lo) * inv_vs)) per axis; box = [c - N_v, c + N_v]
    intersected with [0, dims - 1].  Returns (lo[N,3], hi[N,3]) int64; a box is
    empty when lo > hi on some axis."""
    lo_g = np.asarray(grid.lo, dtype=F32)
    inv = pinned_inv_voxel(grid.voxel)
    q = ((means.astype(F32) - lo_g) * inv).astype(F32)
    dims = np.asarray(grid.dims, dtype=np.int64)
    nv = int(grid.nv)
    # bound the float before converting it; NaN centres cover nothing
    big = F32(max(int(dims.max()) + nv + 2, 4))
    q = np.fmin(np.fmax(q, -big), big)
    c = np.floor(q).astype(np.int64)
    blo = np.maximum(c - nv, 0)
    bhi = np.minimum(c + nv, dims - 1)
    return blo, bhi


def influence_boxes(prims, grid):
    """List region of each primitive under an influence threshold theta
    (reading R21; Supplement "Limitations and Future Work": keep a primitive
    out of the voxels where its occupancy times opacity stays below theta).

    f >= max(|u|,|v|,|w|)^(2/eps1), so p_o sigma >= theta implies
    max(|u|,|v|,|w|) <= r = ln(sigma/theta)^(eps1/2).  The world-space box of
    that canonical cube, x - m = R^T diag(s) u, has half-extent
    h_a = r (|R_0a| s_0 + |R_1a| s_1 + |R_2a| s_2).  The region is the N_v cube
    of R4 intersected with floor(((m_a -/+ h_a) - lo_a) / voxel) per axis, all
    in FP64 on the FP32 inputs; it is empty where sigma <= theta.  theta = 0
    (the default) is the N_v cube itself.  Returns (lo[N,3], hi[N,3]) int64."""
    blo, bhi = centre_boxes(prims.means, grid)
    theta = float(F32(getattr(grid, "theta", 0.0)))     # an FP32 parameter, as the kernels see it
    if not theta > 0.0:
        return blo, bhi
    q = np.asarray(prims.quats, np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    nrm = np.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / nrm, x / nrm, y / nrm, z / nrm
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    s = np.asarray(prims.scales, np.float64)
    e1 = np.asarray(prims.eps, np.float64)[:, 0]
    sig = np.asarray(prims.opacity, np.float64)
    live = sig > theta
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(live, np.exp(0.5 * e1 * np.log(np.log(np.where(live, sig, 1.0) / theta))), 0.0)
    h = r[:, None] * (np.abs(R[:, 0, :]) * s[:, 0:1] + np.abs(R[:, 1, :]) * s[:, 1:2] + np.abs(R[:, 2, :]) * s[:, 2:3])
    m = np.asarray(prims.means, np.float64)
    lo = np.asarray(grid.lo, F32).astype(np.float64)
    vs = float(F32(grid.voxel))
    slo = np.floor(((m - h) - lo) / vs)
    shi = np.floor(((m + h) - lo) / vs)
    big = float(max(int(np.max(grid.dims)) + int(grid.nv) + 2, 4))
    slo = np.clip(np.nan_to_num(slo, nan=big), -big, big).astype(np.int64)
    shi = np.clip(np.nan_to_num(shi, nan=-big), -big, big).astype(np.int64)
    tlo = np.maximum(blo, slo)
    thi = np.minimum(bhi, shi)
    thi[~live] = -1
    tlo[~live] = 0
    return tlo, thi


def box_volume_total(means, grid) -> int:
    """sum_k |box_k| (the number of index entries E)."""
    blo, bhi = centre_boxes(means, grid)
    ext = np.clip(bhi - blo + 1, 0, None)
    return int(np.prod(ext, axis=1).sum())


def build_index(prims, grid):
    """V_n, V_f, V_sq ("Preliminary Construction").

    Every primitive emits the (voxel, id) pairs of its clipped box (R4, and
    R21 when the grid carries an influence threshold theta > 0); the pairs are
    ordered by (voxel, id); V_n counts pairs per voxel and V_f is the exclusive
    prefix sum of V_n.  `prims` is a Prims, or just the [N,3] centres when
    theta = 0.  Returns (counts, offsets, ids) as int32 and the total E."""
    dims = tuple(int(d) for d in grid.dims)
    nvox = dims[0] * dims[1] * dims[2]
    if hasattr(prims, "means"):
        blo, bhi = influence_boxes(prims, grid)
        n = prims.n
    else:
        if float(getattr(grid, "theta", 0.0)) > 0.0:
            raise ValueError("an influence threshold needs the primitives, not only their centres")
        blo, bhi = centre_boxes(prims, grid)
        n = prims.shape[0]
    vox_parts, id_parts = [], []
    for k in range(n):
        if np.any(blo[k] > bhi[k]):
            continue
        ix = np.arange(blo[k, 0], bhi[k, 0] + 1)
        iy = np.arange(blo[k, 1], bhi[k, 1] + 1)
        iz = np.arange(blo[k, 2], bhi[k, 2] + 1)
        gx, gy, gz = np.meshgrid(ix, iy, iz, indexing="ij")
        v = ((gx * dims[1] + gy) * dims[2] + gz).ravel()
        vox_parts.append(v)
        id_parts.append(np.full(v.shape, k, dtype=np.int64))
    if vox_parts:
        vox = np.concatenate(vox_parts)
        ids = np.concatenate(id_parts)
        order = np.lexsort((ids, vox))   # primary key voxel, then id
        vox, ids = vox[order], ids[order]
    else:
        vox = np.zeros(0, np.int64)
        ids = np.zeros(0, np.int64)
    counts = np.bincount(vox, minlength=nvox).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(counts)[:-1]]) if nvox else np.zeros(0, np.int64)
    return (counts.astype(np.int32), offsets.astype(np.int32), ids.astype(np.int32), int(counts.sum()))


# ---------------------------------------------------------------------------
# Geometry (Sec. "SuperQuadrics")
# ---------------------------------------------------------------------------

def rotation_matrix(q: np.ndarray) -> np.ndarray:
    """R(q/|q|) for quaternions (w, x, y, z), Hamilton convention (reading R2)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _powabs(x, p):
    """|x|^p with |0|^p = 0 for p > 0 (guards of reading R1)."""
    return np.abs(x) ** p


def inside_outside(u, v, w, eps1, eps2):
    """Canonical f = ((|u|)^{2/e2} + (|v|)^{2/e2})^{e2/e1} + (|w|)^{2/e1} with
    (u, v, w) = x_S / s (Sec. "SuperQuadrics", unlabeled equation of f)."""
    a = 2.0 / eps2
    b = 2.0 / eps1
    e = eps2 / eps1
    A = _powabs(u, a) + _powabs(v, a)
    return A ** e + _powabs(w, b)


def local_coords(x: np.ndarray, means, R, scales):
    """x_S = R (x - m) and (u, v, w) = x_S / s for pairs (x[P,3], params[P,...])."""
    xs = np.einsum("pij,pj->pi", R, x - means)
    return xs, xs / scales


def occupancy(x: np.ndarray, means, quats, scales, eps) -> np.ndarray:
    """p_o(x, S) = exp(-f(x_S)) (Eq. eq:sq_occupancy_prob), pairwise over P."""
    R = rotation_matrix(quats)
    _, uvw = local_coords(np.asarray(x, np.float64), np.asarray(means, np.float64), R,
                          np.asarray(scales, np.float64))
    eps = np.asarray(eps, np.float64)
    f = inside_outside(uvw[:, 0], uvw[:, 1], uvw[:, 2], eps[:, 0], eps[:, 1])
    return np.exp(-f)


# ---------------------------------------------------------------------------
# Renderer (Sec. "Forward Pass")
# ---------------------------------------------------------------------------

def _pairs_for_sample(v, active, counts, offsets, ids, box_lo, box_hi, grid, brute):
    """Pair lists (ray index, primitive id) of one sample step, ascending id per ray.

    indexed: Q(v) = V_sq[V_f[v] : V_f[v] + V_n[v]];
    brute:   all primitives whose clipped box contains v (membership predicate)."""
    rays = np.nonzero(active)[0]
    if brute:
        dims = np.asarray(grid.dims)
        iz = v[rays] % dims[2]
        iy = (v[rays] // dims[2]) % dims[1]
        ix = v[rays] // (dims[2] * dims[1])
        vi = np.stack([ix, iy, iz], 1)                          # [B,3]
        mem = np.all((vi[:, None, :] >= box_lo[None]) & (vi[:, None, :] <= box_hi[None]), axis=2)
        r_idx, k = np.nonzero(mem)                              # row-major: ascending k per ray
        return rays[r_idx], k
    n = counts[v[rays]].astype(np.int64)
    keep = n > 0
    rays, n = rays[keep], n[keep]
    f = offsets[v[rays]].astype(np.int64)
    r_rep = np.repeat(rays, n)
    start = np.repeat(f, n)
    within = np.arange(n.sum()) - np.repeat(np.cumsum(n) - n, n)
    return r_rep, ids[start + within].astype(np.int64)


class _Prep:
    """FP64 per-primitive constants derived from the FP32 inputs."""

    def __init__(self, prims):
        self.means = prims.means.astype(np.float64)
        self.qraw = prims.quats.astype(np.float64)
        self.R = rotation_matrix(self.qraw)
        self.scales = prims.scales.astype(np.float64)
        self.eps = prims.eps.astype(np.float64)
        self.sigma = prims.opacity.astype(np.float64)
        self.logits = prims.logits.astype(np.float64)


def _eval_pairs(P: _Prep, x, k):
    """Per pair: p = exp(-f), and the intermediates the adjoint needs."""
    xs, uvw = local_coords(x, P.means[k], P.R[k], P.scales[k])
    e1, e2 = P.eps[k, 0], P.eps[k, 1]
    f = inside_outside(uvw[:, 0], uvw[:, 1], uvw[:, 2], e1, e2)
    return np.exp(-f), xs, uvw


def _march(grid, prims, rays_o, rays_d, march, index, brute, P, want_pairs):
    """Front-to-back march of a ray batch.  Returns per-ray depth, semantics
    and final transmittance, the per-sample/pair records the adjoint replays
    (if asked) and, with early termination, each ray's smallest relative
    distance |T_j / kappa - 1| over the transmittances it compared (inf without)."""
    B = rays_o.shape[0]
    C = prims.logits.shape[1]
    counts, offsets, ids = index if index is not None else (None, None, None)
    box_lo, box_hi = influence_boxes(prims, grid) if brute else (None, None)
    t32 = sample_depths(march.n_samples, march.t_near, march.t_far)
    kappa = float(getattr(march, "kappa", 0.0))
    T = np.ones(B)
    depth = np.zeros(B)
    sem = np.zeros((B, C))
    margin = np.full(B, np.inf)
    records = []
    for j, tj in enumerate(t32):
        x32 = (rays_o + (tj * rays_d).astype(F32)).astype(F32)       # pinned FP32 point
        inside, v = voxel_of_points(x32, grid)
        # rays with T == 0 contribute exactly zero from here on (T_{j+1} = 0 * ...);
        # early termination (Sec. "Ray Termination"): a ray stops once T < kappa
        if kappa > 0:
            margin = np.minimum(margin, np.abs(T / kappa - 1.0))
        active = inside & (T > 0) & (T >= kappa)
        r_rep, k = _pairs_for_sample(v, active, counts, offsets, ids, box_lo, box_hi, grid, brute)
        a = np.zeros(B)
        s = np.zeros((B, C))
        if r_rep.size:
            x = x32[r_rep].astype(np.float64)
            p, xs, uvw = _eval_pairs(P, x, k)
            np.add.at(a, r_rep, p * P.sigma[k])                     # Eq. eq:alpha_sem_sq
            np.add.at(s, r_rep, p[:, None] * P.logits[k])
        alpha = np.minimum(1.0, a)                                  # "upper-bounded by 1"
        w = T * alpha                                               # Eq. eq:alpha_composite
        depth += w * np.float64(tj)                                 # Eq. eq:depth_sem
        sem += w[:, None] * s
        if want_pairs:
            records.append(dict(t=np.float64(tj), a=a, alpha=alpha, T=T.copy(), w=w, s=s,
                                r=r_rep, k=k, x=(x32[r_rep].astype(np.float64) if r_rep.size else None)))
        T = T * (1.0 - alpha)
    if kappa > 0:
        margin = np.minimum(margin, np.abs(T / kappa - 1.0))
    return depth, sem, T, records, margin


def pair_records(grid, prims, rays, march, index=None, ray_ids=None):
    """Per-sample records of the front-to-back march ("Forward Pass"), for
    counting the method's units: one dict per sample index j with the FP32
    depth t, every ray's a_j and T_j, and the listed pairs of that sample as
    (r = ray index within the batch, k = primitive id, x = the pinned FP32
    sample point as FP64).  A sample contributes pairs only when its ray is
    still marching (T_j > 0, T_j >= kappa), its point lies in the grid and
    its voxel lists at least one primitive."""
    if index is None:
        index = build_index(prims, grid)[:3]
    P = _Prep(prims)
    o = rays.origins.reshape(-1, 3)
    d = rays.dirs.reshape(-1, 3)
    if ray_ids is not None:
        o, d = o[ray_ids], d[ray_ids]
    return _march(grid, prims, o, d, march, index, False, P, True)[3]


def _softmax(z):
    z = z - z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=-1, keepdims=True)


def _ray_batches(n_rays, batch):
    for s in range(0, n_rays, batch):
        yield s, min(n_rays, s + batch)


def render(grid, prims, rays, march, index=None, brute=False, ray_ids=None, batch=8192):
    """Depth, semantics, class probabilities and final transmittance.

    Returns FP64 arrays shaped like the rig: depth/t_final [cams,H,W],
    sem/probs [cams,C,H,W].  With `ray_ids` (flat ray indices) only those rays
    are rendered and the outputs are flat: depth [n], sem [n,C]."""
    if index is None and not brute:
        index = build_index(prims, grid)[:3]
    P = _Prep(prims)
    o = rays.origins.reshape(-1, 3)
    d = rays.dirs.reshape(-1, 3)
    if ray_ids is not None:
        o, d = o[ray_ids], d[ray_ids]
    n = o.shape[0]
    C = prims.logits.shape[1]
    depth = np.zeros(n)
    sem = np.zeros((n, C))
    tfin = np.zeros(n)
    margin = np.zeros(n)
    for s, e in _ray_batches(n, batch):
        dd, ss, tt, _, mm = _march(grid, prims, o[s:e], d[s:e], march, index, brute, P, False)
        depth[s:e], sem[s:e], tfin[s:e], margin[s:e] = dd, ss, tt, mm
    probs = _softmax(sem)
    if ray_ids is not None:
        return dict(depth=depth, sem=sem, probs=probs, t_final=tfin, kappa_margin=margin)
    cams, H, W = rays.shape
    return dict(depth=depth.reshape(cams, H, W),
                sem=sem.reshape(cams, H, W, C).transpose(0, 3, 1, 2).copy(),
                probs=probs.reshape(cams, H, W, C).transpose(0, 3, 1, 2).copy(),
                t_final=tfin.reshape(cams, H, W), kappa_margin=margin.reshape(cams, H, W))


# ---------------------------------------------------------------------------
# Adjoint (Sec. "Backward Pass"), plain reverse mode
# ---------------------------------------------------------------------------

def _drot_dq(qhat):
    """dR/dq_hat for unit quaternions [P,4] -> [P,3,3,4] (of the matrix of
    `rotation_matrix` before normalisation)."""
    w, x, y, z = qhat[:, 0], qhat[:, 1], qhat[:, 2], qhat[:, 3]
    Z0 = np.zeros_like(w)
    D = np.empty((qhat.shape[0], 3, 3, 4))
    D[:, 0, 0] = np.stack([Z0, Z0, -4 * y, -4 * z], 1)
    D[:, 0, 1] = np.stack([-2 * z, 2 * y, 2 * x, -2 * w], 1)
    D[:, 0, 2] = np.stack([2 * y, 2 * z, 2 * w, 2 * x], 1)
    D[:, 1, 0] = np.stack([2 * z, 2 * y, 2 * x, 2 * w], 1)
    D[:, 1, 1] = np.stack([Z0, -4 * x, Z0, -4 * z], 1)
    D[:, 1, 2] = np.stack([-2 * x, -2 * w, 2 * z, 2 * y], 1)
    D[:, 2, 0] = np.stack([-2 * y, 2 * z, -2 * w, 2 * x], 1)
    D[:, 2, 1] = np.stack([2 * x, 2 * w, 2 * z, 2 * y], 1)
    D[:, 2, 2] = np.stack([Z0, -4 * x, -4 * y, Z0], 1)
    return D


def _pair_param_grads(P: _Prep, x, k, dp):
    """Chain dL/dp of each pair through p = exp(-f(R(x - m) / s)) to
    (m, q, s, eps1, eps2); returns per-pair arrays."""
    m = P.means[k]
    R = P.R[k]
    s = P.scales[k]
    e1, e2 = P.eps[k, 0], P.eps[k, 1]
    d = x - m
    xs = np.einsum("pij,pj->pi", R, d)
    u = xs / s
    a, b, e = 2.0 / e2, 2.0 / e1, e2 / e1
    au = np.abs(u)
    X = au[:, 0] ** a
    Y = au[:, 1] ** a
    Zt = au[:, 2] ** b
    A = X + Y
    B = A ** e
    p = np.exp(-(B + Zt))
    df = -p * dp                                       # dL/df
    with np.errstate(divide="ignore", invalid="ignore"):
        BA = np.where(A > 0, B / A, 0.0)
        # df/du_i (sign-aware derivative of |u|^a), zero where u_i == 0
        dfu = np.where(u[:, 0] != 0, e * a * BA * X / u[:, 0], 0.0)
        dfv = np.where(u[:, 1] != 0, e * a * BA * Y / u[:, 1], 0.0)
        dfw = np.where(u[:, 2] != 0, b * Zt / u[:, 2], 0.0)
        lnA = np.where(A > 0, np.log(A), 0.0)
        Xl = np.where(X > 0, X * np.log(np.where(au[:, 0] > 0, au[:, 0], 1.0)), 0.0)
        Yl = np.where(Y > 0, Y * np.log(np.where(au[:, 1] > 0, au[:, 1], 1.0)), 0.0)
        Zl = np.where(Zt > 0, Zt * np.log(np.where(au[:, 2] > 0, au[:, 2], 1.0)), 0.0)
        Al = np.where(A > 0, (Xl + Yl) / A, 0.0)
    dfdu = np.stack([dfu, dfv, dfw], 1)
    g_u = df[:, None] * dfdu                            # dL/du
    g_xs = g_u / s                                      # dL/dx_S
    g_s = -g_u * u / s                                  # u = x_S / s
    g_m = -np.einsum("pji,pj->pi", R, g_xs)             # x_S = R (x - m)
    g_R = g_xs[:, :, None] * d[:, None, :]              # dL/dR_ij = g_xs_i d_j
    qn = np.linalg.norm(P.qraw[k], axis=1, keepdims=True)
    qhat = P.qraw[k] / qn
    g_qhat = np.einsum("pij,pijc->pc", g_R, _drot_dq(qhat))
    g_q = (g_qhat - qhat * np.sum(qhat * g_qhat, 1, keepdims=True)) / qn
    # d f / d eps: a = 2/e2, b = 2/e1, e = e2/e1
    dfde1 = -(e / e1) * B * lnA - (b / e1) * Zl
    dfde2 = (e * B / e2) * (lnA - a * Al)
    g_eps = np.stack([df * dfde1, df * dfde2], 1)
    return g_m, g_q, g_s, g_eps


def render_grad(grid, prims, rays, march, g_depth, g_sem, index=None, brute=False,
                ray_ids=None, batch=4096):
    """Gradients of L = sum_p g_D,p * D_p + sum_p <g_S,p, S_p> w.r.t. all
    primitive parameters (FP64).

    g_depth [cams,H,W], g_sem [cams,C,H,W] (or flat [n], [n,C] with ray_ids).
    Reverse mode through Eq. eq:depth_sem, eq:alpha_composite,
    eq:alpha_sem_sq and eq:sq_occupancy_prob; per ray the compositing adjoint
    runs back to front: Q_L = 0, Q_j = alpha_j G_j + (1 - alpha_j) Q_{j+1},
    dL/dalpha_j = T_j (G_j - Q_{j+1}), G_j = g_D t_j + <g_S, s_j>."""
    if index is None and not brute:
        index = build_index(prims, grid)[:3]
    P = _Prep(prims)
    N, C = prims.logits.shape
    o = rays.origins.reshape(-1, 3)
    d = rays.dirs.reshape(-1, 3)
    if ray_ids is None:
        gD = np.asarray(g_depth, np.float64).reshape(-1)
        gS = np.asarray(g_sem, np.float64).transpose(0, 2, 3, 1).reshape(-1, C)
    else:
        o, d = o[ray_ids], d[ray_ids]
        gD = np.asarray(g_depth, np.float64).reshape(-1)
        gS = np.asarray(g_sem, np.float64).reshape(-1, C)
    out = dict(means=np.zeros((N, 3)), quats=np.zeros((N, 4)), scales=np.zeros((N, 3)),
               eps=np.zeros((N, 2)), opacity=np.zeros(N), logits=np.zeros((N, C)))
    n = o.shape[0]
    for s0, e0 in _ray_batches(n, batch):
        _, _, _, recs, _ = _march(grid, prims, o[s0:e0], d[s0:e0], march, index, brute, P, True)
        gd = gD[s0:e0]
        gs = gS[s0:e0]
        Q = np.zeros(e0 - s0)
        for rec in reversed(recs):
            G = gd * rec["t"] + np.sum(gs * rec["s"], 1)
            dalpha = rec["T"] * (G - Q)
            Q = rec["alpha"] * G + (1.0 - rec["alpha"]) * Q
            da = np.where(rec["a"] < 1.0, dalpha, 0.0)          # reading R7
            r, k = rec["r"], rec["k"]
            if r.size == 0:
                continue
            p, _, _ = _eval_pairs(P, rec["x"], k)
            ds = rec["w"][r][:, None] * gs[r]                   # dL/ds_j = w_j g_S
            np.add.at(out["opacity"], k, da[r] * p)
            np.add.at(out["logits"], k, p[:, None] * ds)
            dp = da[r] * P.sigma[k] + np.sum(ds * P.logits[k], 1)
            g_m, g_q, g_s, g_eps = _pair_param_grads(P, rec["x"], k, dp)
            np.add.at(out["means"], k, g_m)
            np.add.at(out["quats"], k, g_q)
            np.add.at(out["scales"], k, g_s)
            np.add.at(out["eps"], k, g_eps)
    return out


def loss_value(render_out, g_depth, g_sem) -> float:
    """L = sum g_D * D + sum g_S * S (the linear loss whose gradient is
    `render_grad`)."""
    return float(np.sum(np.asarray(g_depth, np.float64) * render_out["depth"]) +
                 np.sum(np.asarray(g_sem, np.float64) * render_out["sem"]))

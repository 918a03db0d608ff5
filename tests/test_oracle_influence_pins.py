"""Pins of the influence-thresholded index (reading R21; Supplement
"Limitations and Future Work": occupancy-aware indexing).  theta = 0 is the
N_v cube; the region holds every point where p_o sigma >= theta (brute force
on points along the principal axes, where the region reaches furthest, and at
random); with the identity rotation it is the closed-form box
floor((m +- r s - lo) / voxel); low-opacity primitives drop out; the regions
shrink as theta grows; and a render with the thresholded index differs from
the full one by less than the dropped primitives' theta each."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.scenes_small import random_scene


def _scene(seed, n=40, **kw):
    return random_scene(seed, n=n, n_classes=3, width=9, height=7, n_samples=30, opacity_hi=0.9, nv=4,
                        dims=(24, 24, 12), voxel=0.5, lo=(-6.0, -6.0, -3.0), t_far=9.0, **kw)


def _with_theta(grid, theta):
    return dataclasses.replace(grid, theta=theta)


def test_theta_zero_is_the_cube():
    sc = _scene(0)
    a = oracle.influence_boxes(sc.prims, sc.grid)
    b = oracle.centre_boxes(sc.prims.means, sc.grid)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip(oracle.build_index(sc.prims, sc.grid), oracle.build_index(sc.prims.means, sc.grid)):
        assert np.array_equal(x, y)


def _occ(x, prims, k):
    """p_o of primitive k at the points x [P,3]."""
    rep = lambda a: np.repeat(np.asarray(a[k:k + 1], np.float64), x.shape[0], axis=0)
    return oracle.occupancy(x, rep(prims.means), rep(prims.quats), rep(prims.scales), rep(prims.eps))


def _voxel_exact(x, grid):
    return np.floor((x - np.asarray(grid.lo, np.float64)) / float(np.float32(grid.voxel))).astype(np.int64)


def _inside(blo, bhi, idx):
    return np.all((idx >= blo) & (idx <= bhi), axis=-1)


@pytest.mark.parametrize("theta", [1e-2, 1e-4, 1e-8])
def test_region_holds_every_point_above_theta(theta):
    """Points on the principal axes at 0.999 r (where p_o sigma >= theta and
    the region reaches furthest) and random points of the N_v cube with
    p_o sigma >= theta all fall in the thresholded box (when inside the cube)."""
    sc = _scene(1, n=60)
    g = _with_theta(sc.grid, theta)
    blo, bhi = oracle.influence_boxes(sc.prims, g)
    clo, chi = oracle.centre_boxes(sc.prims.means, sc.grid)
    R = oracle.rotation_matrix(sc.prims.quats)
    s = sc.prims.scales.astype(np.float64)
    e1 = sc.prims.eps[:, 0].astype(np.float64)
    sig = sc.prims.opacity.astype(np.float64)
    m = sc.prims.means.astype(np.float64)
    rng = np.random.default_rng(1)
    checked = 0
    for k in range(sc.prims.n):
        if not sig[k] > theta:
            assert np.any(blo[k] > bhi[k])           # empty
            continue
        r = np.log(sig[k] / theta) ** (e1[k] / 2)
        u = np.concatenate([np.eye(3), -np.eye(3)]) * (0.999 * r)
        pts = m[k] + (u * s[k]) @ R[k]              # x - m = R^T diag(s) u
        p = _occ(pts, sc.prims, k) * sig[k]
        assert np.all(p >= theta)
        lo_g = np.asarray(sc.grid.lo, np.float64)
        cube_lo = lo_g + clo[k] * float(np.float32(sc.grid.voxel))
        cube_hi = lo_g + (chi[k] + 1) * float(np.float32(sc.grid.voxel))
        rand = rng.uniform(cube_lo, cube_hi, (400, 3))
        pr = _occ(rand, sc.prims, k) * sig[k]
        allp = np.concatenate([pts, rand[pr >= theta]])
        idx = _voxel_exact(allp, sc.grid)
        in_cube = _inside(clo[k], chi[k], idx)
        assert np.all(_inside(blo[k], bhi[k], idx[in_cube])), k
        checked += int(in_cube.sum())
    assert checked > 100


def test_identity_rotation_closed_form():
    sc = _scene(2, n=30)
    pr = dataclasses.replace(sc.prims, quats=np.tile(np.array([[0.5, 0.0, 0.0, 0.0]], np.float32), (30, 1)))
    theta = 1e-3
    blo, bhi = oracle.influence_boxes(pr, _with_theta(sc.grid, theta))
    clo, chi = oracle.centre_boxes(pr.means, sc.grid)
    sig = pr.opacity.astype(np.float64)
    r = np.log(sig / theta) ** (pr.eps[:, 0].astype(np.float64) / 2)
    h = r[:, None] * pr.scales.astype(np.float64)
    lo = np.asarray(sc.grid.lo, np.float64)
    vs = float(np.float32(sc.grid.voxel))
    want_lo = np.maximum(clo, np.floor((pr.means - h - lo) / vs).astype(np.int64))
    want_hi = np.minimum(chi, np.floor((pr.means + h - lo) / vs).astype(np.int64))
    live = sig > theta
    assert np.array_equal(blo[live], want_lo[live]) and np.array_equal(bhi[live], want_hi[live])


def test_low_opacity_drops_out_and_regions_shrink_with_theta():
    sc = _scene(3, n=50)
    prev = None
    for theta in (0.0, 1e-6, 1e-3, 0.05, 0.5):
        lo, hi = oracle.influence_boxes(sc.prims, _with_theta(sc.grid, theta))
        vol = np.prod(np.clip(hi - lo + 1, 0, None), axis=1)
        if theta > 0:
            assert np.all(vol[sc.prims.opacity <= theta] == 0)
        if prev is not None:
            assert np.all(vol <= prev)
        prev = vol
    assert prev.sum() < oracle.box_volume_total(sc.prims.means, sc.grid)
    # the lists are sub-lists of the full index, still ascending per voxel
    full = oracle.build_index(sc.prims, sc.grid)
    part = oracle.build_index(sc.prims, _with_theta(sc.grid, 0.05))
    for v in np.flatnonzero(part[0]):
        a = full[2][full[1][v]:full[1][v] + full[0][v]]
        b = part[2][part[1][v]:part[1][v] + part[0][v]]
        assert np.all(np.diff(b) > 0) and np.all(np.isin(b, a))


def test_render_differs_by_less_than_theta_per_dropped_pair():
    """Per sample, a_j with the thresholded index differs from the full a_j by
    the dropped pairs' p sigma, each below theta (a small factor covers
    samples on a voxel face)."""
    theta = 2e-3
    sc = _scene(4, n=40)
    g1 = _with_theta(sc.grid, theta)
    P = oracle.sqr_oracle._Prep(sc.prims)
    o = sc.rays.origins.reshape(-1, 3)
    d = sc.rays.dirs.reshape(-1, 3)
    full = oracle.sqr_oracle._march(sc.grid, sc.prims, o, d, sc.march, oracle.build_index(sc.prims, sc.grid)[:3],
                                    False, P, True)[3]
    part = oracle.sqr_oracle._march(sc.grid, sc.prims, o, d, sc.march, oracle.build_index(sc.prims, g1)[:3],
                                    False, P, True)[3]
    fc, _, fi, _ = oracle.build_index(sc.prims, sc.grid)
    pc, _, pi, _ = oracle.build_index(sc.prims, g1)
    dropped_max = int(np.max(fc - pc))
    assert dropped_max > 0
    worst = 0.0
    for rf, rp in zip(full, part):
        da = np.abs(rf["a"] - rp["a"])
        worst = max(worst, float(np.max(da)))
        assert np.all(da <= dropped_max * theta * 1.001)
    assert worst > 0.0


def test_brute_membership_equals_the_lists_with_theta():
    """The renders from the thresholded lists and from the thresholded boxes
    used as a membership predicate (brute) agree bit for bit."""
    sc = _scene(5, n=30)
    g = _with_theta(sc.grid, 1e-3)
    a = oracle.render(g, sc.prims, sc.rays, sc.march)
    b = oracle.render(g, sc.prims, sc.rays, sc.march, brute=True)
    for k in ("depth", "sem", "t_final"):
        assert np.array_equal(a[k], b[k]), k
    va = oracle.voxelise(g, sc.prims)["density"]
    vb = oracle.voxelise(g, sc.prims, brute=True)["density"]
    assert np.array_equal(va, vb)

"""Pins of the voxelisation oracle (Eq. eq:voxelisation) against facts that do
not come from the oracle itself: exact centres, closed forms of p_o, the
neighbourhood cut-off, brute force, linearity, the label rule, and agreement
with the render's per-sample alpha at a sample that sits on a voxel centre."""
import numpy as np
import pytest

import oracle
import synth
from tests.scenes_small import random_scene

F32 = np.float32


def _prims(means, quats, scales, eps, opacity, logits):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    return synth.Prims(f(means), f(quats), f(scales), f(eps), f(opacity), f(logits))


def _vid(grid, i, j, k):
    return (i * grid.dims[1] + j) * grid.dims[2] + k


def test_voxel_centres_exact_and_inside_their_voxel():
    g = synth.Grid(lo=(-2.0, -1.5, 0.25), voxel=0.5, dims=(4, 3, 2), nv=1)
    cx, cy, cz = oracle.voxel_centres(g)
    np.testing.assert_array_equal(cx, F32([-1.75, -1.25, -0.75, -0.25]))
    np.testing.assert_array_equal(cy, F32([-1.25, -0.75, -0.25]))
    np.testing.assert_array_equal(cz, F32([0.5, 1.0]))
    # an awkward grid: every FP32 centre still falls in its own voxel (reading R5/R6 lookup)
    g2 = synth.Grid(lo=(-40.3, 17.1, -3.7), voxel=0.4, dims=(200, 200, 16), nv=5)
    c2 = oracle.voxel_centres(g2)
    for a in range(3):
        pts = np.zeros((g2.dims[a], 3), F32)
        pts[:, a] = c2[a]
        for b in range(3):
            if b != a:
                pts[:, b] = c2[b][0]
        inside, v = oracle.voxel_of_points(pts, g2)
        assert inside.all()
        i = np.stack(np.unravel_index(v, g2.dims), 1)[:, a]
        np.testing.assert_array_equal(i, np.arange(g2.dims[a]))


def test_primitive_on_a_centre_contributes_sigma_and_c_there():
    g = synth.Grid(lo=(-4.0, -4.0, -2.0), voxel=0.5, dims=(16, 16, 8), nv=2)
    cx, cy, cz = oracle.voxel_centres(g)
    m = (cx[5], cy[9], cz[3])
    pr = _prims([m], [(0.3, -0.5, 0.7, 0.2)], [(0.4, 0.9, 0.3)], [(0.6, 1.7)], [0.83], [(0.25, -1.5, 3.0)])
    out = oracle.voxelise(g, pr)
    v = _vid(g, 5, 9, 3)
    assert out["density"][v] == pytest.approx(np.float64(F32(0.83)), abs=0, rel=0)
    np.testing.assert_array_equal(out["sem"][v], pr.logits[0].astype(np.float64))


def test_ellipsoid_values_at_neighbouring_centres():
    """eps = (1, 1), identity rotation: p_o = exp(-(dx/sx)^2 - (dy/sy)^2 - (dz/sz)^2)."""
    g = synth.Grid(lo=(-4.0, -4.0, -2.0), voxel=0.5, dims=(16, 16, 8), nv=2)
    cx, cy, cz = oracle.voxel_centres(g)
    i0, j0, k0 = 7, 8, 4
    s = np.array([0.7, 1.3, 0.45])
    pr = _prims([(cx[i0], cy[j0], cz[k0])], [(1, 0, 0, 0)], [s], [(1.0, 1.0)], [0.6], [(1.0, 2.0)])
    out = oracle.voxelise(g, pr)
    sig = np.float64(F32(0.6))
    sf = s.astype(np.float32).astype(np.float64)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            for dk in range(-2, 3):
                d = np.array([di, dj, dk]) * 0.5
                want = sig * np.exp(-np.sum((d / sf) ** 2))
                got = out["density"][_vid(g, i0 + di, j0 + dj, k0 + dk)]
                assert got == pytest.approx(want, rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("ijk", [(0, 0, 0), (5, 6, 3), (11, 11, 5)])
def test_neighbourhood_cutoff_and_clipping(ijk):
    """A huge primitive (p_o ~ 1 everywhere) counts only inside its clipped
    N_v cube: 2x2x2 voxels in a corner, 3x3x3 inside the grid."""
    g = synth.Grid(lo=(0.0, 0.0, 0.0), voxel=1.0, dims=(12, 12, 6), nv=1)
    cx, cy, cz = oracle.voxel_centres(g)
    i, j, k = ijk
    pr = _prims([(cx[i], cy[j], cz[k])], [(1, 0, 0, 0)], [(500.0, 500.0, 500.0)], [(1.0, 1.0)], [1.0], [(1.0,)])
    out = oracle.voxelise(g, pr)
    dens = out["density"].reshape(g.dims)
    nz = np.argwhere(dens > 0)
    lo = np.maximum(np.array(ijk) - 1, 0)
    hi = np.minimum(np.array(ijk) + 1, np.array(g.dims) - 1)
    assert nz.min(0).tolist() == lo.tolist() and nz.max(0).tolist() == hi.tolist()
    assert len(nz) == int(np.prod(hi - lo + 1))
    # exp(-3 (1/500)^2) at the farthest corner of the cube
    assert np.all(dens[dens > 0] > 0.9999)


@pytest.mark.parametrize("seed,nv", [(0, 0), (1, 2), (2, 5), (3, 40)])
def test_index_walk_equals_brute_force_bitwise(seed, nv):
    sc = random_scene(seed, n=25, n_classes=4, nv=nv, dims=(10, 9, 6), voxel=0.5, lo=(-2.5, -2.0, -1.5))
    a = oracle.voxelise(sc.grid, sc.prims)
    b = oracle.voxelise(sc.grid, sc.prims, brute=True)
    for k in ("density", "sem", "labels"):
        assert np.array_equal(a[k], b[k]), k


def test_voxel_subset_equals_full_grid():
    sc = random_scene(4, n=30, n_classes=3, nv=2, dims=(10, 9, 6), voxel=0.5, lo=(-2.5, -2.0, -1.5))
    full = oracle.voxelise(sc.grid, sc.prims)
    vids = np.random.default_rng(0).choice(sc.grid.n_voxels, 57, replace=False)
    part = oracle.voxelise(sc.grid, sc.prims, voxel_ids=vids)
    for k in ("density", "sem", "labels"):
        assert np.array_equal(part[k], full[k][vids]), k


def test_linear_over_primitive_sets():
    sc = random_scene(5, n=40, n_classes=5, nv=3, dims=(10, 9, 6), voxel=0.5, lo=(-2.5, -2.0, -1.5))
    idx = np.random.default_rng(1).permutation(sc.prims.n)
    a, b = sc.prims.subset(idx[:17]), sc.prims.subset(idx[17:])
    full = oracle.voxelise(sc.grid, sc.prims)
    pa, pb = oracle.voxelise(sc.grid, a), oracle.voxelise(sc.grid, b)
    np.testing.assert_allclose(full["density"], pa["density"] + pb["density"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(full["sem"], pa["sem"] + pb["sem"], rtol=1e-12, atol=1e-12)


def test_label_rule_free_below_tau_and_argmax_above():
    g = synth.Grid(lo=(-4.0, -4.0, -2.0), voxel=0.5, dims=(16, 16, 8), nv=3)
    cx, cy, cz = oracle.voxel_centres(g)
    pr = _prims([(cx[4], cy[4], cz[4]), (cx[11], cy[11], cz[4])], [(1, 0, 0, 0), (1, 0, 0, 0)],
                [(0.5, 0.5, 0.5), (0.5, 0.5, 0.5)], [(1.0, 1.0), (1.0, 1.0)], [0.9, 0.9],
                [(4.0, 0.0, -1.0), (0.0, 4.0, -1.0)])
    out = oracle.voxelise(g, pr, tau=0.05)
    lab = out["labels"].reshape(g.dims)
    assert lab[4, 4, 4] == 0 and lab[11, 11, 4] == 1
    # two voxels away along x: density 0.9 exp(-(1/0.5)^2) = 0.0165 < tau -> free (= C)
    assert out["density"].reshape(g.dims)[6, 4, 4] == pytest.approx(0.9 * np.exp(-4.0), rel=1e-6)
    assert lab[6, 4, 4] == 3
    # one voxel away: 0.9 exp(-1) = 0.33 >= tau -> class 0
    assert lab[5, 4, 4] == 0
    # outside both neighbourhoods: nothing listed, density 0 -> free
    assert lab[0, 15, 0] == 3
    # the rule itself, including the first-maximum tie break
    d = np.array([0.05, 0.0499, 1.0])
    s = np.array([[1.0, 1.0], [3.0, 0.0], [0.0, 2.0]])
    np.testing.assert_array_equal(oracle.labels_from(d, s, 0.05), [0, 2, 1])


def test_density_equals_render_alpha_at_a_centre_sample():
    """A one-sample ray whose FP32 sample lands exactly on a voxel centre sees
    a_j = v_d there: depth = t min(1, v_d) and sem = min(1, v_d) v_s."""
    sc = random_scene(6, n=20, n_classes=3, nv=3, dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0),
                      opacity_hi=0.3)
    g = sc.grid
    cx, cy, cz = oracle.voxel_centres(g)
    rng = np.random.default_rng(2)
    picks = [(int(rng.integers(2, 14)), int(rng.integers(2, 14)), int(rng.integers(1, 7))) for _ in range(12)]
    centres = np.array([(cx[i], cy[j], cz[k]) for i, j, k in picks], F32)
    t = F32(1.0)
    dirs = np.tile(F32([1.0, 0.0, 0.0]), (len(picks), 1))
    origins = (centres - np.array([t, 0, 0], F32)).astype(F32)
    assert np.array_equal((origins + (t * dirs).astype(F32)).astype(F32), centres)
    rays = synth.Rays(origins.reshape(1, 1, -1, 3), dirs.reshape(1, 1, -1, 3))
    march = synth.March(1, float(t), float(t))
    r = oracle.render(g, sc.prims, rays, march)
    vox = oracle.voxelise(g, sc.prims, voxel_ids=[_vid(g, *p) for p in picks])
    alpha = np.minimum(1.0, vox["density"])
    np.testing.assert_allclose(r["depth"].reshape(-1), float(t) * alpha, rtol=1e-14, atol=0)
    sem = r["sem"][0].transpose(1, 2, 0).reshape(len(picks), -1)     # [1, C, 1, n] -> [n, C]
    np.testing.assert_allclose(sem, alpha[:, None] * vox["sem"], rtol=1e-13, atol=1e-15)

"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

The paper prints no worked input->output example, so every pin here is a
closed form, a library routine for a special case, an invariant, a brute-force
re-derivation, or finite differences.  Each is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong exponent, a transposed rotation,
a wrong sample spacing, an off-by-one voxel) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import softmax as scipy_softmax

import oracle
import synth
from tests.scenes_small import random_scene, single_prim_scene


# ---------------------------------------------------------------------------
# geometry: rotation convention and the inside-outside function
# ---------------------------------------------------------------------------

def test_rotation_matches_scipy():
    rng = np.random.default_rng(1)
    q = rng.standard_normal((50, 4)) * rng.uniform(0.3, 3.0, (50, 1))   # unnormalised
    R = oracle.rotation_matrix(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()            # scipy is (x,y,z,w)
    np.testing.assert_allclose(R, ref, atol=1e-13)


def test_rotation_axis_angle():
    # q = (cos(th/2), sin(th/2) n) rotates by th about n (Rodrigues)
    th = 0.7
    n = np.array([1.0, 2.0, -0.5]); n /= np.linalg.norm(n)
    q = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * n])
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    rod = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
    np.testing.assert_allclose(oracle.rotation_matrix(q[None])[0], rod, atol=1e-14)


def test_local_frame_is_R_times_offset():
    # x = m + R^T (s_x, 0, 0) lies on the unit level set iff x_S = R (x - m)
    rng = np.random.default_rng(2)
    q = rng.standard_normal(4)
    R = oracle.rotation_matrix(q[None])[0]
    m = np.array([0.3, -0.2, 0.1]); s = np.array([0.7, 0.4, 0.9])
    for axis in range(3):
        e = np.zeros(3); e[axis] = s[axis]
        x = m + R.T @ e
        p = oracle.occupancy(x[None], m[None], q[None], s[None], np.array([[0.6, 1.4]]))
        assert abs(p[0] - math.exp(-1.0)) < 1e-13
        # the transposed convention puts this point elsewhere
        x_alt = m + R @ e
        p_alt = oracle.occupancy(x_alt[None], m[None], q[None], s[None], np.array([[0.6, 1.4]]))
        assert abs(p_alt[0] - math.exp(-1.0)) > 1e-3


@pytest.mark.parametrize("e1,e2", [(0.2, 0.2), (0.5, 1.7), (1.8, 0.3), (1.0, 1.0), (2.0, 0.1)])
def test_inside_outside_special_directions(e1, e2):
    # on an axis f = |u|^(2/e1); on the xy diagonal f = 2^(e2/e1) |u|^(2/e1)
    for u in (0.3, 0.9, 1.0, 1.7):
        for sgn in (1.0, -1.0):
            f_x = oracle.inside_outside(np.array([sgn * u]), np.array([0.0]), np.array([0.0]), e1, e2)[0]
            f_y = oracle.inside_outside(np.array([0.0]), np.array([sgn * u]), np.array([0.0]), e1, e2)[0]
            f_z = oracle.inside_outside(np.array([0.0]), np.array([0.0]), np.array([sgn * u]), e1, e2)[0]
            f_d = oracle.inside_outside(np.array([u]), np.array([sgn * u]), np.array([0.0]), e1, e2)[0]
            assert math.isclose(f_x, u ** (2 / e1), rel_tol=1e-13)
            assert math.isclose(f_y, u ** (2 / e1), rel_tol=1e-13)
            assert math.isclose(f_z, u ** (2 / e1), rel_tol=1e-13)
            assert math.isclose(f_d, 2 ** (e2 / e1) * u ** (2 / e1), rel_tol=1e-13)
    # f is additive between the xy block and z: f(u,0,w) = |u|^(2/e1) + |w|^(2/e1)
    f = oracle.inside_outside(np.array([0.8]), np.array([0.0]), np.array([-0.6]), e1, e2)[0]
    assert math.isclose(f, 0.8 ** (2 / e1) + 0.6 ** (2 / e1), rel_tol=1e-13)


def test_inside_outside_zero_and_unit_cube_corner():
    assert oracle.inside_outside(np.zeros(1), np.zeros(1), np.zeros(1), 0.7, 1.3)[0] == 0.0
    # eps -> small: the unit level set approaches the cube |u|,|v|,|w| <= 1
    f_in = oracle.inside_outside(np.array([0.9]), np.array([0.9]), np.array([0.9]), 0.1, 0.1)[0]
    f_out = oracle.inside_outside(np.array([1.05]), np.array([0.2]), np.array([0.2]), 0.1, 0.1)[0]
    assert f_in < 1.0 < f_out


def _ellipsoid_quadratic(o, d, m, R, s):
    """f(o + t d) = a t^2 + 2 b t + c for eps1 = eps2 = 1: M = R^T S^-2 R."""
    M = R.T @ np.diag(1.0 / s ** 2) @ R
    dm = o - m
    return d @ M @ d, d @ M @ dm, dm @ M @ dm


def test_ellipsoid_occupancy_is_gaussian_quadratic():
    rng = np.random.default_rng(3)
    for _ in range(10):
        q = rng.standard_normal(4)
        R = oracle.rotation_matrix(q[None])[0]
        s = rng.uniform(0.3, 2.0, 3); m = rng.uniform(-1, 1, 3)
        o = rng.uniform(-3, 3, 3); d = rng.standard_normal(3); d /= np.linalg.norm(d)
        a, b, c = _ellipsoid_quadratic(o, d, m, R, s)
        t = np.linspace(0, 6, 25)
        x = o[None] + t[:, None] * d[None]
        P = t.size
        p = oracle.occupancy(x, np.tile(m, (P, 1)), np.tile(q, (P, 1)), np.tile(s, (P, 1)),
                             np.ones((P, 2)))
        np.testing.assert_allclose(p, np.exp(-(a * t * t + 2 * b * t + c)), rtol=1e-12)


def test_ray_sphere_textbook_hit_depth():
    # sphere radius r: p = exp(-|x-m|^2/r^2); textbook hit t = d.(m-o) - sqrt(r^2 - |perp|^2)
    rng = np.random.default_rng(4)
    for _ in range(10):
        r = rng.uniform(0.5, 2.0)
        m = rng.uniform(-1, 1, 3)
        o = m + rng.uniform(3, 5) * np.array([1.0, 0.2, -0.1])
        d = (m + rng.uniform(-0.3, 0.3, 3) - o); d /= np.linalg.norm(d)
        tc = d @ (m - o)
        perp2 = np.sum((m - o) ** 2) - tc * tc
        t_hit = tc - math.sqrt(r * r - perp2)
        x = o + t_hit * d
        q = rng.standard_normal(4)              # any rotation: a sphere is invariant
        p = oracle.occupancy(x[None], m[None], q[None], np.full((1, 3), r), np.ones((1, 2)))
        assert abs(p[0] - math.exp(-1.0)) < 1e-12


# ---------------------------------------------------------------------------
# samples and voxel decisions
# ---------------------------------------------------------------------------

def test_sample_depths_linspace_endpoints():
    t = oracle.sample_depths(100, 0.1, 45.0)
    assert t.dtype == np.float32 and t.size == 100
    assert t[0] == np.float32(0.1)
    np.testing.assert_allclose(t.astype(np.float64), np.linspace(0.1, 45.0, 100), rtol=2e-7)
    assert abs(float(t[-1]) - 45.0) < 1e-5
    assert np.all(np.diff(t) > 0)
    assert oracle.sample_depths(1, 0.5, 9.0)[0] == np.float32(0.5)


def test_voxel_of_points_faces_and_bounds():
    g = synth.Grid(lo=(-4.0, -4.0, -1.0), voxel=0.5, dims=(16, 16, 4), nv=5)
    pts = np.array([[-4.0, -4.0, -1.0],     # lower corner: voxel (0,0,0)
                    [-3.5, -4.0, -1.0],     # on a face: belongs to the higher voxel (1,0,0)
                    [3.999, 3.999, 0.999],  # last voxel
                    [4.0, 0.0, 0.0],        # upper face: outside
                    [-4.0001, 0.0, 0.0]], dtype=np.float32)
    inside, v = oracle.voxel_of_points(pts, g)
    assert list(inside) == [True, True, True, False, False]
    assert v[0] == 0
    assert v[1] == (1 * 16 + 0) * 4 + 0
    assert v[2] == (15 * 16 + 15) * 4 + 3


# ---------------------------------------------------------------------------
# index
# ---------------------------------------------------------------------------

def _centre_voxel_scalar(m, grid):
    """Per-primitive centre voxel with scalar FP32 ops (independent of the oracle)."""
    inv = np.float32(1.0) / np.float32(grid.voxel)
    out = []
    for ax in range(3):
        q = np.float32(np.float32(m[ax]) - np.float32(grid.lo[ax])) * inv
        out.append(math.floor(float(np.float32(q))))
    return out


@pytest.mark.parametrize("seed,nv,dims", [(0, 5, (16, 16, 4)), (1, 2, (7, 9, 5)), (2, 0, (6, 5, 4)),
                                          (3, 20, (6, 6, 3))])
def test_index_brute_force_membership(seed, nv, dims):
    rng = np.random.default_rng(seed)
    g = synth.Grid(lo=(-2.0, -1.5, -1.0), voxel=0.5, dims=dims, nv=nv)
    hi = np.array(g.lo) + np.array(dims) * 0.5
    n = 40
    means = rng.uniform(np.array(g.lo) - 2.0, hi + 2.0, (n, 3)).astype(np.float32)  # some outside
    counts, offsets, ids, total = oracle.build_index(means, g)
    cv = [_centre_voxel_scalar(means[k], g) for k in range(n)]
    X, Y, Z = dims
    e = 0
    for ix in range(X):
        for iy in range(Y):
            for iz in range(Z):
                v = (ix * Y + iy) * Z + iz
                want = [k for k in range(n) if max(abs(ix - cv[k][0]), abs(iy - cv[k][1]),
                                                   abs(iz - cv[k][2])) <= nv]
                got = list(ids[offsets[v]: offsets[v] + counts[v]])
                assert got == want, (v, got, want)
                assert offsets[v] == e
                e += len(want)
    assert total == e == counts.sum() == ids.size
    assert total == oracle.box_volume_total(means, g)


def test_index_translation_by_whole_voxels():
    rng = np.random.default_rng(5)
    g = synth.Grid(lo=(-4.0, -4.0, -1.0), voxel=0.5, dims=(16, 16, 4), nv=2)
    means = rng.uniform(-2.0, 1.0, (30, 3)).astype(np.float32)
    means[:, 2] = rng.uniform(-0.9, 0.4, 30).astype(np.float32)
    c0, o0, i0, _ = oracle.build_index(means, g)
    shifted = (means + np.float32(1.5)).astype(np.float32)   # +3 voxels in x (exact in f32)
    shifted[:, 1:] = means[:, 1:]
    c1, o1, i1, _ = oracle.build_index(shifted, g)
    c0 = c0.reshape(16, 16, 4); c1 = c1.reshape(16, 16, 4)
    # interior columns (far from the clipped faces) shift by exactly 3 voxels
    np.testing.assert_array_equal(c1[5:13], c0[2:10])


def test_index_empty_and_outside():
    g = synth.Grid(lo=(0.0, 0.0, 0.0), voxel=1.0, dims=(4, 4, 4), nv=1)
    c, o, i, t = oracle.build_index(np.zeros((0, 3), np.float32), g)
    assert t == 0 and c.sum() == 0 and i.size == 0
    far = np.array([[100.0, 1.0, 1.0], [-3.0, 1.0, 1.0], [np.nan, 1.0, 1.0]], np.float32)
    c, o, i, t = oracle.build_index(far, g)
    assert t == 0
    edge = np.array([[-1.5, 1.2, 1.2]], np.float32)   # centre voxel -2: box [-3,-1] misses
    assert oracle.build_index(edge, g)[3] == 0
    edge = np.array([[-0.5, 1.2, 1.2]], np.float32)   # centre voxel -1: box [-2,0] hits x=0
    assert oracle.build_index(edge, g)[3] == 1 * 3 * 3


# ---------------------------------------------------------------------------
# renderer: closed forms
# ---------------------------------------------------------------------------

def test_single_ellipsoid_saturating_depth_closed_form():
    """One ellipsoid with sigma = e^kappa: alpha_j = min(1, e^{kappa - f_j}) and
    alpha_j = 1 exactly iff f_j <= kappa, so the first saturated sample lies in
    the analytic interval of f(t) <= kappa and D = sum_{j<=j*} T_j alpha_j t_j."""
    kappa = 1.5
    rng = np.random.default_rng(6)
    q = rng.standard_normal(4)
    sc = single_prim_scene(mean=(0.2, -0.1, 0.0), quat=q, scales=(0.9, 0.6, 0.5), eps=(1.0, 1.0),
                           opacity=math.exp(kappa), logits=(0.3, -1.0), yaw=-90.0,
                           cam=(0.0, 3.5, 0.1), nv=45, dims=(40, 40, 40), lo=(-10.0, -10.0, -10.0),
                           hfov=40.0, width=8, height=6)
    # the grid holds every sample, so no sample is skipped
    out = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    R = oracle.rotation_matrix(sc.prims.quats.astype(np.float64))[0]
    m = sc.prims.means[0].astype(np.float64); s = sc.prims.scales[0].astype(np.float64)
    t32 = oracle.sample_depths(sc.march.n_samples, sc.march.t_near, sc.march.t_far)
    o_all = sc.rays.origins.reshape(-1, 3); d_all = sc.rays.dirs.reshape(-1, 3)
    sig32 = float(sc.prims.opacity[0])        # e^kappa rounded to f32: saturation iff f <= ln(sig32)
    kappa = math.log(sig32)
    n_sat = 0
    for r in range(o_all.shape[0]):
        o, d = o_all[r].astype(np.float64), d_all[r].astype(np.float64)
        M = R.T @ np.diag(1 / s ** 2) @ R
        T, D = 1.0, 0.0
        jstar = None
        for j, tj in enumerate(t32):
            x = (o_all[r] + (tj * d_all[r]).astype(np.float32)).astype(np.float32).astype(np.float64)
            f = (x - m) @ M @ (x - m)
            alpha = min(1.0, math.exp(kappa - f))
            D += T * alpha * float(tj)
            T *= 1 - alpha
            if alpha == 1.0 and jstar is None:
                jstar = j
        assert math.isclose(out["depth"].reshape(-1)[r], D, rel_tol=1e-12, abs_tol=1e-14)
        a, b, c = _ellipsoid_quadratic(o, d, m, R, s)
        disc = b * b - a * (c - kappa)
        if jstar is not None:
            n_sat += 1
            t_in, t_out = (-b - math.sqrt(disc)) / a, (-b + math.sqrt(disc)) / a
            inside = [j for j, tj in enumerate(t32) if t_in + 1e-5 < tj < t_out - 1e-5]
            assert inside and jstar == inside[0]
            assert out["t_final"].reshape(-1)[r] == 0.0
            assert out["depth"].reshape(-1)[r] <= float(t32[jstar]) + 1e-12
        # with the grid covering every sample, the semantic render is S = c * sum_j w_j p_j
    assert n_sat >= 10


def test_empty_scene_and_zero_opacity():
    sc = random_scene(7, n=0)
    out = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    assert np.all(out["depth"] == 0) and np.all(out["sem"] == 0) and np.all(out["t_final"] == 1)
    sc = random_scene(8, n=5)
    sc.prims.opacity[:] = 0
    out = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    assert np.all(out["depth"] == 0) and np.all(out["t_final"] == 1)
    # sigma = 0 but p > 0: semantics still zero because every weight w_j is zero
    assert np.all(out["sem"] == 0)


def _python_literal_render(sc):
    """All-primitives render with scalar Python loops (math.pow / math.exp)."""
    g, P = sc.grid, sc.prims
    t32 = oracle.sample_depths(sc.march.n_samples, sc.march.t_near, sc.march.t_far)
    inv = np.float32(1) / np.float32(g.voxel)
    o_all = sc.rays.origins.reshape(-1, 3); d_all = sc.rays.dirs.reshape(-1, 3)
    C = P.logits.shape[1]
    res = []
    for r in range(o_all.shape[0]):
        T, D, S = 1.0, 0.0, [0.0] * C
        for tj in t32:
            x32 = (o_all[r] + (tj * d_all[r]).astype(np.float32)).astype(np.float32)
            ok = True
            for ax in range(3):
                qv = np.float32(np.float32(x32[ax] - np.float32(g.lo[ax])) * inv)
                if not (0 <= qv < g.dims[ax]):
                    ok = False
            if not ok:
                continue
            a, s = 0.0, [0.0] * C
            for k in range(P.n):
                w_, x_, y_, z_ = [float(c) for c in P.quats[k]]
                nq = math.sqrt(w_ * w_ + x_ * x_ + y_ * y_ + z_ * z_)
                w_, x_, y_, z_ = w_ / nq, x_ / nq, y_ / nq, z_ / nq
                Rm = [[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
                      [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
                      [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]]
                dx = [float(x32[i]) - float(P.means[k][i]) for i in range(3)]
                xs = [sum(Rm[i][jj] * dx[jj] for jj in range(3)) for i in range(3)]
                u = [abs(xs[i]) / float(P.scales[k][i]) for i in range(3)]
                e1, e2 = float(P.eps[k][0]), float(P.eps[k][1])
                f = math.pow(math.pow(u[0], 2 / e2) + math.pow(u[1], 2 / e2), e2 / e1) + math.pow(u[2], 2 / e1)
                p = math.exp(-f)
                a += p * float(P.opacity[k])
                for c in range(C):
                    s[c] += p * float(P.logits[k][c])
            alpha = min(1.0, a)
            w = T * alpha
            D += w * float(tj)
            for c in range(C):
                S[c] += w * s[c]
            T *= 1 - alpha
        res.append((D, S, T))
    return res


def test_indexed_equals_literal_all_primitives_render():
    # N_v >= grid extent: every in-grid sample lists every primitive
    sc = random_scene(9, n=7, nv=40, width=4, height=3, n_samples=12, opacity_hi=0.4)
    out = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    lit = _python_literal_render(sc)
    dep = out["depth"].reshape(-1)
    sem = out["sem"].transpose(0, 2, 3, 1).reshape(-1, sc.prims.n_classes)
    tf = out["t_final"].reshape(-1)
    for r, (D, S, T) in enumerate(lit):
        assert math.isclose(dep[r], D, rel_tol=1e-11, abs_tol=1e-13)
        np.testing.assert_allclose(sem[r], S, rtol=1e-10, atol=1e-12)
        assert math.isclose(tf[r], T, rel_tol=1e-11, abs_tol=1e-13)


@pytest.mark.parametrize("seed,nv", [(10, 1), (11, 2), (12, 5)])
def test_indexed_equals_brute_force_bitwise(seed, nv):
    sc = random_scene(seed, n=12, nv=nv, width=7, height=5, n_samples=20)
    a = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    b = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, brute=True)
    for key in ("depth", "sem", "t_final"):
        assert np.array_equal(a[key], b[key])


def test_config0_indexed_equals_brute_force_bitwise():
    sc = synth.config(0)
    a = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    b = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, brute=True)
    assert np.array_equal(a["depth"], b["depth"]) and np.array_equal(a["sem"], b["sem"])


# ---------------------------------------------------------------------------
# renderer: invariants
# ---------------------------------------------------------------------------

def _march_records(sc):
    P = oracle.sqr_oracle._Prep(sc.prims)
    idx = oracle.build_index(sc.prims.means, sc.grid)[:3]
    o = sc.rays.origins.reshape(-1, 3); d = sc.rays.dirs.reshape(-1, 3)
    return oracle.sqr_oracle._march(sc.grid, sc.prims, o, d, sc.march, idx, False, P, True)


@pytest.mark.parametrize("seed", [13, 14])
def test_compositing_invariants(seed):
    sc = random_scene(seed, n=15, width=6, height=5, n_samples=24)
    depth, sem, tfin, recs, _ = _march_records(sc)
    W = np.stack([r["w"] for r in recs], 1)
    T = np.stack([r["T"] for r in recs], 1)
    A = np.stack([r["alpha"] for r in recs], 1)
    assert np.all((A >= 0) & (A <= 1)) and np.all(W >= 0)
    assert np.all(np.diff(T, axis=1) <= 0) and np.all(tfin <= T[:, -1])
    np.testing.assert_allclose(W.sum(1), 1 - tfin, atol=1e-13)
    t = np.array([r["t"] for r in recs])
    assert np.all(depth >= t[0] * W.sum(1) - 1e-12) and np.all(depth <= t[-1] * W.sum(1) + 1e-12)


def test_semantics_linear_in_logits_and_opacity_monotone():
    sc = random_scene(15, n=10, width=6, height=4, n_samples=18, opacity_hi=0.6)
    base = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    p2 = sc.prims.subset(np.arange(sc.prims.n))
    p2.logits = (2 * sc.prims.logits).astype(np.float32)
    dbl = oracle.render(sc.grid, p2, sc.rays, sc.march)
    np.testing.assert_allclose(dbl["sem"], 2 * base["sem"], rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(dbl["depth"], base["depth"])
    p3 = sc.prims.subset(np.arange(sc.prims.n))
    p3.opacity = np.minimum(1.0, sc.prims.opacity * 1.5).astype(np.float32)
    more = oracle.render(sc.grid, p3, sc.rays, sc.march)
    assert np.all(more["t_final"] <= base["t_final"] + 1e-15)


def test_softmax_matches_scipy():
    sc = random_scene(16, n=8, width=5, height=4)
    out = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    np.testing.assert_allclose(out["probs"], scipy_softmax(out["sem"], axis=1), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def _fd_check(sc, n_params=None, h=1e-6, seed=0, tol=2e-6):
    rng = np.random.default_rng(seed)
    C = sc.prims.n_classes
    g_d, g_s = synth.upstream_grads(rng, sc.rays, C)
    grads = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)

    def loss(pr):
        return oracle.loss_value(oracle.render(sc.grid, pr, sc.rays, sc.march), g_d, g_s)

    def discrete_state(pr):
        P = oracle.sqr_oracle._Prep(pr)
        idx = oracle.build_index(pr.means, sc.grid)
        o = sc.rays.origins.reshape(-1, 3); d = sc.rays.dirs.reshape(-1, 3)
        recs = oracle.sqr_oracle._march(sc.grid, pr, o, d, sc.march, idx[:3], False, P, True)[3]
        return (idx[2].tobytes(), tuple((r["a"] >= 1).tobytes() for r in recs),
                tuple(r["k"].tobytes() for r in recs))

    base64 = synth.Prims(*(a.astype(np.float64) for a in (sc.prims.means, sc.prims.quats, sc.prims.scales,
                                                          sc.prims.eps, sc.prims.opacity, sc.prims.logits)))
    st0 = discrete_state(sc.prims)
    checked = 0
    worst = 0.0
    for name in ("means", "quats", "scales", "eps", "opacity", "logits"):
        arr = getattr(base64, name)
        flat_idx = list(range(arr.size))
        for fi in flat_idx:
            plus = synth.Prims(*(np.array(a) for a in (base64.means, base64.quats, base64.scales, base64.eps,
                                                        base64.opacity, base64.logits)))
            minus = synth.Prims(*(np.array(a) for a in (base64.means, base64.quats, base64.scales, base64.eps,
                                                         base64.opacity, base64.logits)))
            getattr(plus, name).reshape(-1)[fi] += h
            getattr(minus, name).reshape(-1)[fi] -= h
            if discrete_state(plus) != st0 or discrete_state(minus) != st0:
                continue   # a kink (centre voxel, clamp or list change) lies inside [-h, h]
            fd = (loss(plus) - loss(minus)) / (2 * h)
            an = grads[name].reshape(-1)[fi]
            err = abs(fd - an) / (abs(an) + 1e-3)
            worst = max(worst, err)
            assert err < tol, (name, fi, fd, an)
            checked += 1
    return checked, worst


def test_adjoint_matches_central_differences_unclamped():
    sc = random_scene(17, n=4, n_classes=2, width=4, height=3, n_samples=14, opacity_hi=0.3)
    checked, worst = _fd_check(sc)
    assert checked >= 4 * 15 * 0.9


def test_adjoint_matches_central_differences_with_clamping():
    sc = random_scene(21, n=8, n_classes=2, width=4, height=3, n_samples=14, opacity_hi=1.0,
                      scale_lo=0.7, scale_hi=1.5)
    depth, sem, tfin, recs, _ = _march_records(sc)
    assert any(np.any(r["a"] >= 1) for r in recs)       # the clamp is exercised
    checked, worst = _fd_check(sc, seed=1)
    assert checked >= 8 * 15 * 0.7


def test_logit_gradient_closed_form():
    # dL/dc_k = sum_{r,j} w_rj p_rjk g_S,r  (S is linear in c with weights w p)
    sc = random_scene(19, n=6, n_classes=3, width=5, height=4, n_samples=16)
    rng = np.random.default_rng(2)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 3)
    grads = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    depth, sem, tfin, recs, _ = _march_records(sc)
    gS = g_s.transpose(0, 2, 3, 1).reshape(-1, 3).astype(np.float64)
    want = np.zeros((sc.prims.n, 3))
    P = oracle.sqr_oracle._Prep(sc.prims)
    for rec in recs:
        r, k = rec["r"], rec["k"]
        if r.size == 0:
            continue
        p = oracle.occupancy(rec["x"], P.means[k], P.qraw[k], P.scales[k], P.eps[k])
        for i in range(r.size):
            want[k[i]] += rec["w"][r[i]] * p[i] * gS[r[i]]
    np.testing.assert_allclose(grads["logits"], want, rtol=1e-11, atol=1e-13)


def test_sphere_has_no_rotation_gradient():
    sc = single_prim_scene(mean=(0.1, 0.0, 0.05), quat=(0.3, -0.5, 0.2, 0.7), scales=(0.8, 0.8, 0.8),
                           eps=(1.0, 1.0), opacity=0.7, logits=(0.2, 0.5), yaw=-90.0, cam=(0.0, 3.0, 0.0),
                           n_samples=24)
    rng = np.random.default_rng(3)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 2)
    g = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(g["means"]).max() > 1e-3
    assert np.abs(g["quats"]).max() < 1e-10 * np.abs(g["means"]).max()

"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Index: bit-exact.  Forward: depth within 1e-4 relative (1e-5 m below 0.1 m),
class probabilities within 1e-5 absolute.  Backward: per parameter group
relative L2 within 1e-3 and per element within 1e-3 |g| + 1e-3 rms(g)."""
import numpy as np
import pytest

import oracle
import synth
from tests.scenes_small import random_scene, single_prim_scene

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_17361_amd import api
    from tests import gpu_helpers as H


def _say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# index
# ---------------------------------------------------------------------------

def _index_case(sc):
    grid, prims, _, _ = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    torch.cuda.synchronize()
    e = idx.checked_total()
    c, o, i, t = oracle.build_index(sc.prims.means, sc.grid)
    assert e == t
    np.testing.assert_array_equal(idx.counts.cpu().numpy(), c)
    np.testing.assert_array_equal(idx.offsets.cpu().numpy(), o)
    np.testing.assert_array_equal(idx.ids[:e].cpu().numpy(), i)
    return idx


@pytest.mark.parametrize("seed,nv,n", [(0, 5, 64), (1, 0, 30), (2, 2, 200), (3, 40, 9), (4, 5, 0)])
def test_index_bitexact_small(seed, nv, n):
    _say("index small", seed, nv, n)
    sc = random_scene(seed, n=n, nv=nv, dims=(13, 11, 7), voxel=0.5, lo=(-3.0, -2.5, -1.5))
    # push a few centres outside the grid (boxes partly or fully clipped)
    if n > 4:
        sc.prims.means[:4] = np.array([[-5.0, 0, 0], [0, 9.0, 0], [0, 0, -4.2], [30.0, 30.0, 30.0]], np.float32)
    _index_case(sc)


def test_index_bitexact_config0():
    _index_case(synth.config(0))


def test_index_bitexact_config1_and_repeatable():
    sc = synth.config(1)
    _say("index config1")
    idx = _index_case(sc)
    grid, prims, _, _ = H.gpu_scene(sc)
    idx2 = api.build_index(grid, prims)
    torch.cuda.synchronize()
    e = idx.checked_total()
    assert idx2.checked_total() == e
    # slots past the total are unwritten workspace: compare the filled prefix
    assert torch.equal(idx.ids[:e], idx2.ids[:e]) and torch.equal(idx.counts, idx2.counts)
    assert torch.equal(idx.offsets, idx2.offsets)


def test_index_bitexact_dense_tiles_beyond_the_sort():
    """6,000 primitives crowded into a few voxel tiles: the tiles whose binned
    candidate slice exceeds the in-LDS sort stream every primitive of the
    scene instead, the others sort their slice; both give the oracle's lists
    bit for bit (ascending ids)."""
    sc = random_scene(6, n=6000, nv=5, dims=(24, 20, 18), voxel=0.5, lo=(-6.0, -5.0, -4.5))
    rng = np.random.default_rng(6)
    # two thirds of the centres inside a 1.2 m cube, the rest spread over the grid
    sc.prims.means[:4000] = rng.uniform(-0.6, 0.6, (4000, 3)).astype(np.float32)
    _say("index dense tiles")
    _index_case(sc)


def test_index_capacity_overflow_is_reported():
    sc = random_scene(5, n=50, nv=3, dims=(12, 12, 6))
    grid, prims, _, _ = H.gpu_scene(sc)
    idx = api.build_index(grid, prims, capacity=100)
    torch.cuda.synchronize()
    with pytest.raises(Exception):
        idx.checked_total()
    # the kernels wrote nothing beyond the capacity and the true E is reported
    assert int(idx.total.item()) == oracle.box_volume_total(sc.prims.means, sc.grid)


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------

def _fwd_case(sc, tuning=None, ray_ids=None, what=""):
    out, _ = H.run_fwd(sc, tuning=tuning)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, ray_ids=ray_ids)
    if ray_ids is None:
        H.assert_depth_close(out["depth"], ref["depth"], what)
        H.assert_probs_close(out["probs"], ref["probs"], what)
        H.assert_tfinal_close(out["t_final"], ref["t_final"], what)
    else:
        H.assert_depth_close(out["depth"].reshape(-1)[ray_ids], ref["depth"], what)
        H.assert_probs_close(H.flat_sem(out["probs"])[ray_ids], ref["probs"], what)
        H.assert_tfinal_close(out["t_final"].reshape(-1)[ray_ids], ref["t_final"], what)
    return out, ref


def test_fwd_config0_full():
    _say("fwd config0")
    _fwd_case(synth.config(0), what="cfg0")


@pytest.mark.parametrize("tile_w,wpb", [(8, 4), (4, 1), (16, 2)])
@pytest.mark.parametrize("seed,n,C,nv", [(20, 12, 3, 5), (21, 40, 17, 2), (22, 25, 1, 0), (23, 30, 20, 40),
                                         (24, 18, 32, 3), (25, 15, 8, 5)])
def test_fwd_small_scenes_ragged(seed, n, C, nv, tile_w, wpb):
    _say("fwd small", seed, n, C, nv, tile_w, wpb)
    sc = random_scene(seed, n=n, n_classes=C, nv=nv, width=37, height=23, n_samples=33, opacity_hi=0.7,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    _fwd_case(sc, tuning=api.Tuning(tile_w, wpb), what=f"seed{seed}")


def test_fwd_edge_cases():
    _say("fwd edge: empty scene")
    sc = random_scene(30, n=0, width=9, height=7)
    out, _ = H.run_fwd(sc)
    assert np.all(out["depth"] == 0) and np.all(out["t_final"] == 1) and np.all(out["sem"] == 0)
    _say("fwd edge: single sample")
    sc = random_scene(31, n=10, width=9, height=7, n_samples=1)
    _fwd_case(sc, what="L=1")
    _say("fwd edge: camera outside the grid looking away")
    sc = random_scene(32, n=10, width=9, height=7, cam=(0.0, 0.0, 10.0))
    out, _ = H.run_fwd(sc)
    assert np.all(out["t_final"] == 1)
    _say("fwd edge: primitives all outside the grid")
    sc = random_scene(33, n=10, width=9, height=7)
    sc.prims.means[:] = np.float32(50.0)
    out, _ = H.run_fwd(sc)
    assert np.all(out["depth"] == 0)
    _say("fwd edge: saturating ellipsoid")
    sc = single_prim_scene(mean=(0.2, -0.1, 0.0), quat=(0.9, 0.1, -0.3, 0.2), scales=(0.9, 0.6, 0.5),
                           eps=(1.0, 1.0), opacity=4.48, logits=(0.3, -1.0), yaw=-90.0, cam=(0.0, 3.5, 0.1),
                           nv=45, dims=(40, 40, 40), lo=(-10.0, -10.0, -10.0), hfov=40.0, width=8, height=6)
    _fwd_case(sc, what="ellipsoid")


def test_fwd_config1_sampled_rays():
    sc = synth.config(1)
    rng = np.random.default_rng(0)
    ids = rng.choice(sc.rays.n_rays, 3000, replace=False)
    _say("fwd config1")
    out, _ = _fwd_case(sc, ray_ids=ids, what="cfg1")
    # a whole ragged window too (several tiles)
    win = np.arange(352 * 37, 352 * 37 + 352 * 3)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, ray_ids=win)
    H.assert_depth_close(out["depth"].reshape(-1)[win], ref["depth"], "cfg1 window")
    H.assert_probs_close(H.flat_sem(out["probs"])[win], ref["probs"], "cfg1 window")


def test_fwd_config4_sampled_rays():
    sc = synth.config(4)
    rng = np.random.default_rng(1)
    ids = rng.choice(sc.rays.n_rays, 600, replace=False)
    _say("fwd config4")
    _fwd_case(sc, ray_ids=ids, what="cfg4")


def test_fwd_paper_render_setting_sampled_rays():
    """The paper's render setting that the bench times beside its figure
    (6 x 704x256 rays, 1,600 superquadrics, L = 100 in [0.1, 40] m)."""
    sc = synth.paper_render_scene()
    ids = np.random.default_rng(2).choice(sc.rays.n_rays, 2000, replace=False)
    _say("fwd paper render setting")
    _fwd_case(sc, ray_ids=ids, what="paper setting")


@pytest.mark.parametrize("C", [5, 17, 32])
def test_fwd_bitmap_union_walk_equals_voxel_group_walk(C):
    """140k primitives: with one wave per block the per-wave union bitmap fits
    the LDS budget, with four it does not and mixed-voxel samples walk one
    voxel group at a time.  Both give each lane its own list in ascending id,
    so the outputs agree bit for bit (the matrix-core class sums round as one
    FMA per pair, and lanes outside a visit add exact zeros); sampled rays are
    checked against the oracle."""
    sc = random_scene(26, n=140_000, n_classes=C, nv=1, width=64, height=48, n_samples=40, opacity_hi=0.5,
                      dims=(32, 32, 16), voxel=0.25, lo=(-4.0, -4.0, -2.0), scale_lo=0.03, scale_hi=0.12,
                      t_far=7.0)
    _say("fwd 140k prims, union (wpb 1) vs voxel groups (wpb 4), C", C)
    a, _ = H.run_fwd(sc, ckpt_every=4, tuning=api.Tuning(8, 1))
    b, _ = H.run_fwd(sc, ckpt_every=4, tuning=api.Tuning(8, 4))
    for k in ("depth", "sem", "t_final", "ckpt"):
        assert np.array_equal(a[k], b[k]), k
    ids = np.random.default_rng(26).choice(sc.rays.n_rays, 300, replace=False)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, ray_ids=ids)
    H.assert_depth_close(a["depth"].reshape(-1)[ids], ref["depth"], "140k")
    H.assert_probs_close(H.flat_sem(a["probs"])[ids], ref["probs"], "140k")


def test_fwd_deterministic_and_ckpt_consistent():
    sc = synth.config(0)
    a, _ = H.run_fwd(sc)
    b, _ = H.run_fwd(sc, ckpt_every=8)
    for k in ("depth", "sem", "t_final"):
        assert np.array_equal(a[k], b[k]), k
    ck = b["ckpt"]
    assert ck.shape == (4, sc.rays.n_rays)
    assert np.all(ck[0] == 1.0)
    assert np.all(np.diff(ck, axis=0) <= 0)
    assert np.all(ck[-1] >= b["t_final"].reshape(-1))


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K,mode", [(4, 1), (4, 2), (8, 1), (8, 2), (16, 1), (16, 0)])
@pytest.mark.parametrize("seed,n,C,opac", [(40, 6, 3, 0.4), (41, 12, 4, 1.0), (42, 20, 17, 0.8), (43, 8, 32, 0.6),
                                           (44, 60, 8, 0.9)])
def test_bwd_small_scenes(seed, n, C, opac, K, mode):
    _say("bwd small", seed, n, C, opac, K, mode)
    sc = random_scene(seed, n=n, n_classes=C, width=19, height=13, n_samples=37, opacity_hi=opac,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    rng = np.random.default_rng(seed)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, C)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=K, tuning=api.Tuning(8, 4, mode))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close(g, ref, f"seed{seed} K{K} mode{mode}")


@pytest.mark.parametrize("voxel,dims,K", [(0.1, (80, 80, 40), 8), (0.1, (80, 80, 40), 4), (0.25, (32, 32, 16), 8)])
def test_bwd_voxels_small_against_the_sample_spacing(voxel, dims, K):
    """0.1 m voxels against a 0.3 m sample spacing: consecutive samples of a
    ray skip cells, so a chunk's samples and the primitive boxes they meet
    spread over many more cells than on the bench grid (0.25 m: a middle
    case).  The primitive-major backward still matches the oracle."""
    _say("bwd small voxels", voxel, dims, K)
    sc = random_scene(47, n=40, n_classes=5, width=19, height=13, n_samples=24, opacity_hi=0.6, dims=dims,
                      voxel=voxel, lo=(-4.0, -4.0, -2.0), t_far=7.0, scale_lo=0.15, scale_hi=0.5)
    rng = np.random.default_rng(47)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 5)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=K, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["opacity"]).max() > 0, "the camera must see the primitives"
    H.assert_grads_close(g, ref, f"small voxels {voxel} K{K}")


@pytest.mark.parametrize("eps_pair", [(0.1, 0.1), (2.0, 2.0), (0.1, 2.0), (2.0, 0.1)])
def test_fwd_bwd_at_the_ends_of_the_shape_range(eps_pair):
    """Shape exponents at the ends of the paper's range [0.1, 2]: eps = 0.1
    gives exponents 2/eps = 20 (near-box shapes, steep p), eps = 2 gives
    exponent 1 (near-octahedra).  Forward and gradients against the oracle,
    with half the primitives at each end pair and half random.  At (2, 0.1)
    one primitive's samples pass within 1% of its third axis, where |u|^20
    underflows float32 while (|u|^20 + |v|^20)^(1/20) is still about |u|."""
    _say("fwd+bwd shape range ends", eps_pair)
    sc = random_scene(48, n=24, n_classes=5, width=21, height=15, n_samples=33, opacity_hi=0.8,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    sc.prims.eps[::2] = np.float32(eps_pair)
    _fwd_case(sc, what=f"eps {eps_pair}")
    rng = np.random.default_rng(48)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 5)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["opacity"]).max() > 0, "the camera must see the primitives"
    H.assert_grads_close(g, ref, f"eps {eps_pair}")


@pytest.mark.parametrize("seed", [61, 62, 63, 64, 65, 66])
def test_fwd_bwd_random_shapes_over_the_whole_eps_range(seed):
    """Random scenes whose eps1, eps2 are uniform over the paper's whole range
    [0.1, 2] (the synthetic workloads draw from [0.2, 1.8]), 40 primitives
    of scales 0.2..1.5 in front of one camera.  Forward and gradients
    against the oracle."""
    _say("fwd+bwd random eps over [0.1, 2], seed", seed)
    sc = random_scene(seed, n=40, n_classes=4, width=19, height=13, n_samples=40, opacity_hi=0.9,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0, scale_lo=0.2, scale_hi=1.5)
    rng = np.random.default_rng(seed)
    sc.prims.eps[:] = rng.uniform(0.1, 2.0, sc.prims.eps.shape).astype(np.float32)
    _fwd_case(sc, what=f"random eps seed {seed}")
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 4)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["opacity"]).max() > 0, "the camera must see the primitives"
    H.assert_grads_close(g, ref, f"random eps seed {seed}")


@pytest.mark.parametrize("seed", [71, 72])
def test_fwd_bwd_scale_and_quaternion_norm_extremes(seed):
    """Primitives thinner than the sample spacing (s = 0.03..0.08 against a
    spacing of 0.17), primitives spanning most of the grid (s = 2.5..4),
    and quaternions of norm 0.01 and 30 (the renderer uses r/|r|, so the
    quaternion gradient is tangent to the sphere and scales with 1/|r|).
    Forward and gradients against the oracle."""
    _say("fwd+bwd scale / quaternion-norm extremes, seed", seed)
    sc = random_scene(seed, n=24, n_classes=3, width=17, height=13, n_samples=40, opacity_hi=0.9,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    rng = np.random.default_rng(seed)
    sc.prims.scales[0:6] = rng.uniform(0.03, 0.08, (6, 3)).astype(np.float32)
    sc.prims.scales[6:10] = rng.uniform(2.5, 4.0, (4, 3)).astype(np.float32)
    sc.prims.quats[10:16] *= np.float32(0.01)
    sc.prims.quats[16:20] *= np.float32(30.0)
    _fwd_case(sc, what=f"extremes seed {seed}")
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 3)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["opacity"][0:6]).max() > 0 and np.abs(ref["opacity"][6:10]).max() > 0, \
        "thin and large primitives must be seen"
    H.assert_grads_close(g, ref, f"extremes seed {seed}")


def _quat_taking_to_z(d):
    """(w, x, y, z) of the rotation that maps the unit vector d onto +z."""
    q = np.array([1.0 + d[2], d[1], -d[0], 0.0])
    return q / np.linalg.norm(q)


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("eps1", [2.0, 1.5])
def test_fwd_bwd_samples_near_the_third_axis_of_a_flat_exponent(eps1):
    """Primitives with eps2 = 0.1 (a = 20) whose third local axis runs
    parallel to a camera ray at 0.2% to 3% of s_x: along that ray |u| is the
    offset and v is 0 to rounding, so |u|^a underflows float32 while
    B = (|u|^a + |v|^a)^(eps2/eps1) is |u|^(2/eps1), of order |u|, and dB/du is
    of order 1.  The kernels must form B in the log domain to match the
    oracle here (forward values and every gradient)."""
    _say("fwd+bwd near the third axis, eps1", eps1)
    rays = synth.pinhole_rig(1, 21, 15, 90.0, (0.0, 0.0, 0.0))
    picks = [(7, 10, 2.0, 0.002), (3, 4, 2.6, 0.005), (11, 16, 3.0, 0.01), (5, 13, 1.8, 0.03)]
    scales = np.array([[0.8, 0.6, 1.0], [0.5, 0.7, 0.9], [1.0, 0.9, 0.6], [0.6, 0.6, 1.2]])
    means, quats = [], []
    for (row, col, t0, off), s in zip(picks, scales):
        d = rays.dirs[0, row, col].astype(np.float64)
        q = _quat_taking_to_z(d)
        R = _rot(q)
        assert np.allclose(R @ d, [0.0, 0.0, 1.0])
        means.append(rays.origins[0, row, col] + t0 * d - off * s[0] * R[0])
        quats.append(q)
    rng = np.random.default_rng(7)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    prims = synth.Prims(f32(means), f32(quats), f32(scales), f32([[eps1, 0.1]] * 4),
                        f32([0.9, 0.7, 0.8, 0.6]), f32(rng.standard_normal((4, 3))))
    sc = synth.Scene(synth.Grid(lo=(-4.0, -4.0, -2.0), voxel=0.5, dims=(16, 16, 8), nv=5), prims, rays,
                     synth.March(48, 0.1, 5.0), name="near-axis")
    _fwd_case(sc, what=f"near axis eps1 {eps1}")
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 3)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["means"]).min() > 0, "every primitive must be seen"
    H.assert_grads_close(g, ref, f"near axis eps1 {eps1}")


@pytest.mark.parametrize("eps", [(2.0, 2.0), (1.0, 0.5), (2.0, 0.1), (0.5, 1.0)])
def test_fwd_bwd_samples_exactly_on_principal_planes_and_axes(eps):
    """The centre ray of an odd-sized image runs exactly along +x, and the
    quaternions below give exact permutation matrices, so samples on that
    ray have local coordinates that are exactly 0: v = w = 0 (identity),
    u = v = 0 (the cyclic permutation taking x to the third axis) and w = 0
    (identity, offset in y).  log2 0 = -inf then meets every exponent; at
    eps = 2 (exponent 1) the derivative of |u| at 0 is taken as 0 on both
    sides.  Forward values and every gradient against the oracle."""
    _say("fwd+bwd exact zeros, eps", eps)
    rays = synth.pinhole_rig(1, 21, 15, 90.0, (0.0, 0.0, 0.0))
    assert (rays.dirs[0, 7, 10] == np.float32([1.0, 0.0, 0.0])).all()
    ident, cyc = [1.0, 0.0, 0.0, 0.0], [0.5, -0.5, -0.5, -0.5]
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    rng = np.random.default_rng(11)
    prims = synth.Prims(f32([[2.0, 0.0, 0.0], [3.0, 0.0, 0.0], [1.5, 0.2, 0.0], [2.5, 0.0, 0.0]]),
                        f32([ident, cyc, ident, cyc]),
                        f32([[0.4, 0.3, 0.5], [0.5, 0.4, 0.3], [0.3, 0.6, 0.4], [0.35, 0.35, 0.45]]),
                        f32([eps] * 4), f32([0.8, 0.9, 0.6, 0.7]), f32(rng.standard_normal((4, 3))))
    sc = synth.Scene(synth.Grid(lo=(-4.0, -4.0, -2.0), voxel=0.5, dims=(16, 16, 8), nv=5), prims, rays,
                     synth.March(48, 0.1, 5.0), name="exact-zeros")
    _fwd_case(sc, what=f"exact zeros eps {eps}")
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 3)
    _, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=api.Tuning(8, 4, 2))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    assert np.abs(ref["opacity"]).min() > 0, "every primitive must be seen"
    H.assert_grads_close(g, ref, f"exact zeros eps {eps}")


def test_bwd_forcing_primitive_major_where_it_does_not_apply_is_rejected():
    sc = random_scene(45, n=5, width=9, height=7)
    with pytest.raises(Exception, match="status -4"):
        H.run_fwd_bwd(sc, *synth.upstream_grads(np.random.default_rng(0), sc.rays, 3), ckpt_every=16,
                      tuning=api.Tuning(8, 4, 2))


def test_bwd_config0():
    sc = synth.config(0)
    rng = np.random.default_rng(7)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, sc.prims.n_classes)
    _say("bwd config0")
    _, g = H.run_fwd_bwd(sc, g_d, g_s)
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close(g, ref, "cfg0")


@pytest.mark.parametrize("mode", [1, 2])
def test_bwd_config2_sparse_upstream(mode):
    """Config 2 (config 1 shapes): upstream gradients non-zero on 1500 rays only,
    so the oracle's gradient is exact while touching those rays alone."""
    sc = synth.config(2)
    C = sc.prims.n_classes
    rng = np.random.default_rng(8)
    ids = rng.choice(sc.rays.n_rays, 1500, replace=False)
    g_d = np.zeros(sc.rays.n_rays, np.float32)
    g_s = np.zeros((sc.rays.n_rays, C), np.float32)
    g_d[ids] = rng.standard_normal(ids.size).astype(np.float32)
    g_s[ids] = rng.standard_normal((ids.size, C)).astype(np.float32)
    cams, Hh, Ww = sc.rays.shape
    g_d_img = g_d.reshape(cams, Hh, Ww)
    g_s_img = g_s.reshape(cams, Hh, Ww, C).transpose(0, 3, 1, 2).copy()
    _say("bwd config2", mode)
    _, g = H.run_fwd_bwd(sc, g_d_img, g_s_img, tuning=api.Tuning(8, 4, mode))
    ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d[ids], g_s[ids], ray_ids=ids)
    H.assert_grads_close(g, ref, "cfg2")


def _long_grid_scene(dims, voxel, lo, centres, pitch):
    """A column-shaped grid longer than the packed cell form holds (1023 cells
    along x or y, 511 along z), primitives strung along its axis and a narrow
    camera at the origin looking down it."""
    rng = np.random.Generator(np.random.PCG64(61))
    grid = synth.Grid(lo=lo, voxel=voxel, dims=dims, nv=2)
    prims = synth.make_prims(rng, np.asarray(centres, np.float64), 0.05, 0.15, 5)
    rays = synth.pinhole_rig(1, 16, 12, 2.0, (0.0, 0.0, 0.0), pitch_deg=pitch)
    return synth.Scene(grid, prims, rays, synth.March(64, 0.1, 12.0), name="long")


@pytest.mark.parametrize("axis", ["x", "z"])
def test_grids_beyond_packed_cells(axis):
    """Such grids do not fit the packed-cell membership test: the forward walks
    one voxel group at a time and the backward runs sample-major.  Both still
    match the oracle, and forcing the primitive-major backward is refused."""
    t = np.linspace(1.0, 10.0, 24)
    if axis == "x":
        sc = _long_grid_scene((1100, 8, 8), 0.05, (-0.5, -0.2, -0.2), np.stack([t, 0 * t, 0 * t], 1), 0.0)
    else:
        sc = _long_grid_scene((8, 8, 600), 0.05, (-0.2, -0.2, -0.5), np.stack([0 * t, 0 * t, t], 1), 90.0)
    _say("grid beyond packed cells", axis, sc.grid.dims)
    C = sc.prims.n_classes
    rng = np.random.default_rng(61)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, C)
    out, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=4, tuning=api.Tuning(8, 2))
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    assert np.count_nonzero(ref["depth"] > 0.5) > 20, "the camera must see the primitives"
    H.assert_depth_close(out["depth"], ref["depth"], f"long {axis}")
    H.assert_probs_close(out["probs"], ref["probs"], f"long {axis}")
    H.assert_grads_close(g, oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s), f"long {axis}")
    with pytest.raises(Exception, match="status -4"):
        H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=4, tuning=api.Tuning(8, 2, 2))


@pytest.mark.parametrize("cam,yaw,pitch", [((-6.0, 0.3, 0.2), 0.0, 0.0), ((0.5, -0.5, 0.0), 180.0, 30.0),
                                           ((0.0, 5.0, -0.3), -90.0, -20.0)])
def test_rays_entering_and_leaving_the_grid(cam, yaw, pitch):
    """Rays that start outside the grid and enter it later, rays that leave it
    through every face, and rays that miss it: the forward stops a ray once it
    has left the grid for good and the backward skips such chunks, which must
    not change any output."""
    rng = np.random.Generator(np.random.PCG64(71))
    grid = synth.Grid(lo=(-2.0, -2.0, -1.0), voxel=0.25, dims=(16, 16, 8), nv=3)
    means = rng.uniform((-1.8, -1.8, -0.8), (1.8, 1.8, 0.8), (40, 3))
    prims = synth.make_prims(rng, means, 0.1, 0.5, 4)
    prims.opacity[:] = (prims.opacity * 0.3).astype(np.float32)
    rays = synth.pinhole_rig(1, 24, 20, 100.0, cam, yaw0_deg=yaw, pitch_deg=pitch)
    sc = synth.Scene(grid, prims, rays, synth.March(90, 0.1, 14.0), name="in-out")
    _say("rays entering and leaving", cam, yaw, pitch)
    g_d, g_s = synth.upstream_grads(np.random.default_rng(71), sc.rays, 4)
    out, g = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=4, tuning=api.Tuning(8, 2))
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    assert np.count_nonzero(ref["depth"] > 0) > 0
    H.assert_depth_close(out["depth"], ref["depth"], "in-out")
    H.assert_probs_close(out["probs"], ref["probs"], "in-out")
    H.assert_tfinal_close(out["t_final"], ref["t_final"], "in-out")
    H.assert_grads_close(g, oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s), "in-out")
    # the checkpoints still hold T at every chunk start after a ray has left
    ck = out["ckpt"]
    assert np.all(np.diff(ck, axis=0) <= 0)
    assert np.all(ck[-1] >= out["t_final"].reshape(-1))


def test_config2_gradients_against_central_differences():
    """Config 2 asks for central differences on 200 random visible parameters.
    Upstream gradients sit on 64 rays only, so each difference renders just those
    rays with the FP64 oracle (h = 1e-4); the GPU gradient must match within
    1e-3 |g| + 1e-3 rms(g) of its group.  A parameter whose difference changes
    between h and h/2 straddles a kink (the alpha clamp, a list change) and is
    skipped, as is a centre moved into another voxel."""
    sc = synth.config(2)
    C = sc.prims.n_classes
    rng = np.random.default_rng(9)
    ids = rng.choice(sc.rays.n_rays, 64, replace=False)
    g_d = np.zeros(sc.rays.n_rays, np.float32)
    g_s = np.zeros((sc.rays.n_rays, C), np.float32)
    g_d[ids] = rng.standard_normal(ids.size).astype(np.float32)
    g_s[ids] = rng.standard_normal((ids.size, C)).astype(np.float32)
    cams, Hh, Ww = sc.rays.shape
    _say("config2 central differences")
    _, g = H.run_fwd_bwd(sc, g_d.reshape(cams, Hh, Ww),
                         g_s.reshape(cams, Hh, Ww, C).transpose(0, 3, 1, 2).copy(), tuning=api.Tuning(8, 2))
    index = oracle.build_index(sc.prims, sc.grid)[:3]
    names = ("means", "quats", "scales", "eps", "opacity", "logits")
    base = {k: np.asarray(getattr(sc.prims, k), np.float64) for k in names}
    rms = {k: float(np.sqrt(np.mean(np.square(g[k].astype(np.float64))))) for k in names}
    cand = [(k, i) for k in names for i in np.flatnonzero(np.abs(g[k].reshape(-1)) > 1e-3 * rms[k])]
    pick = [cand[i] for i in rng.choice(len(cand), 200, replace=False)]
    inv = np.float32(1.0) / np.float32(sc.grid.voxel)
    lo = np.asarray(sc.grid.lo, np.float32)

    def loss(name, i, dx):
        arrs = {k: base[k].copy() for k in names}
        arrs[name].reshape(-1)[i] += dx
        pr = synth.Prims(*(arrs[k] for k in names))
        out = oracle.render(sc.grid, pr, sc.rays, sc.march, index=index, ray_ids=ids)
        return oracle.loss_value(out, g_d[ids], g_s[ids])

    def cell(m):
        return np.floor((np.float32(m) - lo) * inv)

    h = 1e-4
    checked = 0
    for name, i in pick:
        if name == "means":
            k, ax = divmod(int(i), 3)
            m = base["means"][k, ax]
            if cell(m + h)[ax] != cell(m - h)[ax] or cell(m + h)[ax] != cell(m)[ax]:
                continue
        fd = (loss(name, i, h) - loss(name, i, -h)) / (2 * h)
        fd2 = (loss(name, i, h / 2) - loss(name, i, -h / 2)) / h
        if abs(fd - fd2) > 1e-4 * abs(fd) + 1e-6 * rms[name]:
            continue
        got = float(g[name].reshape(-1)[i])
        assert abs(got - fd) <= 1e-3 * abs(fd) + 1e-3 * rms[name], (name, int(i), got, fd)
        checked += 1
    assert checked >= 180, checked

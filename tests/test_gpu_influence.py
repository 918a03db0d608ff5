"""GPU parity of the influence-thresholded index (grid.theta; reading R21,
the occupancy-aware indexing of the Supplement's future work): the index is
bit-exact against the oracle's, and the renders, gradients and voxel grids
built on it match the oracle run on the same thresholded lists."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.scenes_small import random_scene

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_17361_amd import api
    from tests import gpu_helpers as H


def _say(*a):
    print(*a, flush=True)


def _theta(sc, theta):
    return dataclasses.replace(sc, grid=dataclasses.replace(sc.grid, theta=theta))


def _index_equal(sc):
    grid, prims, _, _ = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    torch.cuda.synchronize()
    e = idx.checked_total()
    c, o, i, t = oracle.build_index(sc.prims, sc.grid)
    assert e == t
    np.testing.assert_array_equal(idx.counts.cpu().numpy(), c)
    np.testing.assert_array_equal(idx.offsets.cpu().numpy(), o)
    np.testing.assert_array_equal(idx.ids[:e].cpu().numpy(), i)
    return e


@pytest.mark.parametrize("theta", [1e-6, 1e-3, 0.05, 0.6])
def test_index_bitexact_with_theta(theta):
    _say("influence index", theta)
    sc = _theta(random_scene(60, n=120, nv=4, dims=(24, 20, 10), voxel=0.5, lo=(-6.0, -5.0, -2.5)), theta)
    e = _index_equal(sc)
    assert e < oracle.box_volume_total(sc.prims.means, sc.grid)


def test_index_bitexact_with_theta_config1():
    sc = _theta(synth.config(1), 1e-3)
    _say("influence index config1")
    e = _index_equal(sc)
    assert e < oracle.box_volume_total(sc.prims.means, sc.grid)


@pytest.mark.parametrize("seed,C,theta", [(61, 4, 1e-3), (62, 17, 2e-2)])
def test_render_and_grads_with_theta(seed, C, theta):
    _say("influence render", seed, C, theta)
    sc = _theta(random_scene(seed, n=40, n_classes=C, nv=4, width=31, height=19, n_samples=41, opacity_hi=0.9,
                             dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0), theta)
    rng = np.random.default_rng(seed)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, C)
    out, got = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=4)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    H.assert_depth_close(out["depth"], ref["depth"], "theta depth")
    H.assert_probs_close(H.flat_sem(out["probs"]), H.flat_sem(ref["probs"]), "theta probs")
    H.assert_tfinal_close(out["t_final"], ref["t_final"], "theta t_final")
    gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close(got, gref, f"theta grads seed{seed}")
    # the thresholded render is a different (smaller) sum than the full one
    full = oracle.render(dataclasses.replace(sc.grid, theta=0.0), sc.prims, sc.rays, sc.march)
    assert np.max(np.abs(full["depth"] - ref["depth"])) > 0


def test_theta_zero_is_the_plain_index():
    sc = random_scene(63, n=30, n_classes=5, nv=4, width=21, height=13, n_samples=33, opacity_hi=0.9,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    a, _ = H.run_fwd(sc, ckpt_every=4)
    b, _ = H.run_fwd(_theta(sc, 0.0), ckpt_every=4)
    for k in ("depth", "sem", "t_final", "ckpt"):
        assert np.array_equal(a[k], b[k]), k


def test_voxelise_with_theta():
    sc = _theta(random_scene(64, n=40, n_classes=5, nv=3, dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0),
                             opacity_hi=0.9), 1e-3)
    grid, prims, _, _ = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    vx = api.voxelise(grid, idx, prims, tau=0.05)
    torch.cuda.synchronize()
    d = oracle.voxelise(sc.grid, sc.prims)["density"]
    np.testing.assert_allclose(vx["density"].cpu().numpy().reshape(-1), np.asarray(d).reshape(-1),
                               rtol=1e-4, atol=1e-6)


def test_batch_with_theta_matches_oracle_and_single_scene():
    scs = [_theta(random_scene(65 + i, n=n, n_classes=5, width=19, height=13, n_samples=29, opacity_hi=0.8,
                               dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0), 1e-3)
           for i, n in enumerate((23, 0, 11))]
    _say("influence batch")
    grid = api.Grid.of(scs[0].grid)
    march = api.March(scs[0].march.n_samples, scs[0].march.t_near, scs[0].march.t_far, 4)
    b = api.Batch(grid, march, [(api.Prims.from_numpy(s.prims), api.Rays.from_numpy(s.rays)) for s in scs])
    b.build_index()
    b.render_fwd(api.Tuning(8, 2))
    torch.cuda.synchronize()
    for i, sc in enumerate(scs):
        c, _, _, t = oracle.build_index(sc.prims, sc.grid)
        V = sc.grid.n_voxels
        np.testing.assert_array_equal(b.buf["counts"][i * V:(i + 1) * V].cpu().numpy(), c)
        out = {k: v.cpu().numpy() for k, v in b.scene_outputs(i).items()}
        single, _ = H.run_fwd(sc, tuning=api.Tuning(8, 2))
        for k in ("depth", "sem", "t_final"):
            assert np.array_equal(out[k], single[k]), (i, k)

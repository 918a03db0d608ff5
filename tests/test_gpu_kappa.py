"""GPU parity of early ray termination (march.kappa; Supplement "Ray
Termination") against the FP64 oracle.

Where a ray stops is an integer decided by floating point (T_j against
kappa).  Rays whose oracle transmittances all stay more than 1e-3 (relative)
away from kappa are compared with the usual forward tolerances; the rest must
lie between the oracle renders at kappa (1 + 2e-3) and kappa (1 - 2e-3) (depth
is monotone in kappa), i.e. be a valid truncation.  Gradients are compared
with upstream gradients that vanish on the near-threshold rays."""
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

CLEAR = 1e-3


def _say(*a):
    print(*a, flush=True)


def _kappa_scene(sc, kappa, K=4):
    return dataclasses.replace(sc, march=dataclasses.replace(sc.march, kappa=kappa, ckpt_every=K))


def _check_fwd(sc, out, what, ray_ids=None):
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, ray_ids=ray_ids)
    dep = out["depth"].reshape(-1) if ray_ids is None else out["depth"].reshape(-1)[ray_ids]
    prb = H.flat_sem(out["probs"]) if ray_ids is None else H.flat_sem(out["probs"])[ray_ids]
    tfn = out["t_final"].reshape(-1) if ray_ids is None else out["t_final"].reshape(-1)[ray_ids]
    clear = ref["kappa_margin"].reshape(-1) > CLEAR
    rd = ref["depth"].reshape(-1)
    H.assert_depth_close(dep[clear], rd[clear], what)
    H.assert_probs_close(prb[clear], H.flat_sem(ref["probs"])[clear] if ray_ids is None else ref["probs"][clear],
                         what)
    H.assert_tfinal_close(tfn[clear], ref["t_final"].reshape(-1)[clear], what)
    amb = ~clear
    if amb.any():
        k = sc.march.kappa
        lo = oracle.render(sc.grid, sc.prims, sc.rays, dataclasses.replace(sc.march, kappa=k * (1 + 2e-3)),
                           ray_ids=ray_ids)["depth"].reshape(-1)[amb]
        hi = oracle.render(sc.grid, sc.prims, sc.rays, dataclasses.replace(sc.march, kappa=k * (1 - 2e-3)),
                           ray_ids=ray_ids)["depth"].reshape(-1)[amb]
        tol = 1e-4 * np.abs(hi) + 1e-5
        assert np.all((dep[amb] >= lo - tol) & (dep[amb] <= hi + tol)), what
    return clear


@pytest.mark.parametrize("kappa", [0.3, 1e-2, 1e-4])
@pytest.mark.parametrize("seed", [90, 91])
def test_kappa_forward_small_scenes(seed, kappa):
    _say("kappa fwd", seed, kappa)
    sc = _kappa_scene(random_scene(seed, n=30, n_classes=5, nv=4, width=37, height=23, n_samples=41,
                                   opacity_hi=0.9, dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0),
                      kappa)
    out, _ = H.run_fwd(sc, ckpt_every=4)
    clear = _check_fwd(sc, out, f"seed{seed} kappa{kappa}")
    assert clear.mean() > 0.9
    if kappa >= 1e-2:
        tf = out["t_final"].reshape(-1)
        assert np.sum((tf > 0) & (tf < kappa)) > 0          # some rays stopped before saturating


def test_kappa_zero_is_bitwise_the_plain_forward():
    sc = random_scene(92, n=30, n_classes=5, nv=4, width=21, height=13, n_samples=33, opacity_hi=0.9,
                      dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
    a, _ = H.run_fwd(sc, ckpt_every=4)
    b, _ = H.run_fwd(_kappa_scene(sc, 0.0), ckpt_every=4)
    for k in ("depth", "sem", "t_final", "ckpt"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("K,mode", [(4, 2), (8, 2), (4, 1), (16, 1)])
def test_kappa_backward_matches_oracle(K, mode):
    _say("kappa bwd", K, mode)
    sc = _kappa_scene(random_scene(93, n=25, n_classes=4, nv=4, width=29, height=17, n_samples=37, opacity_hi=0.9,
                                   dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0), 2e-2, K)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    clear = ref["kappa_margin"] > CLEAR
    rng = np.random.default_rng(K)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, sc.prims.n_classes)
    g_d = np.where(clear, g_d, 0.0).astype(np.float32)
    g_s = np.where(clear[:, None], g_s, 0.0).astype(np.float32)
    out, got = H.run_fwd_bwd(sc, g_d, g_s, ckpt_every=K, tuning=api.Tuning(8, 4, mode, 1, 0))
    _check_fwd(sc, out, f"kappa bwd fwd K{K}")
    gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close(got, gref, f"kappa K{K} mode{mode}")
    tf = out["t_final"].reshape(-1)
    assert np.sum((tf > 0) & (tf < 2e-2)) > 0


def test_kappa_config1_sampled_rays():
    sc = _kappa_scene(synth.config(1), 1e-2)
    _say("kappa config1")
    out, _ = H.run_fwd(sc, ckpt_every=4)
    ids = np.random.default_rng(5).choice(sc.rays.n_rays, 2000, replace=False)
    _check_fwd(sc, out, "cfg1 kappa", ray_ids=ids)


@pytest.mark.parametrize("K", [4, 8])
def test_kappa_backward_with_the_stash_matches_oracle(K):
    """Early termination with the per-sample stash (the one-scene training
    path with an api.StashPool): the backward's transmittance recursion from
    the stashed a_j stops where the forward stopped; gradients on the rays
    clear of the kappa boundary match the oracle."""
    _say("kappa bwd with the stash", K)
    sc = _kappa_scene(random_scene(94, n=25, n_classes=4, nv=4, width=29, height=17, n_samples=37, opacity_hi=0.9,
                                   dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0), 2e-2, K)
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    clear = ref["kappa_margin"] > CLEAR
    rng = np.random.default_rng(10 + K)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, sc.prims.n_classes)
    g_d = np.where(clear, g_d, 0.0).astype(np.float32)
    g_s = np.where(clear[:, None], g_s, 0.0).astype(np.float32)
    grid, prims, rays, march = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    pool = api.StashPool()
    st = api.render_train_fwd(grid, idx, prims, rays, march, ckpt_every=K, tuning=api.Tuning(8, 4, 2, 1, K),
                              stash=pool)
    g = api.render_train_bwd(st, torch.from_numpy(g_d).cuda(), torch.from_numpy(g_s).cuda())
    torch.cuda.synchronize()
    head = pool.buf[:16].view(torch.int32).cpu().tolist()
    assert head[3] == 1 and 0 < head[4] <= head[5], head
    gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close({k: v.cpu().numpy() for k, v in g.items()}, gref, f"kappa with stash K{K}")
    tf = st["t_final"].cpu().numpy().reshape(-1)
    assert np.sum((tf > 0) & (tf < 2e-2)) > 0

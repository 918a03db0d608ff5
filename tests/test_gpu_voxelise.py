"""GPU parity of superquadric voxelisation (sq_voxelise / sq_batch_voxelise,
Eq. eq:voxelisation) against the FP64 oracle.

Density and semantic voxels: within 1e-4 relative + 1e-6 absolute (density)
and 1e-4 relative + 1e-4 absolute (semantics, whose sums mix signs).  Labels
are an integer decided by floating point: the kernel's label must equal the
label rule applied to the kernel's own float32 outputs, bit for bit, and must
equal the oracle's label wherever the decision is not within the tolerance
of a tie (|density - tau| and the top-two class gap)."""
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

D_REL, D_ABS = 1e-4, 1e-6
S_REL, S_ABS = 1e-4, 1e-4


def _say(*a):
    print(*a, flush=True)


def _run(sc, tau=0.05):
    grid, prims, _, _ = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    out = api.voxelise(grid, idx, prims, tau=tau)
    torch.cuda.synchronize()
    idx.checked_total()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _flat(out, C):
    return out["density"].reshape(-1), out["sem"].reshape(C, -1).T, out["labels"].reshape(-1)


def _check(got, ref, tau, what, vids=None):
    C = ref["sem"].shape[1]
    d, s, lab = _flat(got, C)
    if vids is not None:
        d, s, lab = d[vids], s[vids], lab[vids]
    rd, rs, rl = ref["density"], ref["sem"], ref["labels"]
    err = np.abs(d - rd)
    assert np.all(err <= D_REL * np.abs(rd) + D_ABS), f"{what} density worst {err.max():.3e}"
    err = np.abs(s - rs)
    assert np.all(err <= S_REL * np.abs(rs) + S_ABS), f"{what} sem worst {err.max():.3e}"
    # the kernel's labels follow the rule on its own float32 outputs exactly
    np.testing.assert_array_equal(lab, oracle.labels_from(d, s, np.float32(tau)), err_msg=what)
    # and match the oracle where the decision is clear of the tolerance band
    srt = np.sort(rs, axis=1)
    gap = srt[:, -1] - srt[:, -2] if C > 1 else np.full(rd.shape, np.inf)
    clear = (np.abs(rd - tau) > D_REL * np.abs(rd) + D_ABS) & (gap > 2 * (S_REL * np.abs(srt[:, -1]) + S_ABS))
    clear |= rd < tau - (D_REL * np.abs(rd) + D_ABS)
    # voxels with nothing listed: all-zero sums on both sides, an exact tie both resolve to class 0
    clear |= np.all(rs == 0, axis=1) & np.all(s == 0, axis=1)
    np.testing.assert_array_equal(lab[clear], rl[clear], err_msg=what)
    assert clear.mean() > 0.9, f"{what}: only {clear.mean():.2f} of the labels are clear of ties"


@pytest.mark.parametrize("seed,n,C,nv,dims", [(50, 30, 5, 2, (13, 11, 7)), (51, 60, 17, 5, (16, 16, 8)),
                                              (52, 12, 1, 0, (9, 9, 9)), (53, 45, 20, 3, (5, 17, 6))])
def test_voxelise_small_grids(seed, n, C, nv, dims):
    _say("voxelise small", seed, n, C, nv, dims)
    sc = random_scene(seed, n=n, n_classes=C, nv=nv, dims=dims, voxel=0.5, lo=(-3.0, -3.0, -2.0),
                      scale_lo=0.2, scale_hi=0.9, opacity_hi=0.8)
    got = _run(sc)
    ref = oracle.voxelise(sc.grid, sc.prims, tau=0.05)
    _check(got, ref, 0.05, f"seed{seed}")


def test_voxelise_config4_sampled_voxels():
    """25.6k superquadrics on the 200x200x16 grid: random voxels plus one
    whole column block, against the oracle voxel by voxel."""
    sc = synth.config(4)
    _say("voxelise config4")
    got = _run(sc)
    g = sc.grid
    rng = np.random.default_rng(7)
    vids = rng.choice(g.n_voxels, 1500, replace=False)
    blk = ((np.arange(96, 104)[:, None, None] * g.dims[1] + np.arange(100, 108)[None, :, None]) * g.dims[2]
           + np.arange(16)[None, None, :]).reshape(-1)
    vids = np.unique(np.concatenate([vids, blk]))
    ref = oracle.voxelise(g, sc.prims, tau=0.05, voxel_ids=vids)
    _check(got, ref, 0.05, "cfg4", vids=vids)
    assert (ref["labels"] < sc.prims.n_classes).mean() > 0.05       # the sample holds occupied voxels


def test_voxelise_without_bitmap_matches_oracle():
    """600k primitives: the per-wave bitmap exceeds the LDS budget even at one
    wave per block, so every lane walks its own list."""
    sc = random_scene(54, n=600_000, n_classes=3, nv=1, dims=(24, 24, 12), voxel=0.5, lo=(-6.0, -6.0, -3.0),
                      scale_lo=0.02, scale_hi=0.08, opacity_hi=0.6)
    _say("voxelise 600k prims (no bitmap)")
    got = _run(sc)
    vids = np.random.default_rng(8).choice(sc.grid.n_voxels, 240, replace=False)
    parts = [oracle.voxelise(sc.grid, sc.prims, tau=0.05, voxel_ids=vids[i:i + 12], brute=True)
             for i in range(0, vids.size, 12)]
    ref = {k: np.concatenate([p[k] for p in parts]) for k in ("density", "sem", "labels")}
    _check(got, ref, 0.05, "600k", vids=vids)


def test_voxelise_edge_cases():
    _say("voxelise edge: empty scene")
    sc = random_scene(55, n=0, n_classes=4, dims=(7, 6, 5))
    got = _run(sc)
    assert np.all(got["density"] == 0) and np.all(got["sem"] == 0) and np.all(got["labels"] == 4)
    _say("voxelise edge: tau = 0 labels every voxel by argmax")
    sc = random_scene(56, n=20, n_classes=3, nv=2, dims=(10, 10, 6), voxel=0.5, lo=(-2.5, -2.5, -1.5))
    got = _run(sc, tau=0.0)
    assert np.all(got["labels"] < 3)
    ref = oracle.voxelise(sc.grid, sc.prims, tau=0.0)
    _check(got, ref, 0.0, "tau0")


def test_batch_voxelise_equals_single_scene_calls():
    scenes = [random_scene(60 + i, n=n, n_classes=5, nv=3, dims=(12, 10, 6), voxel=0.5, lo=(-3.0, -2.5, -1.5),
                           width=9, height=7) for i, n in enumerate((25, 0, 40, 7))]
    _say("batch voxelise")
    grid = api.Grid.of(scenes[0].grid)
    march = api.March(scenes[0].march.n_samples, scenes[0].march.t_near, scenes[0].march.t_far, 4)
    b = api.Batch(grid, march, [(api.Prims.from_numpy(s.prims), api.Rays.from_numpy(s.rays)) for s in scenes])
    b.build_index()
    b.voxelise(tau=0.05)
    torch.cuda.synchronize()
    for i, sc in enumerate(scenes):
        single = _run(sc)
        mine = {k: v.cpu().numpy() for k, v in b.scene_voxels(i).items()}
        for k in ("density", "sem", "labels"):
            assert np.array_equal(mine[k], single[k]), (i, k)

"""GPU tests of the batched form: several scenes with uneven primitive and
camera counts in single launches (static and persistent tile scheduling), the
hipGraph-captured step and the autotuner.  Each scene of a batch must match
its own single-scene render (forward bit for bit: the same tile code runs) and
the FP64 oracle."""
import ctypes as ct

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


def _small_batch(seed=60, ns=(5, 0, 23, 11), sizes=((19, 13), (7, 5), (33, 9), (16, 16)), C=5):
    scenes = []
    for i, (n, (w, h)) in enumerate(zip(ns, sizes)):
        sc = random_scene(seed + i, n=n, n_classes=C, width=w, height=h, n_samples=29, opacity_hi=0.8,
                          dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)
        scenes.append(sc)
    return scenes


def _make_batch(scenes, K=4, probs=True):
    grid = api.Grid.of(scenes[0].grid)
    march = api.March(scenes[0].march.n_samples, scenes[0].march.t_near, scenes[0].march.t_far, K)
    dev = [(api.Prims.from_numpy(s.prims), api.Rays.from_numpy(s.rays)) for s in scenes]
    return api.Batch(grid, march, dev, probs=probs)


def _upstream(scenes, seed):
    rng = np.random.default_rng(seed)
    return [synth.upstream_grads(rng, s.rays, s.prims.n_classes) for s in scenes]


@pytest.mark.parametrize("tune", [api.Tuning(8, 4, 0, 0, 0), api.Tuning(4, 2, 0, 1, 0), api.Tuning(16, 1, 2, 1, 8),
                                  api.Tuning(8, 4, 1, 0, 16)] if torch.cuda.is_available() else [None])
def test_batch_matches_single_scenes_and_oracle(tune):
    scenes = _small_batch()
    _say("batch small", tune)
    b = _make_batch(scenes)
    ups = _upstream(scenes, 1)
    for i, (gd, gs) in enumerate(ups):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    b.build_index()
    b.render_fwd(tune)
    b.render_bwd(tune)
    torch.cuda.synchronize()
    totals = b.buf["totals"].cpu().numpy()
    K = tune.chunk or 4
    for i, sc in enumerate(scenes):
        out = {k: v.cpu().numpy() for k, v in b.scene_outputs(i).items()}
        # index of this scene
        c, o, ids, t = oracle.build_index(sc.prims.means, sc.grid)
        assert totals[i] == t
        n0, n, r0, cams, Hh, Ww = b.scene_slices(i)
        V = sc.grid.n_voxels
        np.testing.assert_array_equal(b.buf["counts"][i * V:(i + 1) * V].cpu().numpy(), c)
        np.testing.assert_array_equal(b.buf["offsets"][i * V:(i + 1) * V].cpu().numpy(), o)
        base = sum(b.caps[:i])
        np.testing.assert_array_equal(b.buf["ids"][base:base + t].cpu().numpy(), ids)
        # single-scene render with the same tuning: forward bit for bit
        single, _ = H.run_fwd(sc, tuning=api.Tuning(tune.tile_w, tune.waves_per_block))
        for k in ("depth", "sem", "t_final", "probs"):
            assert np.array_equal(out[k], single[k]), (i, k)
        ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
        H.assert_depth_close(out["depth"], ref["depth"], f"scene {i}")
        H.assert_probs_close(out["probs"], ref["probs"], f"scene {i}")
        gd, gs = ups[i]
        gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, gd, gs)
        got = {k: out["g_" + k] for k in ("means", "quats", "scales", "eps", "opacity", "logits")}
        if sc.prims.n:
            H.assert_grads_close(got, gref, f"scene {i} K{K}")


def test_persistent_forward_is_bitwise_static_forward():
    scenes = _small_batch(seed=70)
    b = _make_batch(scenes)
    b.build_index()
    b.render_fwd(api.Tuning(8, 4, 0, 0, 0))
    torch.cuda.synchronize()
    a = {k: b.buf[k].clone() for k in ("depth", "sem", "t_final")}
    b.render_fwd(api.Tuning(8, 4, 0, 1, 0))
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b.buf[k]), k


def test_graph_replays_match_eager_step():
    scenes = _small_batch(seed=80)
    b = _make_batch(scenes)
    for i, (gd, gs) in enumerate(_upstream(scenes, 2)):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    tune = api.Tuning(8, 4, 0, 1, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.step(tune, stream=s)
    torch.cuda.synchronize()
    eager = {k: b.buf[k].clone() for k in ("depth", "sem", "t_final", "ckpt", "g_means", "g_logits", "g_opacity")}
    b.capture(tune, stream=s)
    for rep in range(3):
        # clobber outputs and run unrelated eager work between replays
        for k in eager:
            b.buf[k].fill_(-7.0)
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        b.replay(stream=s)
        torch.cuda.synchronize()
        for k in ("depth", "sem", "t_final", "ckpt"):
            assert torch.equal(eager[k], b.buf[k]), (rep, k)
        for k in ("g_means", "g_logits", "g_opacity"):
            torch.testing.assert_close(b.buf[k], eager[k], rtol=1e-4, atol=1e-5)
        del junk
    b.release_graph()


def test_autotune_returns_a_timed_candidate():
    scenes = _small_batch(seed=90)
    b = _make_batch(scenes)
    cands = [api.Tuning(8, 4, 0, 0, 4), api.Tuning(16, 2, 0, 1, 8), api.Tuning(4, 4, 1, 0, 16)]
    best, ms = b.autotune(cands, reps=2)
    assert best in cands and len(ms) == 3 and all(m > 0 for m in ms)
    assert ms[cands.index(best)] == min(ms)


def test_autotune_cache_round_trip(tmp_path):
    """The cached autotuner times the candidates once and appends the winner
    under the batch's key; the next call on the same workload reads it back
    without timing, and another workload misses the cache."""
    scenes = _small_batch(seed=91)
    b = _make_batch(scenes)
    cands = [api.Tuning(8, 4, 0, 0, 4), api.Tuning(16, 2, 0, 1, 8)]
    path = tmp_path / "tuning.txt"
    best, hit = b.autotune_cached(cands, path, reps=1)
    assert not hit and best in cands
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith(b.tuning_key() + " => ")
    again, hit = b.autotune_cached(cands, path, reps=1)
    assert hit and again == best
    other = _make_batch(_small_batch(seed=91, ns=(5, 0, 23, 12)))
    assert other.tuning_key() != b.tuning_key()
    third, hit = other.autotune_cached(cands, path, reps=1)
    assert not hit and third in cands and len(path.read_text().splitlines()) == 2


def test_batch_rejects_bad_tuning_without_launch():
    scenes = _small_batch(seed=95)
    b = _make_batch(scenes)
    with pytest.raises(Exception, match="status -1"):
        b.render_fwd(api.Tuning(tile_w=5))
    with pytest.raises(Exception, match="status -1"):
        b.render_bwd(api.Tuning(chunk=3))


def test_config3_batch_equals_single_scene_renders():
    """Config 3 workload: 8 scenes, {2k..25.6k} superquadrics, 6 cameras at
    352x200 each, L=100, one persistent batched step.  Each scene's forward
    equals its single-scene render bit for bit and the oracle on 400 sampled
    rays; every scene carries sparse upstream gradients (200 rays), so each
    scene's batched gradients -- computed at non-zero primitive, ray and id
    offsets through the shared work queues -- are compared with the oracle's
    over exactly those rays."""
    scenes = [synth.config(3, s) for s in range(8)]
    _say("config3 batch")
    b = _make_batch(scenes)
    picks = []
    for i, sc in enumerate(scenes):
        rng = np.random.default_rng(300 + i)
        C = sc.prims.n_classes
        ids = np.sort(rng.choice(sc.rays.n_rays, 200, replace=False))
        gd = np.zeros(sc.rays.n_rays, np.float32)
        gs = np.zeros((sc.rays.n_rays, C), np.float32)
        gd[ids] = rng.standard_normal(ids.size)
        gs[ids] = rng.standard_normal((ids.size, C))
        picks.append((ids, gd[ids].copy(), gs[ids].copy()))
        cams, Hh, Ww = sc.rays.shape
        b.set_upstream(i, torch.from_numpy(gd.reshape(cams, Hh, Ww)).cuda(),
                       torch.from_numpy(gs.reshape(cams, Hh, Ww, -1).transpose(0, 3, 1, 2).copy()).cuda())
    tune = api.Tuning(8, 4, 0, 1, 4)
    b.step(tune)
    torch.cuda.synchronize()
    for i, sc in enumerate(scenes):
        _say(f"config3 scene {i}: {sc.prims.n} superquadrics")
        out = {k: v.cpu().numpy() for k, v in b.scene_outputs(i).items()}
        single, _ = H.run_fwd(sc)
        for k in ("depth", "sem", "t_final"):
            assert np.array_equal(out[k], single[k]), (i, k)
        index = oracle.build_index(sc.prims, sc.grid)[:3]
        ids, gd, gs = picks[i]
        extra = np.random.default_rng(i).choice(sc.rays.n_rays, 200, replace=False)
        rid = np.union1d(ids, extra)
        ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, index=index, ray_ids=rid)
        H.assert_depth_close(out["depth"].reshape(-1)[rid], ref["depth"], f"cfg3 scene {i}")
        H.assert_probs_close(H.flat_sem(out["probs"])[rid], ref["probs"], f"cfg3 scene {i}")
        gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, gd, gs, index=index, ray_ids=ids)
        got = {k: out["g_" + k] for k in ("means", "quats", "scales", "eps", "opacity", "logits")}
        H.assert_grads_close(got, gref, f"cfg3 scene {i}")


def test_backward_after_a_forward_with_another_chunk_writes_nan():
    """The checkpoint rows are laid out by the forward's chunk.  A backward
    with another chunk cannot be refused on the host (the record of the
    forward's chunk is on the device), so its gradients are NaN; with the
    forward's chunk they are finite and equal those of a fresh step."""
    scenes = _small_batch(seed=97)
    b = _make_batch(scenes)
    for i, (gd, gs) in enumerate(_upstream(scenes, 98)):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    b.build_index()
    _say("chunk mismatch: forward K=8, backward K=4")
    b.render_fwd(api.Tuning(8, 2, 0, 1, 8))
    b.render_bwd(api.Tuning(8, 2, 0, 1, 4))
    torch.cuda.synchronize()
    for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
        assert torch.isnan(b.buf["g_" + k]).all(), k
    _say("chunk match: forward K=8, backward K=8")
    b.render_bwd(api.Tuning(8, 2, 0, 1, 8))
    torch.cuda.synchronize()
    for k in ("means", "quats", "scales", "eps", "opacity", "logits"):
        assert torch.isfinite(b.buf["g_" + k]).all(), k


@pytest.fixture(scope="module")
def bench_workload():
    """The bench's workload and the oracle's index of it (built once)."""
    sc = synth.config(4)
    return sc, oracle.build_index(sc.prims, sc.grid)[:3]


BENCH_TUNINGS = [(16, 2, 8), (8, 2, 8), (8, 2, 4)]


@pytest.mark.parametrize("tw,wpb,K", BENCH_TUNINGS)
def test_bench_workload_step_gradients_on_sampled_rays(bench_workload, tw, wpb, K):
    """The bench's workload (6 x 1600x900 rays, 25.6k superquadrics, L = 200)
    in the launch configurations its autotuner picks among (tile 16x4 or 8x8,
    2 waves per block, primitive-major backward, persistent, chunk 8 or 4)
    through a captured step replay.  Upstream gradients are non-zero on 400
    rays only, so the oracle's gradients over those rays are exact; the
    forward is checked on them too."""
    sc, index = bench_workload
    C = sc.prims.n_classes
    rng = np.random.default_rng(44)
    ids = rng.choice(sc.rays.n_rays, 400, replace=False)
    g_d = np.zeros(sc.rays.n_rays, np.float32)
    g_s = np.zeros((sc.rays.n_rays, C), np.float32)
    g_d[ids] = rng.standard_normal(ids.size).astype(np.float32)
    g_s[ids] = rng.standard_normal((ids.size, C)).astype(np.float32)
    cams, Hh, Ww = sc.rays.shape
    b = _make_batch([sc], K=K)
    b.set_upstream(0, torch.from_numpy(g_d.reshape(cams, Hh, Ww)).cuda(),
                   torch.from_numpy(g_s.reshape(cams, Hh, Ww, C).transpose(0, 3, 1, 2).copy()).cuda())
    tune = api.Tuning(tw, wpb, 0, 1, K)
    _say(f"bench workload step, sampled rays, tile {tw}, {wpb} waves per block, chunk {K}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.step(tune, stream=s)
    torch.cuda.synchronize()
    b.capture(tune, stream=s)
    b.replay(stream=s)
    torch.cuda.synchronize()
    b.release_graph()
    out = {k: v.cpu().numpy() for k, v in b.scene_outputs(0).items()}
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, index=index, ray_ids=ids)
    H.assert_depth_close(out["depth"].reshape(-1)[ids], ref["depth"], "bench workload")
    H.assert_probs_close(H.flat_sem(out["probs"])[ids], ref["probs"], "bench workload")
    gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d[ids], g_s[ids], index=index, ray_ids=ids)
    got = {k: out["g_" + k] for k in ("means", "quats", "scales", "eps", "opacity", "logits")}
    H.assert_grads_close(got, gref, "bench workload")


def test_tile_stops_used_and_ignored():
    """The forward records where each tile stopped; a backward with the same
    tiling skips the samples past it, one with another tiling ignores the
    record.  Both give the oracle's gradients, and the record's header names the
    forward's tiling and march."""
    scenes = _small_batch(seed=95, ns=(30, 12, 40), sizes=((24, 16), (9, 7), (16, 16)))
    b = _make_batch(scenes)
    ups = _upstream(scenes, 96)
    for i, (gd, gs) in enumerate(ups):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    b.build_index()
    _say("tile stops: same tiling")
    b.render_fwd(api.Tuning(8, 2, 0, 1, 4))
    b.render_bwd(api.Tuning(8, 2, 2, 1, 4))
    torch.cuda.synchronize()
    head = b.buf["tile_stop"][:4].cpu().tolist()
    assert head == [8, scenes[0].march.n_samples, 4, 1], head
    L = scenes[0].march.n_samples
    stops = b.buf["tile_stop"][4:].cpu().numpy()
    assert np.any(stops < L - 1), "some tile must stop early (opaque or out of the grid)"
    used = [{k: v.clone() for k, v in b.scene_outputs(i).items() if k.startswith("g_")} for i in range(3)]
    _say("tile stops: other tiling")
    b.render_fwd(api.Tuning(8, 2, 0, 1, 4))
    b.render_bwd(api.Tuning(16, 2, 2, 1, 4))
    torch.cuda.synchronize()
    for i, sc in enumerate(scenes):
        o = b.scene_outputs(i)
        gd, gs = ups[i]
        ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, gd, gs)
        ign = {k[2:]: o[k].cpu().numpy() for k in o if k.startswith("g_")}
        H.assert_grads_close({k[2:]: v.cpu().numpy() for k, v in used[i].items()}, ref, f"scene {i} stops used")
        H.assert_grads_close(ign, ref, f"scene {i} stops ignored")


def _grads(b, n):
    return [{k[2:]: v.cpu().numpy() for k, v in b.scene_outputs(i).items() if k.startswith("g_")} for i in range(n)]


@pytest.mark.parametrize("tw,K,C,ns", [(8, 4, 5, (30, 12, 40)), (16, 8, 5, (30, 12, 40)), (8, 8, 3, (30, 12, 40)),
                                       (16, 8, 17, (30, 12, 40)), (8, 8, 32, (30, 12, 40)), (8, 8, 5, (30, 0, 40))])
def test_stash_backward_matches_recompute_and_oracle(tw, K, C, ns):
    """A forward with checkpoints leaves a_j and the class sums in the stash;
    the backward then skips its first evaluation of each chunk's pairs.  The
    forward's outputs do not change (bit for bit), the slots asked for are one
    per chunk each tile entered, and the gradients match the recomputing
    backward and the oracle, with a full pool and with one that covers a
    third of the chunks (the rest recomputed)."""
    scenes = _small_batch(seed=97, ns=ns, sizes=((24, 16), (9, 7), (16, 16)), C=C)
    b = _make_batch(scenes, K=K)
    ups = _upstream(scenes, 98)
    for i, (gd, gs) in enumerate(ups):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    tune = api.Tuning(tw, 2, 2, 1, K)
    b.build_index()
    _say(f"stash: recompute, tile {tw}, chunk {K}, {C} classes, primitives {ns}")
    b.render_fwd(tune)
    b.render_bwd(tune)
    torch.cuda.synchronize()
    fwd0 = {k: b.buf[k].clone() for k in ("depth", "sem", "probs", "t_final", "ckpt")}
    g0 = _grads(b, 3)
    L = scenes[0].march.n_samples
    stops = b.buf["tile_stop"][4:4 + b.buf["tile_stop"].numel() - 4].cpu().numpy()
    _say("stash: header only, counting")
    b.set_stash(0, tune)
    b.render_fwd(tune)
    torch.cuda.synchronize()
    head = b.buf["stash"][:16].view(torch.int32).cpu().tolist()
    demand = b.stash_demand()
    assert head[:4] == [tw, L, K, 1] and head[5] == 0, head
    n_tiles = int(lib_tiles(b, tw))
    assert demand == int(np.sum(stops[:n_tiles] // K + 1)), (demand, n_tiles)
    for slots, what in ((demand, "full pool"), (demand // 3, "a third")):
        _say(f"stash: {what} ({slots} of {demand} slots)")
        b.set_stash(slots, tune)
        b.render_fwd(tune)
        b.render_bwd(tune)
        torch.cuda.synchronize()
        for k, v in fwd0.items():
            assert torch.equal(b.buf[k], v), (what, k)
        h = b.buf["stash"][:16].view(torch.int32).cpu().tolist()
        assert h[4] == demand and h[5] == slots, h
        g = _grads(b, 3)
        for i, sc in enumerate(scenes):
            if not sc.prims.n:
                continue
            for k in g[i]:
                np.testing.assert_allclose(g[i][k], g0[i][k], rtol=2e-4, atol=1e-5 * (np.abs(g0[i][k]).max() + 1e-30),
                                           err_msg=f"{what} scene {i} {k}")
            gd, gs = ups[i]
            ref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, gd, gs)
            H.assert_grads_close(g[i], ref, f"stash {what} scene {i}")


def lib_tiles(b, tw):
    """Tiles of the batch at tile width tw (the length of its stop table less the header)."""
    from paper_2511_17361_amd import _lib as L
    return L.load().sq_batch_tile_stop_len(ct.byref(b.c_batch), ct.byref(api.Tuning(tile_w=tw).c())) - 4


def test_stash_of_another_tiling_or_of_a_plain_forward_is_ignored():
    """A backward whose tiling differs from the stashing forward's, and one
    after a forward without checkpoints (which marks the stash as not its
    own), recompute; both give the oracle's gradients."""
    scenes = _small_batch(seed=99, ns=(25, 18), sizes=((20, 12), (12, 12)))
    b = _make_batch(scenes, K=4)
    ups = _upstream(scenes, 100)
    for i, (gd, gs) in enumerate(ups):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    b.set_stash(4096)
    b.build_index()
    _say("stash ignored: other tiling")
    b.render_fwd(api.Tuning(8, 2, 2, 1, 4))
    b.render_bwd(api.Tuning(16, 2, 2, 1, 4))
    torch.cuda.synchronize()
    g = _grads(b, 2)
    for i, sc in enumerate(scenes):
        gd, gs = ups[i]
        H.assert_grads_close(g[i], oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, gd, gs), f"other tiling {i}")
    _say("stash marked by a forward without checkpoints")
    ck = b.buf.pop("ckpt")
    b.render_fwd(api.Tuning(8, 2, 2, 1, 4))
    b.buf["ckpt"] = ck
    torch.cuda.synchronize()
    assert b.buf["stash"][:16].view(torch.int32)[3].item() == 0


def test_graph_replays_with_stash_match_eager_step():
    scenes = _small_batch(seed=101)
    b = _make_batch(scenes, K=8)
    for i, (gd, gs) in enumerate(_upstream(scenes, 3)):
        b.set_upstream(i, torch.from_numpy(gd).cuda(), torch.from_numpy(gs).cuda())
    tune = api.Tuning(8, 2, 2, 1, 8)
    b.set_stash(0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.step(tune, stream=s)
    torch.cuda.synchronize()
    b.set_stash(b.stash_demand())
    with torch.cuda.stream(s):
        b.step(tune, stream=s)
    torch.cuda.synchronize()
    eager = {k: b.buf[k].clone() for k in ("depth", "sem", "t_final", "ckpt", "g_means", "g_logits", "g_opacity", "g_eps")}
    # (the checkpoint buffer is sized for chunk 4; chunk 8 writes its first half)
    used = -(-scenes[0].march.n_samples // 8) * b.n_rays
    b.capture(tune, stream=s)
    for rep in range(3):
        for k in eager:
            b.buf[k].fill_(-7.0)
        b.buf["stash"][16:].fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        b.replay(stream=s)
        torch.cuda.synchronize()
        for k in ("depth", "sem", "t_final", "ckpt"):
            n = used if k == "ckpt" else None
            assert torch.equal(eager[k][:n], b.buf[k][:n]), (rep, k)
        for k in ("g_means", "g_logits", "g_opacity", "g_eps"):
            torch.testing.assert_close(b.buf[k], eager[k], rtol=1e-4, atol=1e-5)
        del junk
    b.release_graph()


@pytest.mark.parametrize("tw,wpb,K", BENCH_TUNINGS)
def test_bench_workload_step_with_stash_on_sampled_rays(bench_workload, tw, wpb, K):
    """The bench's workload with the stash sized by a first forward, through a
    captured step replay, against the oracle on 400 rays with upstream
    gradients (the rest zero)."""
    sc, index = bench_workload
    C = sc.prims.n_classes
    rng = np.random.default_rng(45)
    ids = rng.choice(sc.rays.n_rays, 400, replace=False)
    g_d = np.zeros(sc.rays.n_rays, np.float32)
    g_s = np.zeros((sc.rays.n_rays, C), np.float32)
    g_d[ids] = rng.standard_normal(ids.size).astype(np.float32)
    g_s[ids] = rng.standard_normal((ids.size, C)).astype(np.float32)
    cams, Hh, Ww = sc.rays.shape
    b = _make_batch([sc], K=K)
    b.set_upstream(0, torch.from_numpy(g_d.reshape(cams, Hh, Ww)).cuda(),
                   torch.from_numpy(g_s.reshape(cams, Hh, Ww, C).transpose(0, 3, 1, 2).copy()).cuda())
    tune = api.Tuning(tw, wpb, 0, 1, K)
    _say(f"bench workload with stash, tile {tw}, {wpb} waves per block, chunk {K}: sizing forward")
    b.set_stash(0)
    b.build_index()
    b.render_fwd(tune)
    torch.cuda.synchronize()
    demand = b.stash_demand()
    assert demand > 0
    b.set_stash(demand)
    _say(f"bench workload with stash: {demand} slots, {b.buf['stash'].numel() * 4 / 2**30:.2f} GiB; step replay")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.step(tune, stream=s)
    torch.cuda.synchronize()
    b.capture(tune, stream=s)
    b.replay(stream=s)
    torch.cuda.synchronize()
    b.release_graph()
    assert b.stash_demand() == demand
    out = {k: v.cpu().numpy() for k, v in b.scene_outputs(0).items()}
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march, index=index, ray_ids=ids)
    H.assert_depth_close(out["depth"].reshape(-1)[ids], ref["depth"], "bench workload, stash")
    gref = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d[ids], g_s[ids], index=index, ray_ids=ids)
    got = {k: out["g_" + k] for k in ("means", "quats", "scales", "eps", "opacity", "logits")}
    H.assert_grads_close(got, gref, "bench workload, stash")

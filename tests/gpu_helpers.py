"""Helpers for the GPU tests: run the HIP path through the C ABI on a synth
scene and compare with the oracle at the stated tolerances."""
import numpy as np
import torch

from paper_2511_17361_amd import api

# tolerances (FP32 kernel vs FP64 oracle)
DEPTH_REL = 1e-4        # |dD| <= 1e-4 * D_ref for D_ref >= 0.1 m
DEPTH_ABS = 1e-5        # |dD| <= 1e-5 m otherwise
PROB_ABS = 1e-5         # max |d softmax(S)|
GRAD_REL = 1e-3         # per group ||dg|| / ||g_ref||; per element 1e-3 |g_ref| + 1e-3 rms(g_ref)


def gpu_scene(sc, device="cuda"):
    return (api.Grid.of(sc.grid), api.Prims.from_numpy(sc.prims, device), api.Rays.from_numpy(sc.rays, device),
            api.March.of(sc.march))


def run_fwd(sc, ckpt_every=0, tuning=None, stats=False):
    grid, prims, rays, march = gpu_scene(sc)
    idx = api.build_index(grid, prims)
    out = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=ckpt_every, tuning=tuning, stats=stats)
    torch.cuda.synchronize()
    idx.checked_total()
    return {k: v.cpu().numpy() for k, v in out.items()}, idx


def run_fwd_bwd(sc, g_d, g_s, ckpt_every=8, tuning=None):
    grid, prims, rays, march = gpu_scene(sc)
    idx = api.build_index(grid, prims)
    out = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=ckpt_every, tuning=tuning)
    gd = torch.from_numpy(np.ascontiguousarray(g_d, np.float32)).cuda()
    gs = torch.from_numpy(np.ascontiguousarray(g_s, np.float32)).cuda()
    g = api.render_bwd(grid, idx, prims, rays, march, out["ckpt"], ckpt_every, gd, gs, tuning=tuning)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, {k: v.cpu().numpy() for k, v in g.items()}


def assert_depth_close(got, ref, what=""):
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    tol = np.where(ref >= 0.1, DEPTH_REL * ref, DEPTH_ABS)
    err = np.abs(got - ref)
    bad = err > tol
    assert not bad.any(), (f"{what} depth: {bad.sum()} of {bad.size} outside tolerance; "
                           f"worst rel {np.max(err / np.maximum(ref, 0.1)):.3e}")


def assert_probs_close(got, ref, what=""):
    err = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    assert err.max(initial=0) <= PROB_ABS, f"{what} probs max err {err.max():.3e}"


def assert_tfinal_close(got, ref, what=""):
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    err = np.abs(got - ref)
    assert np.all(err <= 1e-5 + 1e-4 * ref), f"{what} t_final max err {err.max():.3e}"


def assert_grads_close(got, ref, what="", exclude=None):
    """Per parameter group: relative L2 <= 1e-3 and per element
    |dg| <= 1e-3 |g_ref| + 1e-3 rms(g_ref).  `exclude` masks primitives whose
    gradient crosses a kink between FP32 and FP64 (clamp decisions)."""
    for name in ("means", "quats", "scales", "eps", "opacity", "logits"):
        g = np.asarray(got[name], np.float64)
        r = np.asarray(ref[name], np.float64)
        if exclude is not None and exclude.any():
            keep = ~exclude
            g, r = g[keep], r[keep]
        nr = np.linalg.norm(r)
        if nr == 0:
            assert np.abs(g).max(initial=0) < 1e-6, f"{what} {name}: expected zero gradient"
            continue
        rel = np.linalg.norm(g - r) / nr
        assert rel <= GRAD_REL, f"{what} {name}: relative L2 error {rel:.3e}"
        rms = np.sqrt(np.mean(r * r))
        err = np.abs(g - r)
        tol = GRAD_REL * np.abs(r) + GRAD_REL * rms
        bad = err > tol
        assert not bad.any(), (f"{what} {name}: {bad.sum()} of {bad.size} elements outside tolerance; "
                               f"worst {np.max(err / tol):.2f}x tol")


def flat_sem(sem):
    """[cams,C,H,W] -> [R,C]."""
    s = np.asarray(sem)
    return s.transpose(0, 2, 3, 1).reshape(-1, s.shape[1])

"""Pins of early ray termination in the oracle (Sec. "Ray Termination"; a ray
stops once its transmittance falls below kappa): kappa = 0 is the plain
render, the kappa render is a prefix of the plain per-sample sums, it is
monotone in kappa, kappa = 1 stops after the first sample with alpha > 0, and
the adjoint matches central differences away from the threshold."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.scenes_small import random_scene


def _with_kappa(march, kappa):
    return dataclasses.replace(march, kappa=kappa)


def _records(sc, march):
    P = oracle.sqr_oracle._Prep(sc.prims)
    idx = oracle.build_index(sc.prims.means, sc.grid)[:3]
    o = sc.rays.origins.reshape(-1, 3)
    d = sc.rays.dirs.reshape(-1, 3)
    return oracle.sqr_oracle._march(sc.grid, sc.prims, o, d, march, idx, False, P, True)


def _scene(seed=30):
    return random_scene(seed, n=20, n_classes=3, width=11, height=8, n_samples=40, opacity_hi=0.9, nv=4,
                        dims=(16, 16, 8), voxel=0.5, lo=(-4.0, -4.0, -2.0), t_far=7.0)


def test_kappa_zero_is_the_plain_render():
    sc = _scene()
    a = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    b = oracle.render(sc.grid, sc.prims, sc.rays, _with_kappa(sc.march, 0.0))
    for k in ("depth", "sem", "t_final"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("kappa", [0.5, 0.1, 1e-2, 1e-4])
def test_kappa_render_is_the_truncated_plain_sum(kappa):
    sc = _scene(31)
    _, _, _, recs, _ = _records(sc, sc.march)
    T = np.stack([r["T"] for r in recs], 1)                       # T_j before sample j (no termination)
    w = np.stack([r["w"] for r in recs], 1)
    t = np.array([r["t"] for r in recs])
    s = np.stack([r["s"] for r in recs], 1)                       # [R, L, C]
    keep = np.cumprod(T >= kappa, axis=1).astype(bool)            # samples before the first T_j < kappa
    want_d = np.sum(np.where(keep, w * t, 0.0), 1)
    want_s = np.sum(np.where(keep[..., None], w[..., None] * s, 0.0), 1)
    last = keep.sum(1)                                            # first dropped sample
    T_ext = np.concatenate([T, (T[:, -1] * (1 - recs[-1]["alpha"]))[:, None]], 1)
    want_t = T_ext[np.arange(T.shape[0]), last]
    r = oracle.render(sc.grid, sc.prims, sc.rays, _with_kappa(sc.march, kappa))
    np.testing.assert_allclose(r["depth"].reshape(-1), want_d, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.sqr_oracle._softmax(want_s), r["probs"].transpose(0, 2, 3, 1).reshape(-1, 3),
                               rtol=1e-12)
    np.testing.assert_allclose(r["t_final"].reshape(-1), want_t, rtol=1e-13, atol=0)
    if kappa >= 1e-2:
        assert (last < T.shape[1]).any()                          # some rays do terminate early


def test_monotone_in_kappa():
    sc = _scene(32)
    prev = None
    for kappa in (0.0, 1e-4, 1e-2, 0.1, 0.5, 0.9):
        r = oracle.render(sc.grid, sc.prims, sc.rays, _with_kappa(sc.march, kappa))
        if prev is not None:
            assert np.all(r["depth"] <= prev["depth"] + 1e-15)
            assert np.all(r["t_final"] >= prev["t_final"] - 1e-15)
        prev = r


def test_kappa_one_stops_after_the_first_sample_that_absorbs():
    """kappa = 1: T stays 1 (>= kappa) until the first sample with alpha > 0,
    which is composited; then T < 1 and the ray stops: D = alpha_j* t_j*."""
    sc = _scene(33)
    _, _, _, recs, _ = _records(sc, sc.march)
    A = np.stack([r["alpha"] for r in recs], 1)
    t = np.array([r["t"] for r in recs])
    first = np.argmax(A > 0, axis=1)
    hit = (A > 0).any(1)
    want = np.where(hit, A[np.arange(A.shape[0]), first] * t[first], 0.0)
    r = oracle.render(sc.grid, sc.prims, sc.rays, _with_kappa(sc.march, 1.0))
    np.testing.assert_allclose(r["depth"].reshape(-1), want, rtol=1e-14, atol=0)
    assert hit.any() and (A > 0).sum(1).max() > 1


def test_adjoint_with_kappa_matches_central_differences():
    sc = random_scene(34, n=6, n_classes=2, width=5, height=4, n_samples=20, opacity_hi=0.9)
    march = _with_kappa(sc.march, 0.05)
    rng = np.random.default_rng(0)
    g_d, g_s = synth.upstream_grads(rng, sc.rays, 2)
    r0 = oracle.render(sc.grid, sc.prims, sc.rays, march)
    assert np.min(r0["kappa_margin"]) > 1e-6                     # no ray sits on the threshold
    tf = r0["t_final"].reshape(-1)
    assert np.sum((tf > 0) & (tf < 0.05)) >= 2                   # some rays stop before saturating
    grads = oracle.render_grad(sc.grid, sc.prims, sc.rays, march, g_d, g_s)

    def loss(pr):
        return oracle.loss_value(oracle.render(sc.grid, pr, sc.rays, march), g_d, g_s)

    p64 = synth.Prims(*(a.astype(np.float64) for a in (sc.prims.means, sc.prims.quats, sc.prims.scales,
                                                       sc.prims.eps, sc.prims.opacity, sc.prims.logits)))
    h = 1e-7
    for name in ("means", "quats", "scales", "eps", "opacity", "logits"):
        fi = int(np.argmax(np.abs(grads[name]).reshape(-1)))
        an = grads[name].reshape(-1)[fi]
        assert abs(an) > 1e-4, (name, an)
        plus = synth.Prims(*(np.array(a) for a in (p64.means, p64.quats, p64.scales, p64.eps, p64.opacity,
                                                    p64.logits)))
        minus = synth.Prims(*(np.array(a) for a in (p64.means, p64.quats, p64.scales, p64.eps, p64.opacity,
                                                     p64.logits)))
        getattr(plus, name).reshape(-1)[fi] += h
        getattr(minus, name).reshape(-1)[fi] -= h
        fd = (loss(plus) - loss(minus)) / (2 * h)
        assert abs(fd - an) <= 1e-5 * abs(an), (name, fi, fd, an)

"""Pins of the loss oracle (Eq. eq:loss): closed forms, a library
log-softmax, central differences of the loss in its inputs, label masking and
normalisation, and the whole chain through the renderer's adjoint."""
import numpy as np
import pytest
from scipy.special import log_softmax

import oracle
import synth
from tests.scenes_small import random_scene


def _inputs(seed, R=23, C=5, ignore=0.2, no_depth=0.3):
    rng = np.random.default_rng(seed)
    sem = rng.normal(0, 2, (R, C))
    depth = rng.uniform(0.5, 20, R)
    lab = rng.integers(0, C, R)
    lab[rng.random(R) < ignore] = -1
    dl = depth + rng.normal(0, 1.5, R)
    dl[rng.random(R) < no_depth] = 0.0
    return sem, depth, lab, dl


def test_uniform_logits_cost_log_C_and_mse_closed_form():
    C = 7
    sem = np.full((4, C), 3.25)
    out = oracle.fused_loss(sem, np.array([1.0, 2.0, 3.0, 4.0]), np.array([0, 3, 6, 2]),
                            np.array([1.5, 0.0, 2.0, 8.0]), lambda_sem=2.0, lambda_depth=0.05)
    assert out["loss_sem"] == pytest.approx(np.log(C), rel=1e-15)
    # labelled depths: (1-1.5)^2, (3-2)^2, (4-8)^2 over 3 pixels
    assert out["loss_depth"] == pytest.approx((0.25 + 1.0 + 16.0) / 3, rel=1e-15)
    assert out["loss"] == pytest.approx(2.0 * np.log(C) + 0.05 * (17.25 / 3), rel=1e-15)
    assert out["n_sem"] == 4 and out["n_depth"] == 3


def test_cross_entropy_equals_library_log_softmax():
    sem, depth, lab, dl = _inputs(1)
    out = oracle.fused_loss(sem, depth, lab, dl)
    m = lab >= 0
    want = -np.mean(log_softmax(sem[m], axis=1)[np.arange(m.sum()), lab[m]])
    assert out["loss_sem"] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("seed", [2, 3])
def test_gradient_matches_central_differences(seed):
    sem, depth, lab, dl = _inputs(seed)
    out = oracle.fused_loss(sem, depth, lab, dl, lambda_sem=2.0, lambda_depth=0.05)
    h = 1e-6
    for r in range(sem.shape[0]):
        for c in range(sem.shape[1]):
            p, q = sem.copy(), sem.copy()
            p[r, c] += h
            q[r, c] -= h
            fd = (oracle.fused_loss(p, depth, lab, dl)["loss"] - oracle.fused_loss(q, depth, lab, dl)["loss"]) / (2 * h)
            assert fd == pytest.approx(out["g_sem"][r, c], abs=1e-8), (r, c)
        p, q = depth.copy(), depth.copy()
        p[r] += h
        q[r] -= h
        fd = (oracle.fused_loss(sem, p, lab, dl)["loss"] - oracle.fused_loss(sem, q, lab, dl)["loss"]) / (2 * h)
        assert fd == pytest.approx(out["g_depth"][r], abs=1e-8), r


def test_unlabelled_pixels_do_not_count_and_means_normalise():
    sem, depth, lab, dl = _inputs(4)
    out = oracle.fused_loss(sem, depth, lab, dl)
    # unlabelled pixels: no gradient, and changing their renders changes nothing
    assert np.all(out["g_sem"][lab < 0] == 0) and np.all(out["g_depth"][~(dl > 0)] == 0)
    sem2, depth2 = sem.copy(), depth.copy()
    sem2[lab < 0] += 7.0
    depth2[~(dl > 0)] -= 3.0
    assert oracle.fused_loss(sem2, depth2, lab, dl)["loss"] == pytest.approx(out["loss"], rel=1e-15)
    # duplicating every pixel leaves the means unchanged and halves each gradient
    dup = oracle.fused_loss(np.vstack([sem, sem]), np.concatenate([depth, depth]), np.concatenate([lab, lab]),
                            np.concatenate([dl, dl]))
    assert dup["loss"] == pytest.approx(out["loss"], rel=1e-14)
    np.testing.assert_allclose(dup["g_sem"][:len(lab)], out["g_sem"] / 2, rtol=1e-14, atol=1e-300)
    # no labels at all: zero loss and gradient
    none = oracle.fused_loss(sem, depth, np.full_like(lab, -1), np.zeros_like(dl))
    assert none["loss"] == 0 and not none["g_sem"].any() and not none["g_depth"].any()
    # labels outside [0, C) and non-finite depths are "no label"
    odd = oracle.fused_loss(sem, depth, np.where(lab < 0, sem.shape[1] + 2, lab), np.where(dl > 0, dl, np.nan))
    assert odd["loss"] == pytest.approx(out["loss"], rel=1e-15)


def test_chain_through_the_renderer_matches_central_differences():
    """d L(render(theta)) / d theta from render_grad with the loss gradients as
    upstream equals FP64 central differences of the composed function, at the
    largest-gradient element of every parameter group."""
    sc = random_scene(18, n=8, n_classes=3, width=6, height=5, n_samples=20, opacity_hi=0.9)
    rng = np.random.default_rng(5)
    R, C = sc.rays.n_rays, sc.prims.n_classes
    lab = rng.integers(-1, C, R)
    dl = rng.uniform(0.5, 4.0, R)
    dl[rng.random(R) < 0.25] = 0.0
    cams, H, W = sc.rays.shape

    def total(pr):
        r = oracle.render(sc.grid, pr, sc.rays, sc.march)
        return oracle.fused_loss(r["sem"].transpose(0, 2, 3, 1).reshape(-1, C), r["depth"].reshape(-1), lab, dl)

    base = total(sc.prims)
    g_d = base["g_depth"].reshape(cams, H, W)
    g_s = base["g_sem"].reshape(cams, H, W, C).transpose(0, 3, 1, 2)
    grads = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    p64 = synth.Prims(*(a.astype(np.float64) for a in (sc.prims.means, sc.prims.quats, sc.prims.scales,
                                                       sc.prims.eps, sc.prims.opacity, sc.prims.logits)))
    h = 1e-6
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
        fd = (total(plus)["loss"] - total(minus)["loss"]) / (2 * h)
        assert abs(fd - an) <= 1e-5 * abs(an), (name, fi, fd, an)

"""The torch.autograd.Function over the C ABI (`autograd.render`): its forward
matches the FP64 oracle's render, and `loss.backward()` leaves in every leaf
tensor the oracle's gradient of L = sum g_D D + sum <g_S, S> (Sec. 3.3
"Backward Pass"), at the tolerances of the direct ABI tests."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_17361_amd import api, autograd
    from tests import gpu_helpers as H

NAMES = ("means", "quats", "scales", "eps", "opacity", "logits")


def _say(*a):
    print(*a, flush=True)


def _leaves(sc):
    return {k: torch.tensor(getattr(sc.prims, k), dtype=torch.float32, device="cuda", requires_grad=True)
            for k in NAMES}


def _render(sc, p, ckpt_every=8, stash=None):
    rays = api.Rays.from_numpy(sc.rays)
    return autograd.render(p["means"], p["quats"], p["scales"], p["eps"], p["opacity"], p["logits"],
                           rays.origins, rays.dirs, api.Grid.of(sc.grid), api.March.of(sc.march),
                           ckpt_every=ckpt_every, stash=stash)


def _softmax(sem):
    s = np.asarray(sem, np.float64)
    e = np.exp(s - s.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("ckpt_every", [4, 8])
def test_autograd_config0_forward_and_gradients(ckpt_every):
    sc = synth.config(0)
    _say("autograd config0, K =", ckpt_every)
    g_d, g_s = synth.upstream_grads(np.random.default_rng(11), sc.rays, sc.prims.n_classes)
    p = _leaves(sc)
    depth, sem = _render(sc, p, ckpt_every)
    loss = (depth * torch.from_numpy(g_d).cuda()).sum() + (sem * torch.from_numpy(g_s).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    H.assert_depth_close(depth.detach().cpu().numpy(), ref["depth"], "autograd cfg0")
    H.assert_probs_close(_softmax(sem.detach().cpu().numpy()), ref["probs"], "autograd cfg0")
    ref_g = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    H.assert_grads_close({k: p[k].grad.cpu().numpy() for k in NAMES}, ref_g, "autograd cfg0")


def test_autograd_depth_only_leaves_zero_logit_gradients():
    """With only the depth in the loss, the semantic output's gradient reaches
    the backward as zeros; the logits then get exactly zero gradient and the
    rest match the oracle with g_S = 0."""
    sc = synth.config(0)
    _say("autograd depth only")
    g_d, _ = synth.upstream_grads(np.random.default_rng(12), sc.rays, sc.prims.n_classes)
    p = _leaves(sc)
    depth, _sem = _render(sc, p)
    (depth * torch.from_numpy(g_d).cuda()).sum().backward()
    torch.cuda.synchronize()
    got = {k: p[k].grad.cpu().numpy() for k in NAMES}
    assert np.all(got["logits"] == 0.0)
    g_s0 = np.zeros((*sc.rays.shape[:1], sc.prims.n_classes, *sc.rays.shape[1:]), np.float32)
    ref_g = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s0)
    H.assert_grads_close(got, ref_g, "autograd depth only")


def test_autograd_composes_with_a_reparametrisation():
    """Scales as exp(log s): torch's chain rule through the Function gives
    d/d(log s) = s * dL/ds, with dL/ds the oracle's."""
    sc = synth.config(0)
    _say("autograd reparametrised scales")
    g_d, g_s = synth.upstream_grads(np.random.default_rng(13), sc.rays, sc.prims.n_classes)
    p = _leaves(sc)
    log_s = torch.log(p["scales"].detach()).requires_grad_(True)
    q = dict(p, scales=torch.exp(log_s))
    depth, sem = _render(sc, q)
    loss = (depth * torch.from_numpy(g_d).cuda()).sum() + (sem * torch.from_numpy(g_s).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref_g = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    want = dict(ref_g, scales=np.asarray(ref_g["scales"], np.float64) * sc.prims.scales.astype(np.float64))
    got = {k: p[k].grad.cpu().numpy() for k in NAMES if k != "scales"}
    got["scales"] = log_s.grad.cpu().numpy()
    H.assert_grads_close(got, want, "autograd exp(log s)")


@pytest.mark.parametrize("ckpt_every", [4, 8])
def test_autograd_with_a_stash_pool_over_two_steps(ckpt_every):
    """The same render and loss with an api.StashPool: the first step sizes
    the pool (a forward that counts the slots, then the pool), the second
    reuses it; both steps' forward and gradients match the oracle, and the
    second step asks for no more slots than the pool holds."""
    sc = synth.config(0)
    g_d, g_s = synth.upstream_grads(np.random.default_rng(13), sc.rays, sc.prims.n_classes)
    pool = api.StashPool()
    ref = oracle.render(sc.grid, sc.prims, sc.rays, sc.march)
    ref_g = oracle.render_grad(sc.grid, sc.prims, sc.rays, sc.march, g_d, g_s)
    for step in range(2):
        _say("autograd with a stash pool, K =", ckpt_every, "step", step)
        p = _leaves(sc)
        depth, sem = _render(sc, p, ckpt_every, stash=pool)
        loss = (depth * torch.from_numpy(g_d).cuda()).sum() + (sem * torch.from_numpy(g_s).cuda()).sum()
        loss.backward()
        torch.cuda.synchronize()
        H.assert_depth_close(depth.detach().cpu().numpy(), ref["depth"], f"autograd stash step {step}")
        H.assert_probs_close(_softmax(sem.detach().cpu().numpy()), ref["probs"], f"autograd stash step {step}")
        H.assert_grads_close({k: p[k].grad.cpu().numpy() for k in NAMES}, ref_g, f"autograd stash step {step}")
    head = pool.buf[:16].view(torch.int32).cpu().tolist()
    assert head[3] == 1 and 0 < head[4] <= head[5], head

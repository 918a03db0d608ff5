"""GPU test of sq_render_fwd_noalloc, the forward whose scratch is the
library's fixed per-GPU array (for callers that cannot allocate): two calls
in a row, the second on a smaller scene, each equal bit for bit to
sq_render_fwd with a caller workspace (the same kernels run on the same
inputs), and the first also within the oracle's tolerances."""
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


def _both(sc, ckpt_every, tuning):
    grid, prims, rays, march = H.gpu_scene(sc)
    idx = api.build_index(grid, prims)
    ref = api.render_fwd(grid, idx, prims, rays, march, ckpt_every=ckpt_every, tuning=tuning)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    got = api.render_fwd_noalloc(grid, idx, prims, rays, march, ckpt_every=ckpt_every, tuning=tuning)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    return ref, got


def test_noalloc_forward_equals_workspace_forward_on_two_calls():
    print("noalloc: config 0 then a smaller scene", flush=True)
    sc0 = synth.config(0)
    ref0, got0 = _both(sc0, 8, api.Tuning(8, 2, 0, 1, 0))
    for k in ("depth", "sem", "probs", "t_final", "ckpt"):
        assert np.array_equal(ref0[k], got0[k]), k
    o = oracle.render(sc0.grid, sc0.prims, sc0.rays, sc0.march)
    H.assert_depth_close(got0["depth"], o["depth"], "noalloc config 0")
    H.assert_probs_close(got0["probs"], o["probs"], "noalloc config 0")
    # a smaller scene second: the array keeps the first call's contents
    sc1 = random_scene(7, n=11, n_classes=3, width=9, height=5, n_samples=13, dims=(9, 7, 5), voxel=0.5,
                       lo=(-2.0, -2.0, -1.0), t_far=5.0)
    ref1, got1 = _both(sc1, 0, api.Tuning(4, 1, 0, 0, 0))
    for k in ("depth", "sem", "probs", "t_final"):
        assert np.array_equal(ref1[k], got1[k]), k
    o1 = oracle.render(sc1.grid, sc1.prims, sc1.rays, sc1.march)
    H.assert_depth_close(got1["depth"], o1["depth"], "noalloc small")
    H.assert_probs_close(got1["probs"], o1["probs"], "noalloc small")

"""Small hand-built scenes shared by the CPU and GPU tests (inputs only)."""
import numpy as np

import synth


def grid_small(nv=5, dims=(8, 8, 4), voxel=0.5, lo=(-2.0, -2.0, -1.0)):
    return synth.Grid(lo=lo, voxel=voxel, dims=dims, nv=nv)


def random_scene(seed, n=6, n_classes=3, width=5, height=4, n_samples=16, nv=5,
                 opacity_hi=1.0, dims=(8, 8, 4), voxel=0.5, lo=(-2.0, -2.0, -1.0),
                 scale_lo=0.3, scale_hi=1.2, t_far=5.0, cam=(0.0, 0.0, 0.0), yaw=0.0):
    """A few superquadrics in front of one small camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = grid_small(nv, dims, voxel, lo)
    lo_a = np.array(lo)
    hi_a = lo_a + np.array(dims) * voxel
    means = rng.uniform(lo_a + 0.2, hi_a - 0.2, (n, 3))
    prims = synth.make_prims(rng, means, scale_lo, scale_hi, n_classes)
    prims.opacity[:] = (prims.opacity * opacity_hi).astype(np.float32)
    rays = synth.pinhole_rig(1, width, height, 90.0, cam, yaw0_deg=yaw)
    march = synth.March(n_samples, 0.1, t_far)
    return synth.Scene(grid, prims, rays, march, name=f"rand{seed}")


def single_prim_scene(mean, quat, scales, eps, opacity, logits, width=6, height=5,
                      n_samples=40, t_far=6.0, nv=32, dims=(16, 16, 8), voxel=0.5,
                      lo=(-4.0, -4.0, -2.0), cam=(0.0, 0.0, 0.0), yaw=0.0, hfov=90.0):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    prims = synth.Prims(f([mean]), f([quat]), f([scales]), f([eps]), f([opacity]), f([logits]))
    grid = synth.Grid(lo=lo, voxel=voxel, dims=dims, nv=nv)
    rays = synth.pinhole_rig(1, width, height, hfov, cam, yaw0_deg=yaw)
    march = synth.March(n_samples, 0.1, t_far)
    return synth.Scene(grid, prims, rays, march, name="single")

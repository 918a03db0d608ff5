"""ctypes binding of libsqr.so (the C ABI declared in include/sqr.h).

Argument marshalling only: every step of the renderer runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsqr.so")

SQ_OK = 0
SQ_ERR_INVALID = -1
SQ_ERR_CAPACITY = -2
SQ_ERR_HIP = -3
SQ_ERR_UNSUPPORTED = -4
SQ_MAX_CLASSES = 32
SQ_MAX_SCENE_PRIMS = (1 << 25) - 1

EXPORTED = [
    "sq_last_error", "sq_version", "sq_default_tuning", "sq_index_capacity_bound",
    "sq_build_index_workspace", "sq_build_index", "sq_render_workspace", "sq_render_fwd", "sq_render_bwd",
    "sq_batch_workspace", "sq_batch_build_index", "sq_batch_render_fwd", "sq_batch_render_bwd", "sq_batch_step",
    "sq_batch_step_graph_create", "sq_graph_launch", "sq_graph_destroy", "sq_batch_autotune",
    "sq_voxelise_workspace", "sq_voxelise", "sq_batch_voxelise",
    "sq_render_fwd_loss", "sq_batch_render_fwd_loss", "sq_batch_train_step", "sq_batch_train_graph_create",
    "sq_sq_major_workspace", "sq_render_bwd_sq_major", "sq_batch_tile_stop_len", "sq_render_fwd_noalloc",
    "sq_batch_autotune_cached", "sq_batch_tuning_key", "sq_batch_stash_len",
]
# int32 words of the stash header: tile width, L, K, written, slots asked for, slots held
SQ_STASH_HEAD = 16
SQ_NOALLOC_SCRATCH_BYTES = 16 << 20


class SqGrid(ct.Structure):
    _fields_ = [("lo", ct.c_float * 3), ("voxel", ct.c_float), ("dims", ct.c_int32 * 3), ("nv", ct.c_int32),
                ("theta", ct.c_float)]


class SqIndex(ct.Structure):
    _fields_ = [("counts", ct.c_void_p), ("offsets", ct.c_void_p), ("ids", ct.c_void_p),
                ("capacity", ct.c_int64), ("total", ct.c_void_p)]


class SqPrims(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("n_classes", ct.c_int32), ("means", ct.c_void_p), ("quats", ct.c_void_p),
                ("scales", ct.c_void_p), ("eps", ct.c_void_p), ("opacity", ct.c_void_p), ("logits", ct.c_void_p)]


class SqRays(ct.Structure):
    _fields_ = [("n_cams", ct.c_int32), ("height", ct.c_int32), ("width", ct.c_int32),
                ("origins", ct.c_void_p), ("dirs", ct.c_void_p)]


class SqMarch(ct.Structure):
    _fields_ = [("n_samples", ct.c_int32), ("t_near", ct.c_float), ("t_far", ct.c_float),
                ("ckpt_every", ct.c_int32), ("kappa", ct.c_float)]


class SqGrads(ct.Structure):
    _fields_ = [("means", ct.c_void_p), ("quats", ct.c_void_p), ("scales", ct.c_void_p), ("eps", ct.c_void_p),
                ("opacity", ct.c_void_p), ("logits", ct.c_void_p)]


SQ_BWD_AUTO = 0
SQ_BWD_SAMPLE_MAJOR = 1
SQ_BWD_PRIMITIVE_MAJOR = 2


class SqTuning(ct.Structure):
    _fields_ = [("tile_w", ct.c_int32), ("waves_per_block", ct.c_int32), ("bwd_mode", ct.c_int32),
                ("persistent", ct.c_int32), ("chunk", ct.c_int32)]


SQ_MAX_SCENES = 32


class SqScene(ct.Structure):
    _fields_ = [("n_prims", ct.c_int32), ("n_cams", ct.c_int32), ("height", ct.c_int32), ("width", ct.c_int32),
                ("index_capacity", ct.c_int64)]


class SqBatch(ct.Structure):
    _fields_ = [("n_scenes", ct.c_int32), ("n_classes", ct.c_int32), ("grid", SqGrid), ("march", SqMarch),
                ("scenes", SqScene * SQ_MAX_SCENES)]


class SqBatchIO(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in (
        "means", "quats", "scales", "eps", "opacity", "logits", "origins", "dirs",
        "counts", "offsets", "ids", "totals", "depth", "sem", "probs", "t_final", "ckpt",
        "g_depth", "g_sem", "g_means", "g_quats", "g_scales", "g_eps", "g_opacity", "g_logits",
        "vox_density", "vox_sem", "vox_labels", "sem_label", "depth_label", "loss", "tile_stop")] + [
        ("tile_stop_len", ct.c_int64), ("ckpt_len", ct.c_int64), ("stash", ct.c_void_p), ("stash_len", ct.c_int64)]


class SqLossWeights(ct.Structure):
    _fields_ = [("lambda_sem", ct.c_float), ("lambda_depth", ct.c_float)]


_lib = None


def load(path: str = LIB_PATH) -> ct.CDLL:
    """Load libsqr.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2511_17361_amd.build` "
                           "(or __graft_entry__.build()) first")
    lib = ct.CDLL(path)
    P = ct.POINTER
    lib.sq_last_error.restype = ct.c_char_p
    lib.sq_version.restype = ct.c_int32
    lib.sq_default_tuning.restype = SqTuning
    lib.sq_index_capacity_bound.restype = ct.c_int64
    lib.sq_index_capacity_bound.argtypes = [P(SqGrid), ct.c_int32]
    lib.sq_build_index_workspace.restype = ct.c_size_t
    lib.sq_build_index_workspace.argtypes = [P(SqGrid), ct.c_int32]
    lib.sq_build_index.restype = ct.c_int32
    lib.sq_build_index.argtypes = [P(SqGrid), P(SqPrims), P(SqIndex), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_render_workspace.restype = ct.c_size_t
    lib.sq_render_workspace.argtypes = [P(SqGrid), P(SqPrims), P(SqRays), P(SqMarch)]
    lib.sq_render_fwd.restype = ct.c_int32
    lib.sq_render_fwd.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), P(SqRays), P(SqMarch),
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                  P(SqTuning), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_render_fwd_noalloc.restype = ct.c_int32
    lib.sq_render_fwd_noalloc.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), P(SqRays), P(SqMarch),
                                          ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                          ct.c_void_p, P(SqTuning), ct.c_void_p]
    lib.sq_render_bwd.restype = ct.c_int32
    lib.sq_render_bwd.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), P(SqRays), P(SqMarch),
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, P(SqGrads), ct.c_void_p, P(SqTuning),
                                  ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_batch_workspace.restype = ct.c_size_t
    lib.sq_batch_workspace.argtypes = [P(SqBatch)]
    lib.sq_batch_tile_stop_len.restype = ct.c_int64
    lib.sq_batch_tile_stop_len.argtypes = [P(SqBatch), P(SqTuning)]
    lib.sq_batch_stash_len.restype = ct.c_int64
    lib.sq_batch_stash_len.argtypes = [P(SqBatch), P(SqTuning), ct.c_int64]
    lib.sq_batch_build_index.restype = ct.c_int32
    lib.sq_batch_build_index.argtypes = [P(SqBatch), P(SqBatchIO), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    for fn in (lib.sq_batch_render_fwd, lib.sq_batch_render_bwd):
        fn.restype = ct.c_int32
        fn.argtypes = [P(SqBatch), P(SqBatchIO), ct.c_void_p, P(SqTuning), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_batch_step.restype = ct.c_int32
    lib.sq_batch_step.argtypes = [P(SqBatch), P(SqBatchIO), P(SqTuning), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_batch_step_graph_create.restype = ct.c_int32
    lib.sq_batch_step_graph_create.argtypes = [P(SqBatch), P(SqBatchIO), P(SqTuning), ct.c_void_p, ct.c_size_t,
                                               ct.c_void_p, P(ct.c_void_p)]
    lib.sq_graph_launch.restype = ct.c_int32
    lib.sq_graph_launch.argtypes = [ct.c_void_p, ct.c_void_p]
    lib.sq_graph_destroy.restype = ct.c_int32
    lib.sq_graph_destroy.argtypes = [ct.c_void_p]
    lib.sq_batch_autotune.restype = ct.c_int32
    lib.sq_batch_autotune.argtypes = [P(SqBatch), P(SqBatchIO), P(SqTuning), ct.c_int32, ct.c_int32,
                                      P(ct.c_int32), P(ct.c_float), ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_batch_autotune_cached.restype = ct.c_int32
    lib.sq_batch_autotune_cached.argtypes = [P(SqBatch), P(SqBatchIO), P(SqTuning), ct.c_int32, ct.c_int32,
                                             ct.c_char_p, P(SqTuning), P(ct.c_int32), ct.c_void_p, ct.c_size_t,
                                             ct.c_void_p]
    lib.sq_batch_tuning_key.restype = ct.c_int32
    lib.sq_batch_tuning_key.argtypes = [P(SqBatch), ct.c_char_p, ct.c_int32]
    lib.sq_voxelise_workspace.restype = ct.c_size_t
    lib.sq_voxelise_workspace.argtypes = [P(SqGrid), P(SqPrims)]
    lib.sq_voxelise.restype = ct.c_int32
    lib.sq_voxelise.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), ct.c_float, ct.c_void_p, ct.c_void_p,
                                ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_batch_voxelise.restype = ct.c_int32
    lib.sq_batch_voxelise.argtypes = [P(SqBatch), P(SqBatchIO), ct.c_float, ct.c_void_p, ct.c_size_t, ct.c_void_p]
    lib.sq_render_fwd_loss.restype = ct.c_int32
    lib.sq_render_fwd_loss.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), P(SqRays), P(SqMarch), P(SqLossWeights),
                                       ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                       ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, P(SqTuning), ct.c_void_p,
                                       ct.c_size_t, ct.c_void_p]
    for fn in (lib.sq_batch_render_fwd_loss, lib.sq_batch_train_step):
        fn.restype = ct.c_int32
        fn.argtypes = [P(SqBatch), P(SqBatchIO), P(SqLossWeights), P(SqTuning), ct.c_void_p, ct.c_size_t,
                       ct.c_void_p]
    lib.sq_batch_train_graph_create.restype = ct.c_int32
    lib.sq_batch_train_graph_create.argtypes = [P(SqBatch), P(SqBatchIO), P(SqLossWeights), P(SqTuning),
                                                ct.c_void_p, ct.c_size_t, ct.c_void_p, P(ct.c_void_p)]
    lib.sq_sq_major_workspace.restype = ct.c_size_t
    lib.sq_sq_major_workspace.argtypes = [P(SqGrid), P(SqPrims), P(SqRays), P(SqMarch), ct.c_int64]
    lib.sq_render_bwd_sq_major.restype = ct.c_int32
    lib.sq_render_bwd_sq_major.argtypes = [P(SqGrid), P(SqIndex), P(SqPrims), P(SqRays), P(SqMarch), ct.c_void_p,
                                           ct.c_void_p, ct.c_void_p, P(SqGrads), ct.c_int64, ct.c_void_p,
                                           ct.c_void_p, ct.c_size_t, P(SqTuning), ct.c_void_p, ct.c_size_t,
                                           ct.c_void_p]
    _lib = lib
    return lib


class SqrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sqr status {code}: {msg}")
        self.code = code


def check(code: int) -> None:
    if code != SQ_OK:
        raise SqrError(code, load().sq_last_error().decode(errors="replace"))

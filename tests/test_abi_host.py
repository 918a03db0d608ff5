"""Host-only checks of the C ABI library: it loads, exports every symbol
include/sqr.h declares, and rejects bad arguments before launching anything.
No compute call here touches a GPU."""
import ctypes as ct
import os
import re

import pytest

from paper_2511_17361_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "sqr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sq_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared_symbols()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    assert set(L.EXPORTED) == set(declared)


def test_version_and_defaults():
    lib = L.load()
    assert lib.sq_version() >= 200
    t = lib.sq_default_tuning()
    assert t.tile_w in (4, 8, 16) and 1 <= t.waves_per_block <= 4


def _grid(dims=(200, 200, 16), nv=5, voxel=0.4):
    g = L.SqGrid()
    for i, v in enumerate((-40.0, -40.0, -1.0)):
        g.lo[i] = v
    for i, d in enumerate(dims):
        g.dims[i] = d
    g.voxel = voxel
    g.nv = nv
    return g


def test_capacity_bound_and_workspace():
    lib = L.load()
    g = _grid()
    assert lib.sq_index_capacity_bound(ct.byref(g), 1000) == 1000 * 11 * 11 * 11
    g2 = _grid(dims=(4, 5, 6), nv=10)
    assert lib.sq_index_capacity_bound(ct.byref(g2), 3) == 3 * 4 * 5 * 6
    assert lib.sq_build_index_workspace(ct.byref(g), 6400) >= 6400 * 16
    bad = _grid(nv=-1)
    assert lib.sq_index_capacity_bound(ct.byref(bad), 10) == -1


def _march(L_=100, tn=0.1, tf=45.0, K=0):
    m = L.SqMarch()
    m.n_samples, m.t_near, m.t_far, m.ckpt_every = L_, tn, tf, K
    return m


FAKE = 0x1000   # never dereferenced: every call below must fail validation first


def _prims(n=10, C=17):
    p = L.SqPrims()
    p.n, p.n_classes = n, C
    for f in ("means", "quats", "scales", "eps", "opacity", "logits"):
        setattr(p, f, FAKE)
    return p


def _rays():
    r = L.SqRays()
    r.n_cams, r.height, r.width = 1, 8, 8
    r.origins = FAKE
    r.dirs = FAKE
    return r


def _index():
    i = L.SqIndex()
    i.counts = FAKE
    i.offsets = FAKE
    i.ids = FAKE
    i.capacity = 100
    i.total = FAKE
    return i


@pytest.mark.parametrize("mutate,code", [
    (lambda a: setattr(a["grid"], "voxel", 0.0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["grid"], "nv", -2), L.SQ_ERR_INVALID),
    (lambda a: a["grid"].dims.__setitem__(1, 0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "n_classes", 33), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "n_classes", 0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "n", -1), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "opacity", None), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["march"], "n_samples", 0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["march"], "t_far", 0.05), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["march"], "t_near", -1.0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["rays"], "dirs", None), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["index"], "counts", None), L.SQ_ERR_INVALID),
    (lambda a: a.__setitem__("ws_bytes", 16), L.SQ_ERR_CAPACITY),
    (lambda a: a.__setitem__("tile_w", 5), L.SQ_ERR_INVALID),
    (lambda a: a.__setitem__("tile_w", 0), L.SQ_ERR_INVALID),
])
def test_render_fwd_rejects_bad_arguments_without_launch(mutate, code):
    lib = L.load()
    args = dict(grid=_grid(), prims=_prims(), rays=_rays(), march=_march(), index=_index(), ws_bytes=1 << 30,
                tile_w=8)
    mutate(args)
    t = L.SqTuning(args["tile_w"], 4, 0, 0, 0)
    rc = lib.sq_render_fwd(ct.byref(args["grid"]), ct.byref(args["index"]), ct.byref(args["prims"]),
                           ct.byref(args["rays"]), ct.byref(args["march"]), FAKE, FAKE, None, FAKE, None, None,
                           ct.byref(t), 0x100000, args["ws_bytes"], None)
    assert rc == code
    assert lib.sq_last_error().decode()


def test_render_bwd_needs_supported_chunk():
    lib = L.load()
    g, p, r, i = _grid(), _prims(), _rays(), _index()
    gr = L.SqGrads(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE)
    for K in (0, 3, 32):
        m = _march(K=K)
        rc = lib.sq_render_bwd(ct.byref(g), ct.byref(i), ct.byref(p), ct.byref(r), ct.byref(m), FAKE, FAKE, FAKE,
                               ct.byref(gr), None, None, 0x100000, 1 << 30, None)
        assert rc == L.SQ_ERR_INVALID
    m = _march(K=8)
    rc = lib.sq_render_bwd(ct.byref(g), ct.byref(i), ct.byref(p), ct.byref(r), ct.byref(m), None, FAKE, FAKE,
                           ct.byref(gr), None, None, 0x100000, 1 << 30, None)
    assert rc == L.SQ_ERR_INVALID and "ckpt" in lib.sq_last_error().decode()


def test_build_index_rejects_bad_arguments():
    lib = L.load()
    g, p, i = _grid(), _prims(), _index()
    rc = lib.sq_build_index(ct.byref(g), ct.byref(p), ct.byref(i), 0x100000, 8, None)
    assert rc == L.SQ_ERR_CAPACITY
    i.total = None
    rc = lib.sq_build_index(ct.byref(g), ct.byref(p), ct.byref(i), 0x100000, 1 << 30, None)
    assert rc == L.SQ_ERR_INVALID
    big = _grid(dims=(40000, 2, 2))
    i = _index()
    rc = lib.sq_build_index(ct.byref(big), ct.byref(p), ct.byref(i), 0x100000, 1 << 30, None)
    assert rc == L.SQ_ERR_INVALID


@pytest.mark.parametrize("theta", [-1e-3, 1.0, 2.5, float("nan"), float("inf")])
def test_grid_rejects_bad_influence_threshold(theta):
    lib = L.load()
    g, p, i = _grid(), _prims(), _index()
    g.theta = theta
    rc = lib.sq_build_index(ct.byref(g), ct.byref(p), ct.byref(i), 0x100000, 1 << 30, None)
    assert rc == L.SQ_ERR_INVALID and "theta" in lib.sq_last_error().decode()


def test_thresholded_index_needs_the_primitive_parameters():
    """With theta = 0 the index needs only the centres; with theta > 0 it
    reads the quaternions, scales, eps and opacity as well."""
    lib = L.load()
    g, i = _grid(), _index()
    g.theta = 1e-3
    for f in ("quats", "scales", "eps", "opacity"):
        p = _prims()
        setattr(p, f, None)
        rc = lib.sq_build_index(ct.byref(g), ct.byref(p), ct.byref(i), 0x100000, 1 << 30, None)
        assert rc == L.SQ_ERR_INVALID and "theta" in lib.sq_last_error().decode(), f


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a.__setitem__("tau", float("nan")), L.SQ_ERR_INVALID),
    (lambda a: a.__setitem__("tau", float("inf")), L.SQ_ERR_INVALID),
    (lambda a: a.__setitem__("density", None), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "opacity", None), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["prims"], "n_classes", 0), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["index"], "offsets", None), L.SQ_ERR_INVALID),
    (lambda a: setattr(a["grid"], "voxel", -0.4), L.SQ_ERR_INVALID),
    (lambda a: a.__setitem__("ws_bytes", 64), L.SQ_ERR_CAPACITY),
    (lambda a: a.__setitem__("ws", 0x100010), L.SQ_ERR_INVALID),
])
def test_voxelise_rejects_bad_arguments_without_launch(mutate, code):
    lib = L.load()
    args = dict(grid=_grid(), prims=_prims(), index=_index(), tau=0.05, density=FAKE, ws=0x100000, ws_bytes=1 << 30)
    mutate(args)
    rc = lib.sq_voxelise(ct.byref(args["grid"]), ct.byref(args["index"]), ct.byref(args["prims"]), args["tau"],
                         args["density"], None, None, args["ws"], args["ws_bytes"], None)
    assert rc == code
    assert lib.sq_last_error().decode()


def test_voxelise_workspace_matches_render_records():
    lib = L.load()
    g, p = _grid(), _prims(n=25600)
    need = lib.sq_voxelise_workspace(ct.byref(g), ct.byref(p))
    assert need >= 25600 * (24 + 17) * 4
    bad = _prims(C=40)
    assert lib.sq_voxelise_workspace(ct.byref(g), ct.byref(bad)) == 0


def _batch(n_scenes=3, C=5):
    b = L.SqBatch()
    b.n_scenes, b.n_classes = n_scenes, C
    b.grid = _grid()
    b.march = _march(K=4)
    for i in range(n_scenes):
        b.scenes[i].n_prims = 10 * (i + 1)
        b.scenes[i].n_cams, b.scenes[i].height, b.scenes[i].width = 2, 9, 13
        b.scenes[i].index_capacity = 1000
    return b


def _batch_io():
    io = L.SqBatchIO()
    for name, _ in L.SqBatchIO._fields_:
        setattr(io, name, FAKE)
    io.tile_stop_len = 1 << 40
    io.ckpt_len = 1 << 40
    io.stash_len = 1 << 40
    return io


@pytest.mark.parametrize("mutate,code", [
    (lambda b, io: setattr(b, "n_scenes", 0), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b, "n_scenes", 33), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b, "n_classes", 0), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b.scenes[1], "n_prims", -1), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b.scenes[2], "width", -3), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b.scenes[0], "index_capacity", -1), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(b.march, "n_samples", 0), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(io, "counts", None), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(io, "ids", None), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(io, "logits", None), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(io, "origins", None), L.SQ_ERR_INVALID),
    (lambda b, io: setattr(io, "depth", None), L.SQ_ERR_INVALID),
])
def test_batch_forward_rejects_bad_arguments_without_launch(mutate, code):
    lib = L.load()
    b, io = _batch(), _batch_io()
    mutate(b, io)
    io.ckpt = None
    t = L.SqTuning(8, 4, 0, 0, 0)
    rc = lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30, None)
    assert rc == code
    assert lib.sq_last_error().decode()


def test_batch_calls_reject_bad_tuning_chunk_and_workspace():
    lib = L.load()
    b, io = _batch(), _batch_io()
    for t in (L.SqTuning(5, 4, 0, 0, 0), L.SqTuning(8, 0, 0, 0, 0), L.SqTuning(8, 4, 3, 0, 0),
              L.SqTuning(8, 4, 0, 2, 0), L.SqTuning(8, 4, 0, 0, -1)):
        assert lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30,
                                       None) == L.SQ_ERR_INVALID
    t = L.SqTuning(8, 4, 0, 0, 3)
    assert lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30,
                                   None) == L.SQ_ERR_INVALID
    t = L.SqTuning(8, 4, 0, 0, 4)
    assert lib.sq_batch_step(ct.byref(b), ct.byref(io), ct.byref(t), 0x100000, 256, None) == L.SQ_ERR_CAPACITY
    need = lib.sq_batch_workspace(ct.byref(b))
    assert need > 0
    assert lib.sq_batch_voxelise(ct.byref(b), ct.byref(io), float("nan"), 0x100000, need, None) == L.SQ_ERR_INVALID
    io.vox_density = None
    assert lib.sq_batch_voxelise(ct.byref(b), ct.byref(io), 0.05, 0x100000, need, None) == L.SQ_ERR_INVALID
    bad = _batch()
    bad.n_scenes = 40
    assert lib.sq_batch_workspace(ct.byref(bad)) == 0


def _key(lib, b):
    n = lib.sq_batch_tuning_key(ct.byref(b), None, 0)
    buf = ct.create_string_buffer(n + 1)
    assert lib.sq_batch_tuning_key(ct.byref(b), buf, n + 1) == n
    return buf.value.decode()


def test_tuning_key_names_the_workload():
    """The autotune cache key: one line without spaces that changes with every
    scene shape, the grid, the march and the class count."""
    lib = L.load()
    b = _batch()
    k = _key(lib, b)
    assert k and " " not in k and "\n" not in k and k == _key(lib, _batch())
    assert k.startswith("v%d|" % lib.sq_version())
    short = ct.create_string_buffer(8)
    assert lib.sq_batch_tuning_key(ct.byref(b), short, 8) == len(k) and short.value.decode() == k[:7]
    assert lib.sq_batch_tuning_key(None, None, 0) == -1
    for mutate in (lambda x: setattr(x.scenes[1], "width", 14), lambda x: setattr(x, "n_classes", 6),
                   lambda x: setattr(x.march, "n_samples", 40), lambda x: setattr(x.grid, "voxel", 0.5),
                   lambda x: setattr(x.scenes[2], "n_prims", 31)):
        b2 = _batch()
        mutate(b2)
        assert _key(lib, b2) != k


def test_autotune_cache_hit_launches_nothing(tmp_path):
    """A cache line under the batch's key is returned without timing (nothing
    is launched: on a host without a GPU any launch would fail); lines of other
    keys, lines that do not parse and tunings the library cannot run are
    skipped, the last matching line wins; the candidates are still validated."""
    lib = L.load()
    b, io = _batch(), _batch_io()
    key = _key(lib, b)
    path = tmp_path / "tuning.txt"
    path.write_text("\n".join([
        "some other workload => 4 2 0 1 4",
        key + " => 16 2 1",                      # does not parse
        key + " => 5 2 0 1 4",                   # tile width the library does not run
        key + " => 8 2 0 1 4",
        key + " => 16 4 0 1 8",                  # the last valid line wins
    ]) + "\n")
    cands = (L.SqTuning * 2)(L.SqTuning(8, 4, 0, 1, 4), L.SqTuning(16, 2, 0, 1, 4))
    best, hit = L.SqTuning(), ct.c_int32(-1)
    st = lib.sq_batch_autotune_cached(ct.byref(b), ct.byref(io), cands, 2, 1, str(path).encode(), ct.byref(best),
                                      ct.byref(hit), 0x100000, 1 << 40, None)
    assert st == L.SQ_OK, lib.sq_last_error()
    assert hit.value == 1
    assert (best.tile_w, best.waves_per_block, best.bwd_mode, best.persistent, best.chunk) == (16, 4, 0, 1, 8)
    # an invalid candidate is rejected before the cache is read
    bad = (L.SqTuning * 1)(L.SqTuning(5, 4, 0, 1, 4))
    assert lib.sq_batch_autotune_cached(ct.byref(b), ct.byref(io), bad, 1, 1, str(path).encode(), ct.byref(best),
                                        ct.byref(hit), 0x100000, 1 << 40, None) == L.SQ_ERR_INVALID
    assert lib.sq_batch_autotune_cached(ct.byref(b), ct.byref(io), cands, 2, 1, str(path).encode(), None,
                                        ct.byref(hit), 0x100000, 1 << 40, None) == L.SQ_ERR_INVALID


@pytest.mark.parametrize("kappa", [-0.1, 1.5, float("nan"), float("inf")])
def test_march_kappa_outside_unit_interval_is_rejected(kappa):
    lib = L.load()
    m = _march(K=4)
    m.kappa = kappa
    t = L.SqTuning(8, 4, 0, 0, 0)
    rc = lib.sq_render_fwd(ct.byref(_grid()), ct.byref(_index()), ct.byref(_prims()), ct.byref(_rays()), ct.byref(m),
                           FAKE, FAKE, None, FAKE, None, None, ct.byref(t), 0x100000, 1 << 30, None)
    assert rc == L.SQ_ERR_INVALID and "kappa" in lib.sq_last_error().decode()


def test_stash_length_query_and_short_buffer():
    """Header and slot table (16 + tiles x ceil(L/K) int32, rounded up to 64
    floats), then K x 64 x (Q + 2) floats per slot, Q = the class count padded
    to the matrix-core width (8 at C = 5); a buffer shorter than header and
    table is refused before any launch, by forwards with checkpoints and the
    backward; a forward without checkpoints needs the header only."""
    lib = L.load()
    b = _batch()          # L = 100, C = 5
    for tw, tiles in ((8, 24), (16, 18), (4, 24)):
        for K in (4, 8):
            t = L.SqTuning(tw, 4, 0, 0, K)
            n0 = lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), 0)
            nck = -(-100 // K)
            assert n0 == -(-(16 + tiles * nck) // 64) * 64
            assert lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), 3) == n0 + 3 * K * 64 * (8 + 2)
    t = L.SqTuning(8, 4, 0, 0, 8)
    assert lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), -1) == 0
    assert lib.sq_batch_stash_len(ct.byref(b), ct.byref(L.SqTuning(8, 4, 0, 0, 5)), 0) == 0
    assert lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), 1 << 31) == 0
    b17 = _batch(C=17)
    n0 = lib.sq_batch_stash_len(ct.byref(b17), ct.byref(t), 0)
    assert lib.sq_batch_stash_len(ct.byref(b17), ct.byref(t), 1) == n0 + 8 * 64 * (16 + 2)
    io = _batch_io()
    io.stash_len = lib.sq_batch_stash_len(ct.byref(b), ct.byref(t), 0) - 1
    w = L.SqLossWeights(2.0, 0.05)
    for call in (lambda: lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30, None),
                 lambda: lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30, None),
                 lambda: lib.sq_batch_render_fwd_loss(ct.byref(b), ct.byref(io), ct.byref(w), ct.byref(t), 0x100000,
                                                      1 << 30, None),
                 lambda: lib.sq_batch_step(ct.byref(b), ct.byref(io), ct.byref(t), 0x100000, 1 << 30, None)):
        assert call() == L.SQ_ERR_CAPACITY
        assert "stash" in lib.sq_last_error().decode()
    io.ckpt = None
    io.stash_len = 15
    assert lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30,
                                   None) == L.SQ_ERR_CAPACITY


def test_tile_stop_length_query_and_short_buffer():
    """4 + tiles of the call's tiling; a shorter buffer is refused before any
    launch by the forwards and the backward."""
    lib = L.load()
    b = _batch()
    # 3 scenes x 2 cameras of 13 x 9 pixels: 8 x 8 tiles 2 x 2, 16 x 4 tiles 1 x 3, 4 x 16 tiles 4 x 1
    for tw, tiles in ((8, 24), (16, 18), (4, 24)):
        t = L.SqTuning(tw, 4, 0, 0, 4)
        assert lib.sq_batch_tile_stop_len(ct.byref(b), ct.byref(t)) == 4 + tiles
    assert lib.sq_batch_tile_stop_len(ct.byref(b), ct.byref(L.SqTuning(5, 4, 0, 0, 4))) == 0
    io = _batch_io()
    io.tile_stop_len = 4 + 24 - 1
    t = L.SqTuning(8, 4, 0, 0, 4)
    assert lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30,
                                   None) == L.SQ_ERR_CAPACITY
    assert "tile_stop" in lib.sq_last_error().decode()
    assert lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 30,
                                   None) == L.SQ_ERR_CAPACITY
    w = L.SqLossWeights(2.0, 0.05)
    assert lib.sq_batch_render_fwd_loss(ct.byref(b), ct.byref(io), ct.byref(w), ct.byref(t), 0x100000, 1 << 30,
                                        None) == L.SQ_ERR_CAPACITY


def test_index_offsets_must_fit_int32():
    """V_f holds int32 offsets: a scene whose capacity, or whose worst-case
    entry count n * prod(min(2 N_v + 1, dims)), exceeds 2^31 - 1 is refused
    before any launch (index build, renders, steps)."""
    lib = L.load()
    INT32_MAX = 2 ** 31 - 1
    g = _grid()                                   # 11^3 = 1331 cells per primitive at N_v = 5
    n_ok = INT32_MAX // 1331
    assert lib.sq_index_capacity_bound(ct.byref(g), n_ok) <= INT32_MAX
    assert lib.sq_index_capacity_bound(ct.byref(g), n_ok + 1) > INT32_MAX
    b, io = _batch(), _batch_io()
    b.scenes[1].n_prims = n_ok + 1
    t = L.SqTuning(8, 4, 0, 0, 4)
    calls = (lambda: lib.sq_batch_build_index(ct.byref(b), ct.byref(io), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_step(ct.byref(b), ct.byref(io), ct.byref(t), 0x100000, 1 << 40, None))
    for call in calls:
        assert call() == L.SQ_ERR_UNSUPPORTED
        assert "int32" in lib.sq_last_error().decode()
    b.scenes[1].n_prims = n_ok
    b.scenes[2].index_capacity = INT32_MAX + 1
    for call in calls:
        assert call() == L.SQ_ERR_UNSUPPORTED
    # single-scene index build: the capacity alone
    ix = _index()
    ix.capacity = INT32_MAX + 1
    assert lib.sq_build_index(ct.byref(g), ct.byref(_prims()), ct.byref(ix), 0x100000, 1 << 40,
                              None) == L.SQ_ERR_UNSUPPORTED


def test_scene_primitive_count_is_bounded_for_32_bit_record_offsets():
    """The kernels reach primitive k's record and logits through a 32-bit byte
    offset from the scene's base, and the scene's logit rows through a buffer
    range of at most 2^32 - 1 bytes, so a scene of more than SQ_MAX_SCENE_PRIMS
    primitives is refused before any launch, also where the index bound would
    still fit (one voxel per primitive)."""
    lib = L.load()
    assert L.SQ_MAX_SCENE_PRIMS * 32 * 4 <= 2 ** 32 - 1     # widest logit rows: 32 classes
    assert L.SQ_MAX_SCENE_PRIMS * 28 * 4 <= 2 ** 32 - 1     # records
    b, io = _batch(), _batch_io()
    b.grid = _grid(dims=(1, 1, 1), nv=1)
    b.scenes[0].n_prims = L.SQ_MAX_SCENE_PRIMS + 1
    assert lib.sq_index_capacity_bound(ct.byref(b.grid), L.SQ_MAX_SCENE_PRIMS + 1) <= 2 ** 31 - 1
    t = L.SqTuning(8, 4, 0, 0, 4)
    calls = (lambda: lib.sq_batch_build_index(ct.byref(b), ct.byref(io), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
             lambda: lib.sq_batch_step(ct.byref(b), ct.byref(io), ct.byref(t), 0x100000, 1 << 40, None))
    for call in calls:
        assert call() == L.SQ_ERR_UNSUPPORTED
        assert "SQ_MAX_SCENE_PRIMS" in lib.sq_last_error().decode()
    # single-scene calls take the same bound
    p = _prims()
    p.n = L.SQ_MAX_SCENE_PRIMS + 1
    ix = _index()
    assert lib.sq_build_index(ct.byref(b.grid), ct.byref(p), ct.byref(ix), 0x100000, 1 << 40,
                              None) == L.SQ_ERR_UNSUPPORTED


def test_checkpoint_length_and_chunk_are_checked():
    """ckpt_len must hold ceil(L/K) * rays floats for the call's chunk K, and a
    batched forward writes checkpoints only with a chunk the backward takes."""
    lib = L.load()
    b = _batch()                                  # L = 100, 3 scenes x 2 x 9 x 13 rays
    rays = 3 * 2 * 9 * 13
    io = _batch_io()
    w = L.SqLossWeights(2.0, 0.05)
    for K, chunk in ((4, 0), (8, 8), (16, 16)):
        t = L.SqTuning(8, 4, 0, 0, chunk)
        need = -(-100 // K) * rays
        io.ckpt_len = need - 1
        for rc in (lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
                   lib.sq_batch_render_bwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40, None),
                   lib.sq_batch_render_fwd_loss(ct.byref(b), ct.byref(io), ct.byref(w), ct.byref(t), 0x100000,
                                                1 << 40, None),
                   lib.sq_batch_step(ct.byref(b), ct.byref(io), ct.byref(t), 0x100000, 1 << 40, None)):
            assert rc == L.SQ_ERR_CAPACITY
            assert "ckpt_len" in lib.sq_last_error().decode()
    # the autotuner checks every candidate before timing any
    io.ckpt_len = -(-100 // 8) * rays
    cands = (L.SqTuning * 2)(L.SqTuning(8, 4, 0, 0, 8), L.SqTuning(8, 4, 0, 0, 4))
    best = ct.c_int32(-1)
    assert lib.sq_batch_autotune(ct.byref(b), ct.byref(io), cands, 2, 1, ct.byref(best), None, 0x100000, 1 << 40,
                                 None) == L.SQ_ERR_CAPACITY
    # a chunk the backward cannot take is refused for checkpoints
    io.ckpt_len = 1 << 40
    for chunk in (1, 2, 3, 5, 32):
        t = L.SqTuning(8, 4, 0, 0, chunk)
        assert lib.sq_batch_render_fwd(ct.byref(b), ct.byref(io), None, ct.byref(t), 0x100000, 1 << 40,
                                       None) == L.SQ_ERR_INVALID
        assert lib.sq_batch_render_fwd_loss(ct.byref(b), ct.byref(io), ct.byref(w), ct.byref(t), 0x100000, 1 << 40,
                                            None) == L.SQ_ERR_INVALID


def test_noalloc_forward_refuses_scenes_beyond_its_array_without_touching_the_device():
    """The allocation-free forward checks its scratch need on the host: a scene
    whose workspace exceeds the fixed array, or invalid arguments, are refused
    before any device call (the pointers here are never dereferenced)."""
    lib = L.load()
    big = _prims(n=200000, C=32)
    assert lib.sq_render_workspace(ct.byref(_grid()), ct.byref(big), ct.byref(_rays()),
                                   ct.byref(_march())) > L.SQ_NOALLOC_SCRATCH_BYTES
    t = L.SqTuning(8, 4, 0, 0, 0)
    rc = lib.sq_render_fwd_noalloc(ct.byref(_grid()), ct.byref(_index()), ct.byref(big), ct.byref(_rays()),
                                   ct.byref(_march()), FAKE, FAKE, None, FAKE, None, None, ct.byref(t), None)
    assert rc == L.SQ_ERR_CAPACITY
    assert "fixed" in lib.sq_last_error().decode()
    bad = _grid(nv=-1)
    rc = lib.sq_render_fwd_noalloc(ct.byref(bad), ct.byref(_index()), ct.byref(_prims()), ct.byref(_rays()),
                                   ct.byref(_march()), FAKE, FAKE, None, FAKE, None, None, ct.byref(t), None)
    assert rc == L.SQ_ERR_INVALID

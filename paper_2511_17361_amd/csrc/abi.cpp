// C ABI of the renderer: host-side validation, workspace queries and dispatch
// to the kernel launchers.  Nothing is launched for a rejected call.  Every
// call is a batch of scenes internally; the single-scene entry points build a
// batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/sqr.h"
#include "sqr_internal.h"

namespace {

thread_local char g_err[512] = "";

sq_status fail(sq_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

int32_t sqr::set_error(int32_t code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

namespace {

sq_status ok() {
    g_err[0] = '\0';
    return SQ_OK;
}

sq_status hip_status(hipError_t e, const char* where) {
    if (e != hipSuccess) return fail(SQ_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
    return ok();
}

bool grid_ok(const sq_grid* g) {
    if (!g) return false;
    for (int i = 0; i < 3; ++i)
        if (!(g->dims[i] > 0 && g->dims[i] <= 32767) || !std::isfinite(g->lo[i])) return false;
    return std::isfinite(g->voxel) && g->voxel > 0.0f && g->nv >= 0 && g->nv <= 32767 && g->theta >= 0.0f &&
           g->theta < 1.0f;
}

sq_status check_grid(const sq_grid* g) {
    if (!grid_ok(g))
        return fail(SQ_ERR_INVALID, "invalid grid (dims in [1,32767], voxel > 0, nv >= 0, theta in [0, 1))");
    if ((int64_t)g->dims[0] * g->dims[1] * g->dims[2] >= ((int64_t)1 << 31))
        return fail(SQ_ERR_INVALID, "grid has >= 2^31 voxels");
    return SQ_OK;
}

sqr::GridDev to_dev(const sq_grid* g) {
    sqr::GridDev d;
    d.lox = g->lo[0]; d.loy = g->lo[1]; d.loz = g->lo[2];
    d.inv = 1.0f / g->voxel;   // fl32(1/voxel): x86 SSE division is correctly rounded
    d.X = g->dims[0]; d.Y = g->dims[1]; d.Z = g->dims[2];
    d.nv = g->nv;
    d.vs = g->voxel;
    d.theta = g->theta;
    d.fX = (float)d.X; d.fY = (float)d.Y; d.fZ = (float)d.Z;   // exact: dims are below 2^24
    return d;
}

sq_status check_march(const sq_march* m) {
    if (!m) return fail(SQ_ERR_INVALID, "march is NULL");
    if (m->n_samples < 1 || m->n_samples > (1 << 20))
        return fail(SQ_ERR_INVALID, "n_samples = %d outside [1, 2^20]", m->n_samples);
    if (!std::isfinite(m->t_near) || !std::isfinite(m->t_far) || m->t_near < 0.0f)
        return fail(SQ_ERR_INVALID, "t_near/t_far must be finite and t_near >= 0");
    if (m->n_samples > 1 ? !(m->t_near < m->t_far) : !(m->t_near <= m->t_far))
        return fail(SQ_ERR_INVALID, "need t_near < t_far (got %g, %g)", m->t_near, m->t_far);
    if (m->ckpt_every < 0) return fail(SQ_ERR_INVALID, "ckpt_every < 0");
    if (!(m->kappa >= 0.0f && m->kappa <= 1.0f)) return fail(SQ_ERR_INVALID, "kappa must lie in [0, 1]");
    return SQ_OK;
}

sqr::MarchDev to_dev(const sq_march* m, int K) {
    sqr::MarchDev d;
    d.L = m->n_samples;
    d.t_near = m->t_near;
    // delta = fl32(fl32(t_far - t_near) / fl32(L - 1)), as the pinned sample sequence states
    const float span = m->t_far - m->t_near;
    d.delta = m->n_samples > 1 ? span / (float)(m->n_samples - 1) : 0.0f;
    d.K = K;
    d.kappa = m->kappa;
    return d;
}

sq_tuning default_tuning() {
    sq_tuning t;
    t.tile_w = 8;
    t.waves_per_block = 4;
    t.bwd_mode = SQ_BWD_AUTO;
    t.persistent = 1;
    t.chunk = 0;
    return t;
}

sq_status tuning_of(const sq_tuning* t, sqr::TuneDev& d) {
    sq_tuning v = t ? *t : default_tuning();
    if (!(v.tile_w == 4 || v.tile_w == 8 || v.tile_w == 16))
        return fail(SQ_ERR_INVALID, "tile_w = %d not in {4, 8, 16}", v.tile_w);
    if (v.waves_per_block < 1 || v.waves_per_block > 4)
        return fail(SQ_ERR_INVALID, "waves_per_block = %d not in [1, 4]", v.waves_per_block);
    if (v.bwd_mode < SQ_BWD_AUTO || v.bwd_mode > SQ_BWD_PRIMITIVE_MAJOR)
        return fail(SQ_ERR_INVALID, "bwd_mode = %d not in {0, 1, 2}", v.bwd_mode);
    if (v.persistent < 0 || v.persistent > 1) return fail(SQ_ERR_INVALID, "persistent must be 0 or 1");
    if (v.chunk < 0) return fail(SQ_ERR_INVALID, "chunk < 0");
    d.tile_w = v.tile_w;
    d.waves_per_block = v.waves_per_block;
    d.bwd_mode = v.bwd_mode;
    d.persistent = v.persistent;
    return SQ_OK;
}

// Upper bound of E for n primitives: n * prod_axis min(2 nv + 1, dims).
int64_t index_bound(const sq_grid* g, int32_t n) {
    int64_t per = 1;
    for (int i = 0; i < 3; ++i) {
        const int64_t side = 2 * (int64_t)g->nv + 1;
        per *= side < g->dims[i] ? side : g->dims[i];
    }
    return per * n;
}

// A validated batch: host description plus the per-call constants.
struct Plan {
    sqr::GridDev g;
    sqr::BatchDesc d;
    sq_march m;
};

sq_status make_plan(const sq_batch* b, int tile_w, Plan& p) {
    if (!b) return fail(SQ_ERR_INVALID, "batch is NULL");
    sq_status s;
    if ((s = check_grid(&b->grid))) return s;
    if ((s = check_march(&b->march))) return s;
    if (b->n_scenes < 1 || b->n_scenes > SQ_MAX_SCENES)
        return fail(SQ_ERR_INVALID, "n_scenes = %d outside [1, %d]", b->n_scenes, SQ_MAX_SCENES);
    if (b->n_classes < 1 || b->n_classes > SQ_MAX_CLASSES)
        return fail(SQ_ERR_INVALID, "n_classes = %d outside [1, %d]", b->n_classes, SQ_MAX_CLASSES);
    std::memset(&p.d, 0, sizeof(p.d));
    p.d.n_scenes = b->n_scenes;
    p.d.C = b->n_classes;
    int64_t prims = 0, rays = 0;
    for (int i = 0; i < b->n_scenes; ++i) {
        const sq_scene& sc = b->scenes[i];
        if (sc.n_prims < 0 || sc.n_cams < 0 || sc.height < 0 || sc.width < 0)
            return fail(SQ_ERR_INVALID, "scene %d: negative size", i);
        if (sc.index_capacity < 0) return fail(SQ_ERR_INVALID, "scene %d: index_capacity < 0", i);
        // V_f holds int32 offsets into the scene's ids: every entry the index
        // can hold (the capacity) and every entry it can need (the box bound)
        // must stay addressable by them
        if (sc.index_capacity > INT32_MAX)
            return fail(SQ_ERR_UNSUPPORTED, "scene %d: index_capacity %lld exceeds the int32 offsets of V_f", i,
                        (long long)sc.index_capacity);
        if (sc.n_prims > SQ_MAX_SCENE_PRIMS)
            return fail(SQ_ERR_UNSUPPORTED, "scene %d: %d primitives exceed SQ_MAX_SCENE_PRIMS = %d", i, sc.n_prims,
                        SQ_MAX_SCENE_PRIMS);
        if (index_bound(&b->grid, sc.n_prims) > INT32_MAX)
            return fail(SQ_ERR_UNSUPPORTED,
                        "scene %d: %d primitives can need %lld index entries, beyond the int32 offsets of V_f", i,
                        sc.n_prims, (long long)index_bound(&b->grid, sc.n_prims));
        prims += sc.n_prims;
        rays += (int64_t)sc.n_cams * sc.height * sc.width;
        if (prims >= ((int64_t)1 << 30)) return fail(SQ_ERR_INVALID, "too many primitives");
        if (rays > ((int64_t)1 << 31) / 32) return fail(SQ_ERR_INVALID, "too many rays (%lld)", (long long)rays);
        sqr::SceneDev& S = p.d.s[i];
        S.n = sc.n_prims;
        S.cams = sc.n_cams;
        S.H = sc.height;
        S.W = sc.width;
        S.cap = sc.index_capacity;
    }
    sqr::finish_desc(p.d, tile_w);
    p.g = to_dev(&b->grid);
    p.m = b->march;
    return SQ_OK;
}

// Every autotune candidate checked against the batch before any launch.
sq_status check_candidates(const sq_batch* b, const sq_batch_io* io, const sq_tuning* candidates, int n_candidates,
                           int reps, void* ws, size_t ws_bytes);

// The autotune cache key of a batch (one line, no spaces; floats in hex).
std::string tuning_key(const sq_batch* b) {
    char arch[128] = "nodevice";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
        for (char* c = arch; *c; ++c)
            if (*c == ' ' || *c == '|') *c = '_';
    } else {
        (void)hipGetLastError();
    }
    char t[512];
    const sq_grid& g = b->grid;
    const sq_march& m = b->march;
    std::snprintf(t, sizeof(t), "v%d|%s|C%d|g%dx%dx%d,%a,%a,%a,%a,%d,%a|m%d,%a,%a,%d,%a|S%d", sq_version(), arch,
                  b->n_classes, g.dims[0], g.dims[1], g.dims[2], g.lo[0], g.lo[1], g.lo[2], g.voxel, g.nv, g.theta,
                  m.n_samples, m.t_near, m.t_far, m.ckpt_every, m.kappa, b->n_scenes);
    std::string k = t;
    const int ns = std::max(0, std::min<int>(b->n_scenes, SQ_MAX_SCENES));
    for (int i = 0; i < ns; ++i) {
        const sq_scene& sc = b->scenes[i];
        std::snprintf(t, sizeof(t), "|%d,%d,%d,%d", sc.n_prims, sc.n_cams, sc.height, sc.width);
        k += t;
    }
    return k;
}

sq_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(SQ_ERR_CAPACITY, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % sqr::WS_ALIGN) return fail(SQ_ERR_INVALID, "workspace must be 256-byte aligned");
    return SQ_OK;
}

sq_status check_io_index(const Plan& p, const sq_batch_io* io) {
    if (!io) return fail(SQ_ERR_INVALID, "io is NULL");
    if (!io->counts || !io->offsets) return fail(SQ_ERR_INVALID, "index counts/offsets is NULL");
    int64_t cap = 0;
    for (int i = 0; i < p.d.n_scenes; ++i) cap += p.d.s[i].cap;
    if (cap > 0 && !io->ids) return fail(SQ_ERR_INVALID, "index ids is NULL");
    if (p.d.total_prims > 0 && !io->means) return fail(SQ_ERR_INVALID, "means is NULL");
    return SQ_OK;
}

sq_status check_io_render(const Plan& p, const sq_batch_io* io) {
    sq_status s;
    if ((s = check_io_index(p, io))) return s;
    if (p.d.total_prims > 0 && (!io->quats || !io->scales || !io->eps || !io->opacity || !io->logits))
        return fail(SQ_ERR_INVALID, "a primitive parameter array is NULL");
    if (p.d.total_rays > 0 && (!io->origins || !io->dirs)) return fail(SQ_ERR_INVALID, "ray origins/dirs is NULL");
    return SQ_OK;
}

int chunk_of(const sq_tuning* t, const sq_march& m) {
    if (t && t->chunk > 0) return t->chunk;
    return m.ckpt_every;
}

sqr::BatchIO to_dev(const sq_batch_io* io) {
    sqr::BatchIO b;
    std::memset(&b, 0, sizeof(b));
    b.means = io->means; b.quats = io->quats; b.scales = io->scales; b.eps = io->eps;
    b.opacity = io->opacity; b.logits = io->logits; b.origins = io->origins; b.dirs = io->dirs;
    b.counts = io->counts; b.offsets = io->offsets; b.ids = io->ids; b.totals = io->totals;
    b.depth = io->depth; b.sem = io->sem; b.probs = io->probs; b.t_final = io->t_final; b.ckpt = io->ckpt;
    b.g_depth = io->g_depth; b.g_sem = io->g_sem;
    b.g_means = io->g_means; b.g_quats = io->g_quats; b.g_scales = io->g_scales; b.g_eps = io->g_eps;
    b.g_opacity = io->g_opacity; b.g_logits = io->g_logits;
    b.vox_density = io->vox_density; b.vox_sem = io->vox_sem; b.vox_labels = io->vox_labels;
    b.sem_label = io->sem_label; b.depth_label = io->depth_label; b.loss = io->loss;
    b.tile_stop = io->tile_stop;
    b.stash = io->stash; b.stash_len = io->stash_len;
    return b;
}

sq_status index_checked(const Plan& p, const sq_batch_io* io, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_io_index(p, io))) return s;
    if (!io->totals) return fail(SQ_ERR_INVALID, "index totals is NULL");
    // the influence-thresholded boxes read every primitive parameter but the logits
    if (p.g.theta > 0.0f && p.d.total_prims > 0 && (!io->quats || !io->scales || !io->eps || !io->opacity))
        return fail(SQ_ERR_INVALID, "theta > 0 needs quats, scales, eps and opacity for the index");
    if ((s = check_ws(ws, ws_bytes, sqr::index_workspace_bytes(p.g, p.d)))) return s;
    return hip_status(sqr::launch_batch_index(p.g, p.d, to_dev(io), ws, stream), "build_index");
}

// The per-tile stops (nullable): a header and one entry per tile of this tiling.
sq_status check_tile_stop(const Plan& p, const sq_batch_io* io) {
    if (!io->tile_stop) return SQ_OK;
    const int64_t need = 4 + (int64_t)p.d.total_tiles;
    if (io->tile_stop_len < need)
        return fail(SQ_ERR_CAPACITY, "tile_stop_len %lld < %lld for this tiling", (long long)io->tile_stop_len,
                    (long long)need);
    return SQ_OK;
}

// The per-sample stash (nullable): at least its header, and for a call that
// reads or writes it with chunk K (> 0) its slot table for this tiling.
sq_status check_stash(const Plan& p, const sq_batch_io* io, int K) {
    if (!io->stash) return SQ_OK;
    const int64_t need = K > 0 ? sqr::stash_geom(p.d, p.m.n_samples, K).pool_off : sqr::STASH_HEAD;
    if (io->stash_len < need)
        return fail(SQ_ERR_CAPACITY, "stash_len %lld < %lld floats (header and slot table) for this tiling",
                    (long long)io->stash_len, (long long)need);
    return SQ_OK;
}

// The checkpoints of a chunk K: ceil(L/K) rows of every ray of the batch must
// fit the caller's ckpt_len floats.
sq_status check_ckpt(const Plan& p, const sq_batch_io* io, int K) {
    if (!io->ckpt) return SQ_OK;
    if (K < 1) return fail(SQ_ERR_INVALID, "ckpt given but the checkpoint spacing is < 1");
    const int64_t need = (int64_t)((p.m.n_samples + K - 1) / K) * p.d.total_rays;
    if (io->ckpt_len < need)
        return fail(SQ_ERR_CAPACITY, "ckpt_len %lld < %lld floats for chunk %d", (long long)io->ckpt_len,
                    (long long)need, K);
    return SQ_OK;
}

bool chunk_ok(int K) { return K == 4 || K == 8 || K == 16; }

sq_status fwd_checked(const Plan& p, const sq_batch_io* io, int64_t* stats, const sq_tuning* tuning, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_io_render(p, io))) return s;
    if (p.d.total_rays > 0 && (!io->depth || !io->sem || !io->t_final))
        return fail(SQ_ERR_INVALID, "depth/sem/t_final is NULL");
    const int K = chunk_of(tuning, p.m);
    if ((s = check_ckpt(p, io, K))) return s;
    if ((s = check_tile_stop(p, io))) return s;
    if ((s = check_stash(p, io, io->ckpt ? K : 0))) return s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
    const hipError_t e = sqr::launch_batch_fwd(p.g, p.d, to_dev(&p.m, io->ckpt ? K : 0), to_dev(io), stats, tune,
                                               ws, stream);
    return hip_status(e, "render_fwd");
}

sq_status bwd_checked(const Plan& p, const sq_batch_io* io, int64_t* stats, const sq_tuning* tuning, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_io_render(p, io))) return s;
    const int K = chunk_of(tuning, p.m);
    if (!chunk_ok(K))
        return fail(SQ_ERR_INVALID, "backward needs a checkpoint spacing in {4, 8, 16} (got %d)", K);
    if (p.d.total_rays > 0 && !io->ckpt) return fail(SQ_ERR_INVALID, "ckpt is NULL");
    if ((s = check_ckpt(p, io, K))) return s;
    if (p.d.total_prims > 0 && (!io->g_means || !io->g_quats || !io->g_scales || !io->g_eps || !io->g_opacity ||
                                !io->g_logits))
        return fail(SQ_ERR_INVALID, "a gradient output array is NULL");
    if ((s = check_tile_stop(p, io))) return s;
    if ((s = check_stash(p, io, K))) return s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if (tune.bwd_mode == SQ_BWD_PRIMITIVE_MAJOR &&
        !sqr::bwd_primitive_major_ok(p.g, p.d.max_n, K, tune.waves_per_block))
        return fail(SQ_ERR_UNSUPPORTED, "primitive-major backward does not apply (chunk %d, max n %d)", K,
                    p.d.max_n);
    if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
    const hipError_t e = sqr::launch_batch_bwd(p.g, p.d, to_dev(&p.m, K), to_dev(io), stats, tune, ws, stream);
    return hip_status(e, "render_bwd");
}

sq_status check_loss(const Plan& p, const sq_batch_io* io, const sq_loss_weights* w) {
    if (!w) return fail(SQ_ERR_INVALID, "loss weights are NULL");
    if (!std::isfinite(w->lambda_sem) || !std::isfinite(w->lambda_depth))
        return fail(SQ_ERR_INVALID, "loss weights must be finite");
    if (!io->loss) return fail(SQ_ERR_INVALID, "loss output is NULL");
    if (p.d.total_rays > 0 && (!io->sem_label || !io->depth_label))
        return fail(SQ_ERR_INVALID, "semantic/depth labels are NULL");
    if (p.d.total_rays > 0 && (!io->g_depth || !io->g_sem))
        return fail(SQ_ERR_INVALID, "g_depth/g_sem (written by the fused loss) are NULL");
    return SQ_OK;
}

sq_status fwd_loss_checked(const Plan& p, const sq_batch_io* io, const sq_loss_weights* w,
                           const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_io_render(p, io))) return s;
    if (p.d.total_rays > 0 && (!io->depth || !io->sem || !io->t_final))
        return fail(SQ_ERR_INVALID, "depth/sem/t_final is NULL");
    if ((s = check_loss(p, io, w))) return s;
    const int K = chunk_of(tuning, p.m);
    if ((s = check_ckpt(p, io, K))) return s;
    if ((s = check_tile_stop(p, io))) return s;
    if ((s = check_stash(p, io, io->ckpt ? K : 0))) return s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
    const sqr::LossArgs la{w->lambda_sem, w->lambda_depth};
    const hipError_t e = sqr::launch_batch_fwd(p.g, p.d, to_dev(&p.m, io->ckpt ? K : 0), to_dev(io), nullptr, tune,
                                               ws, stream, &la);
    return hip_status(e, "render_fwd_loss");
}

sq_status vox_checked(const Plan& p, const sq_batch_io* io, float tau, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
    sq_status s;
    if ((s = check_io_index(p, io))) return s;
    if (p.d.total_prims > 0 && (!io->quats || !io->scales || !io->eps || !io->opacity || !io->logits))
        return fail(SQ_ERR_INVALID, "a primitive parameter array is NULL");
    if (!std::isfinite(tau)) return fail(SQ_ERR_INVALID, "tau must be finite");
    if (!io->vox_density) return fail(SQ_ERR_INVALID, "density output is NULL");
    if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
    return hip_status(sqr::launch_batch_voxelise(p.g, p.d, to_dev(io), tau, ws, stream), "voxelise");
}

// ---- single-scene adapters --------------------------------------------------
void one_scene(const sq_grid* grid, const sq_march* march, int n, int C, int cams, int H, int W, int64_t cap,
               sq_batch& b) {
    std::memset(&b, 0, sizeof(b));
    b.n_scenes = 1;
    b.n_classes = C;
    b.grid = *grid;
    b.march = *march;
    b.scenes[0].n_prims = n;
    b.scenes[0].n_cams = cams;
    b.scenes[0].height = H;
    b.scenes[0].width = W;
    b.scenes[0].index_capacity = cap;
}

sq_status check_prims(const sq_prims* p, bool need_params) {
    if (!p) return fail(SQ_ERR_INVALID, "prims is NULL");
    if (p->n < 0) return fail(SQ_ERR_INVALID, "prims->n = %d < 0", p->n);
    if (need_params && (p->n_classes < 1 || p->n_classes > SQ_MAX_CLASSES))
        return fail(SQ_ERR_INVALID, "n_classes = %d outside [1, %d]", p->n_classes, SQ_MAX_CLASSES);
    if (p->n > 0) {
        if (!p->means) return fail(SQ_ERR_INVALID, "prims->means is NULL");
        if (need_params && (!p->quats || !p->scales || !p->eps || !p->opacity || !p->logits))
            return fail(SQ_ERR_INVALID, "a primitive parameter array is NULL");
    }
    return SQ_OK;
}

sq_status check_rays(const sq_rays* r) {
    if (!r) return fail(SQ_ERR_INVALID, "rays is NULL");
    if (r->n_cams < 0 || r->height < 0 || r->width < 0) return fail(SQ_ERR_INVALID, "negative ray dimensions");
    const int64_t n = (int64_t)r->n_cams * r->height * r->width;
    if (n > 0 && (!r->origins || !r->dirs)) return fail(SQ_ERR_INVALID, "ray origins/dirs is NULL");
    return SQ_OK;
}

sq_status check_index(const sq_index* idx, bool for_render) {
    if (!idx) return fail(SQ_ERR_INVALID, "index is NULL");
    if (!idx->counts || !idx->offsets) return fail(SQ_ERR_INVALID, "index counts/offsets is NULL");
    if (idx->capacity < 0) return fail(SQ_ERR_INVALID, "index capacity < 0");
    if (idx->capacity > 0 && !idx->ids) return fail(SQ_ERR_INVALID, "index ids is NULL");
    if (!for_render && !idx->total) return fail(SQ_ERR_INVALID, "index total is NULL");
    return SQ_OK;
}

void io_from(const sq_index* idx, const sq_prims* pr, const sq_rays* rays, sq_batch_io& io) {
    std::memset(&io, 0, sizeof(io));
    io.means = pr->means; io.quats = pr->quats; io.scales = pr->scales; io.eps = pr->eps;
    io.opacity = pr->opacity; io.logits = pr->logits;
    if (rays) { io.origins = rays->origins; io.dirs = rays->dirs; }
    io.counts = idx->counts; io.offsets = idx->offsets; io.ids = idx->ids; io.totals = idx->total;
}

// Rows of the single-scene checkpoint layout [ceil(L/K), R] (0 without checkpoints).
sq_status check_candidates(const sq_batch* b, const sq_batch_io* io, const sq_tuning* candidates, int n_candidates,
                           int reps, void* ws, size_t ws_bytes) {
    if (!candidates || n_candidates < 1 || reps < 1)
        return fail(SQ_ERR_INVALID, "need candidates, n_candidates >= 1 and reps >= 1");
    // an invalid candidate rejects the call before any launch
    for (int i = 0; i < n_candidates; ++i) {
        sqr::TuneDev tune;
        sq_status s;
        if ((s = tuning_of(&candidates[i], tune))) return s;
        Plan p;
        if ((s = make_plan(b, tune.tile_w, p))) return s;
        if ((s = check_io_render(p, io))) return s;
        if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
        const int K = chunk_of(&candidates[i], p.m);
        if (!chunk_ok(K)) return fail(SQ_ERR_INVALID, "candidate %d: chunk %d", i, K);
        if (!io->ckpt) return fail(SQ_ERR_INVALID, "autotune times full steps: ckpt is NULL");
        if ((s = check_ckpt(p, io, K))) return s;
        if ((s = check_tile_stop(p, io))) return s;
        if ((s = check_stash(p, io, K))) return s;
        if (tune.bwd_mode == SQ_BWD_PRIMITIVE_MAJOR &&
            !sqr::bwd_primitive_major_ok(p.g, p.d.max_n, K, tune.waves_per_block))
            return fail(SQ_ERR_UNSUPPORTED, "candidate %d: primitive-major backward does not apply", i);
    }
    return SQ_OK;
}

int64_t ckpt_rows(const sq_march* m) {
    return m->ckpt_every > 0 ? (m->n_samples + m->ckpt_every - 1) / m->ckpt_every : 0;
}

struct GraphImpl {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

const sq_march kIndexMarch = {1, 0.0f, 1.0f, 0, 0.0f};

}  // namespace

extern "C" {

const char* sq_last_error(void) { return g_err; }

int32_t sq_version(void) { return 209; }

sq_tuning sq_default_tuning(void) { return default_tuning(); }

int64_t sq_index_capacity_bound(const sq_grid* grid, int32_t n) {
    if (!grid_ok(grid) || n < 0) return -1;
    return index_bound(grid, n);
}

size_t sq_build_index_workspace(const sq_grid* grid, int32_t n) {
    if (!grid_ok(grid) || n < 0) return 0;
    sq_batch b;
    one_scene(grid, &kIndexMarch, n, 1, 0, 0, 0, 0, b);
    Plan p;
    if (make_plan(&b, 8, p)) return 0;
    return sqr::index_workspace_bytes(p.g, p.d);
}

sq_status sq_build_index(const sq_grid* grid, const sq_prims* prims, sq_index* idx, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_prims(prims, false))) return s;
    if ((s = check_index(idx, false))) return s;
    sq_batch b;
    one_scene(grid, &kIndexMarch, prims->n, 1, 0, 0, 0, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, 8, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, nullptr, io);
    return index_checked(p, &io, ws, ws_bytes, stream);
}

size_t sq_render_workspace(const sq_grid* grid, const sq_prims* prims, const sq_rays* rays, const sq_march* march) {
    if (!grid_ok(grid) || !prims || prims->n < 0 || prims->n_classes < 1 || prims->n_classes > SQ_MAX_CLASSES)
        return 0;
    sq_batch b;
    const sq_march m = march ? *march : kIndexMarch;
    const int cams = rays ? rays->n_cams : 0, H = rays ? rays->height : 0, W = rays ? rays->width : 0;
    one_scene(grid, &m, prims->n, prims->n_classes, cams, H, W, 0, b);
    Plan p;
    if (make_plan(&b, 8, p)) return 0;
    return sqr::batch_workspace_bytes(p.g, p.d);
}

sq_status sq_render_fwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, const sq_rays* rays,
                        const sq_march* march, float* depth, float* sem, float* probs, float* t_final, float* ckpt,
                        int64_t* stats, const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    if ((s = check_rays(rays))) return s;
    if ((s = check_march(march))) return s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if (ckpt && march->ckpt_every < 1) return fail(SQ_ERR_INVALID, "ckpt given but ckpt_every < 1");
    sq_batch b;
    one_scene(grid, march, prims->n, prims->n_classes, rays->n_cams, rays->height, rays->width, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, tune.tile_w, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, rays, io);
    io.depth = depth; io.sem = sem; io.probs = probs; io.t_final = t_final; io.ckpt = ckpt;
    io.ckpt_len = ckpt_rows(march) * p.d.total_rays;     // [ceil(L/K), R] by this call's contract
    sq_tuning t = tuning ? *tuning : default_tuning();
    t.chunk = march->ckpt_every;
    return fwd_checked(p, &io, stats, &t, ws, ws_bytes, stream);
}

sq_status sq_render_bwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, const sq_rays* rays,
                        const sq_march* march, const float* ckpt, const float* g_depth, const float* g_sem,
                        const sq_grads* grads, int64_t* stats, const sq_tuning* tuning, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    if ((s = check_rays(rays))) return s;
    if ((s = check_march(march))) return s;
    if (!(march->ckpt_every == 4 || march->ckpt_every == 8 || march->ckpt_every == 16))
        return fail(SQ_ERR_INVALID, "backward needs ckpt_every in {4, 8, 16} (got %d)", march->ckpt_every);
    const int64_t nr = (int64_t)rays->n_cams * rays->height * rays->width;
    if (nr > 0 && !ckpt) return fail(SQ_ERR_INVALID, "ckpt is NULL");
    if (!grads) return fail(SQ_ERR_INVALID, "grads is NULL");
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    sq_batch b;
    one_scene(grid, march, prims->n, prims->n_classes, rays->n_cams, rays->height, rays->width, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, tune.tile_w, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, rays, io);
    io.ckpt = const_cast<float*>(ckpt);
    io.ckpt_len = ckpt_rows(march) * p.d.total_rays;
    io.g_depth = g_depth; io.g_sem = g_sem;
    io.g_means = grads->means; io.g_quats = grads->quats; io.g_scales = grads->scales; io.g_eps = grads->eps;
    io.g_opacity = grads->opacity; io.g_logits = grads->logits;
    sq_tuning t = tuning ? *tuning : default_tuning();
    t.chunk = march->ckpt_every;
    return bwd_checked(p, &io, stats, &t, ws, ws_bytes, stream);
}

sq_status sq_render_fwd_loss(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, const sq_rays* rays,
                             const sq_march* march, const sq_loss_weights* weights, const int32_t* sem_label,
                             const float* depth_label, float* depth, float* sem, float* probs, float* t_final,
                             float* ckpt, float* g_depth, float* g_sem, float* loss, const sq_tuning* tuning,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    if ((s = check_rays(rays))) return s;
    if ((s = check_march(march))) return s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if (ckpt && march->ckpt_every < 1) return fail(SQ_ERR_INVALID, "ckpt given but ckpt_every < 1");
    sq_batch b;
    one_scene(grid, march, prims->n, prims->n_classes, rays->n_cams, rays->height, rays->width, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, tune.tile_w, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, rays, io);
    io.depth = depth; io.sem = sem; io.probs = probs; io.t_final = t_final; io.ckpt = ckpt;
    io.ckpt_len = ckpt_rows(march) * p.d.total_rays;
    io.sem_label = sem_label; io.depth_label = depth_label; io.g_depth = g_depth; io.g_sem = g_sem; io.loss = loss;
    sq_tuning t = tuning ? *tuning : default_tuning();
    t.chunk = march->ckpt_every;
    return fwd_loss_checked(p, &io, weights, &t, ws, ws_bytes, stream);
}

size_t sq_sq_major_workspace(const sq_grid* grid, const sq_prims* prims, const sq_rays* rays, const sq_march* march,
                             int64_t capacity) {
    if (!grid_ok(grid) || !prims || !rays || !march || capacity < 0 || prims->n < 0 || prims->n_classes < 1 ||
        prims->n_classes > SQ_MAX_CLASSES)
        return 0;
    sq_batch b;
    one_scene(grid, march, prims->n, prims->n_classes, rays->n_cams, rays->height, rays->width, 0, b);
    Plan p;
    if (make_plan(&b, 8, p)) return 0;
    return sqr::sq_major_workspace_bytes(p.g, p.d, to_dev(march, march->ckpt_every), capacity);
}

sq_status sq_render_bwd_sq_major(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                                 const sq_rays* rays, const sq_march* march, const float* ckpt,
                                 const float* g_depth, const float* g_sem, const sq_grads* grads, int64_t capacity,
                                 int64_t* interactions, void* iws, size_t iws_bytes, const sq_tuning* tuning,
                                 void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    if ((s = check_rays(rays))) return s;
    if ((s = check_march(march))) return s;
    if (!(march->ckpt_every == 4 || march->ckpt_every == 8 || march->ckpt_every == 16))
        return fail(SQ_ERR_INVALID, "backward needs ckpt_every in {4, 8, 16} (got %d)", march->ckpt_every);
    const int64_t nr = (int64_t)rays->n_cams * rays->height * rays->width;
    if (nr > 0 && !ckpt) return fail(SQ_ERR_INVALID, "ckpt is NULL");
    if (!grads) return fail(SQ_ERR_INVALID, "grads is NULL");
    if (!interactions) return fail(SQ_ERR_INVALID, "interactions (device int64) is NULL");
    if (capacity < 0 || capacity > ((int64_t)1 << 40)) return fail(SQ_ERR_INVALID, "capacity out of range");
    if (nr * (int64_t)march->n_samples >= ((int64_t)1 << 32))
        return fail(SQ_ERR_UNSUPPORTED, "rays x samples must stay below 2^32 for the interaction ids");
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    sq_batch b;
    one_scene(grid, march, prims->n, prims->n_classes, rays->n_cams, rays->height, rays->width, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, tune.tile_w, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, rays, io);
    io.ckpt = const_cast<float*>(ckpt);
    io.ckpt_len = ckpt_rows(march) * p.d.total_rays;
    io.g_depth = g_depth; io.g_sem = g_sem;
    io.g_means = grads->means; io.g_quats = grads->quats; io.g_scales = grads->scales; io.g_eps = grads->eps;
    io.g_opacity = grads->opacity; io.g_logits = grads->logits;
    if (p.d.total_prims > 0 && (!io.g_means || !io.g_quats || !io.g_scales || !io.g_eps || !io.g_opacity ||
                                !io.g_logits))
        return fail(SQ_ERR_INVALID, "a gradient output array is NULL");
    if ((s = check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d)))) return s;
    const sqr::MarchDev md = to_dev(march, march->ckpt_every);
    const size_t need = sqr::sq_major_workspace_bytes(p.g, p.d, md, capacity);
    if (!iws || iws_bytes < need) return fail(SQ_ERR_CAPACITY, "interaction workspace %zu < %zu bytes", iws_bytes, need);
    if ((uintptr_t)iws % sqr::WS_ALIGN) return fail(SQ_ERR_INVALID, "interaction workspace must be 256-byte aligned");
    const hipError_t e = sqr::launch_batch_bwd_sq_major(p.g, p.d, md, to_dev(&io), capacity, interactions, iws, tune,
                                                        ws, stream);
    return hip_status(e, "render_bwd_sq_major");
}

size_t sq_voxelise_workspace(const sq_grid* grid, const sq_prims* prims) {
    return sq_render_workspace(grid, prims, nullptr, nullptr);
}

sq_status sq_voxelise(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, float tau, float* density,
                      float* sem, int32_t* labels, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_grid(grid))) return s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    sq_batch b;
    one_scene(grid, &kIndexMarch, prims->n, prims->n_classes, 0, 0, 0, idx->capacity, b);
    Plan p;
    if ((s = make_plan(&b, 8, p))) return s;
    sq_batch_io io;
    io_from(idx, prims, nullptr, io);
    io.vox_density = density; io.vox_sem = sem; io.vox_labels = labels;
    return vox_checked(p, &io, tau, ws, ws_bytes, stream);
}

// ---- batched -------------------------------------------------------------------
int64_t sq_batch_tile_stop_len(const sq_batch* b, const sq_tuning* tuning) {
    sqr::TuneDev tune;
    if (tuning_of(tuning, tune)) return 0;
    Plan p;
    if (make_plan(b, tune.tile_w, p)) return 0;
    return 4 + (int64_t)p.d.total_tiles;
}

int64_t sq_batch_stash_len(const sq_batch* b, const sq_tuning* tuning, int64_t slots) {
    sqr::TuneDev tune;
    if (slots < 0 || tuning_of(tuning, tune)) return 0;
    Plan p;
    if (make_plan(b, tune.tile_w, p)) return 0;
    const int K = chunk_of(tuning, p.m);
    if (!chunk_ok(K)) return 0;
    const sqr::StashGeom g = sqr::stash_geom(p.d, p.m.n_samples, K);
    if (slots > (int64_t)INT32_MAX || slots > (INT64_MAX - g.pool_off) / g.slot_floats) return 0;
    return g.pool_off + slots * g.slot_floats;
}

size_t sq_batch_workspace(const sq_batch* b) {
    Plan p;
    if (make_plan(b, 4, p)) return 0;
    return sqr::batch_workspace_bytes(p.g, p.d);
}

sq_status sq_batch_build_index(const sq_batch* b, const sq_batch_io* io, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
    Plan p;
    sq_status s;
    if ((s = make_plan(b, 8, p))) return s;
    return index_checked(p, io, ws, ws_bytes, stream);
}

sq_status sq_batch_render_fwd(const sq_batch* b, const sq_batch_io* io, int64_t* stats, const sq_tuning* tuning,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
    sqr::TuneDev tune;
    sq_status s;
    if ((s = tuning_of(tuning, tune))) return s;
    Plan p;
    if ((s = make_plan(b, tune.tile_w, p))) return s;
    if (io && io->ckpt && !chunk_ok(chunk_of(tuning, p.m)))
        return fail(SQ_ERR_INVALID, "checkpoints need a chunk in {4, 8, 16} (got %d)", chunk_of(tuning, p.m));
    return fwd_checked(p, io, stats, tuning, ws, ws_bytes, stream);
}

sq_status sq_batch_render_fwd_loss(const sq_batch* b, const sq_batch_io* io, const sq_loss_weights* weights,
                                   const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream) {
    sqr::TuneDev tune;
    sq_status s;
    if ((s = tuning_of(tuning, tune))) return s;
    Plan p;
    if ((s = make_plan(b, tune.tile_w, p))) return s;
    if (io && io->ckpt && !chunk_ok(chunk_of(tuning, p.m)))
        return fail(SQ_ERR_INVALID, "checkpoints need a chunk in {4, 8, 16} (got %d)", chunk_of(tuning, p.m));
    return fwd_loss_checked(p, io, weights, tuning, ws, ws_bytes, stream);
}

sq_status sq_batch_voxelise(const sq_batch* b, const sq_batch_io* io, float tau, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
    sq_status s;
    Plan p;
    if ((s = make_plan(b, 8, p))) return s;
    return vox_checked(p, io, tau, ws, ws_bytes, stream);
}

sq_status sq_batch_render_bwd(const sq_batch* b, const sq_batch_io* io, int64_t* stats, const sq_tuning* tuning,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
    sqr::TuneDev tune;
    sq_status s;
    if ((s = tuning_of(tuning, tune))) return s;
    Plan p;
    if ((s = make_plan(b, tune.tile_w, p))) return s;
    return bwd_checked(p, io, stats, tuning, ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

// Validates every stage of a step (index, forward, backward; with `w`, the
// fused loss too) before the first launch.
sq_status check_step(const sq_batch* b, const sq_batch_io* io, const sq_tuning* tuning, const sq_loss_weights* w,
                     void* ws, size_t ws_bytes) {
    sq_status s;
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    Plan p;
    if ((s = make_plan(b, tune.tile_w, p))) return s;
    if ((s = check_io_render(p, io))) return s;
    if (!io->totals || !io->depth || !io->sem || !io->t_final || !io->ckpt || !io->g_means || !io->g_quats ||
        !io->g_scales || !io->g_eps || !io->g_opacity || !io->g_logits)
        return fail(SQ_ERR_INVALID, "a step needs totals, forward outputs, ckpt and gradient outputs");
    if (w && (s = check_loss(p, io, w))) return s;
    const int K = chunk_of(tuning, p.m);
    if (!chunk_ok(K)) return fail(SQ_ERR_INVALID, "step needs a chunk in {4, 8, 16}");
    if ((s = check_ckpt(p, io, K))) return s;
    if ((s = check_tile_stop(p, io))) return s;
    if ((s = check_stash(p, io, K))) return s;
    if (tune.bwd_mode == SQ_BWD_PRIMITIVE_MAJOR &&
        !sqr::bwd_primitive_major_ok(p.g, p.d.max_n, K, tune.waves_per_block))
        return fail(SQ_ERR_UNSUPPORTED, "primitive-major backward does not apply");
    return check_ws(ws, ws_bytes, sqr::batch_workspace_bytes(p.g, p.d));
}

// Captures `launch(stream)` into an instantiated graph.
template <typename F>
sq_status capture_graph(hipStream_t stream, sq_graph* out, F&& launch) {
    if (!out) return fail(SQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!stream) return fail(SQ_ERR_INVALID, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e, "hipStreamBeginCapture");
    const sq_status st = launch(stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(stream, &graph);
    if (st != SQ_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_status(e, "hipGraphInstantiate");
    }
    GraphImpl* g = new (std::nothrow) GraphImpl{graph, exec};
    if (!g) {
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        return fail(SQ_ERR_HIP, "out of host memory");
    }
    *out = reinterpret_cast<sq_graph>(g);
    return ok();
}

}  // namespace

extern "C" {

sq_status sq_batch_step(const sq_batch* b, const sq_batch_io* io, const sq_tuning* tuning, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_step(b, io, tuning, nullptr, ws, ws_bytes))) return s;
    if ((s = sq_batch_build_index(b, io, ws, ws_bytes, stream))) return s;
    if ((s = sq_batch_render_fwd(b, io, nullptr, tuning, ws, ws_bytes, stream))) return s;
    return sq_batch_render_bwd(b, io, nullptr, tuning, ws, ws_bytes, stream);
}

sq_status sq_batch_train_step(const sq_batch* b, const sq_batch_io* io, const sq_loss_weights* weights,
                              const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s;
    if ((s = check_step(b, io, tuning, weights, ws, ws_bytes))) return s;
    if ((s = sq_batch_build_index(b, io, ws, ws_bytes, stream))) return s;
    if ((s = sq_batch_render_fwd_loss(b, io, weights, tuning, ws, ws_bytes, stream))) return s;
    return sq_batch_render_bwd(b, io, nullptr, tuning, ws, ws_bytes, stream);
}

sq_status sq_batch_step_graph_create(const sq_batch* b, const sq_batch_io* io, const sq_tuning* tuning, void* ws,
                                     size_t ws_bytes, hipStream_t stream, sq_graph* out) {
    return capture_graph(stream, out, [&](hipStream_t st) { return sq_batch_step(b, io, tuning, ws, ws_bytes, st); });
}

sq_status sq_batch_train_graph_create(const sq_batch* b, const sq_batch_io* io, const sq_loss_weights* weights,
                                      const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream,
                                      sq_graph* out) {
    return capture_graph(stream, out, [&](hipStream_t st) {
        return sq_batch_train_step(b, io, weights, tuning, ws, ws_bytes, st);
    });
}

sq_status sq_graph_launch(sq_graph graph, hipStream_t stream) {
    if (!graph) return fail(SQ_ERR_INVALID, "graph is NULL");
    GraphImpl* g = reinterpret_cast<GraphImpl*>(graph);
    return hip_status(hipGraphLaunch(g->exec, stream), "hipGraphLaunch");
}

sq_status sq_graph_destroy(sq_graph graph) {
    if (!graph) return ok();
    GraphImpl* g = reinterpret_cast<GraphImpl*>(graph);
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
    return ok();
}

sq_status sq_batch_autotune(const sq_batch* b, const sq_batch_io* io, const sq_tuning* candidates,
                            int32_t n_candidates, int32_t reps, int32_t* best_index, float* ms_per_candidate,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!best_index) return fail(SQ_ERR_INVALID, "best_index is NULL");
    sq_status st = check_candidates(b, io, candidates, n_candidates, reps, ws, ws_bytes);
    if (st) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(SQ_ERR_HIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(SQ_ERR_HIP, "hipEventCreate");
    }
    float best = 0.0f;
    int bi = -1;
    for (int i = 0; i < n_candidates && st == SQ_OK; ++i) {
        st = sq_batch_step(b, io, &candidates[i], ws, ws_bytes, stream);   // warm-up
        if (st) break;
        hipEventRecord(e0, stream);
        for (int r = 0; r < reps && st == SQ_OK; ++r) st = sq_batch_step(b, io, &candidates[i], ws, ws_bytes, stream);
        hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = fail(SQ_ERR_HIP, "hipEventSynchronize");
            break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (ms_per_candidate) ms_per_candidate[i] = ms;
        if (bi < 0 || ms < best) {
            best = ms;
            bi = i;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    *best_index = bi;
    return ok();
}

int32_t sq_batch_tuning_key(const sq_batch* b, char* buf, int32_t n) {
    if (!b) return -1;
    const std::string k = tuning_key(b);
    if (buf && n > 0) {
        const size_t m = std::min<size_t>((size_t)n - 1, k.size());
        std::memcpy(buf, k.data(), m);
        buf[m] = '\0';
    }
    return (int32_t)k.size();
}

sq_status sq_batch_autotune_cached(const sq_batch* b, const sq_batch_io* io, const sq_tuning* candidates,
                                   int32_t n_candidates, int32_t reps, const char* cache_path, sq_tuning* best,
                                   int32_t* from_cache, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!best) return fail(SQ_ERR_INVALID, "best is NULL");
    sq_status st = check_candidates(b, io, candidates, n_candidates, reps, ws, ws_bytes);
    if (st) return st;
    const std::string key = tuning_key(b);
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[4096];
            bool hit = false;
            sq_tuning found{};
            while (std::fgets(line, sizeof(line), f)) {
                const char* sep = std::strstr(line, " => ");
                if (!sep || (size_t)(sep - line) != key.size() || std::strncmp(line, key.c_str(), key.size()) != 0)
                    continue;
                sq_tuning t{};
                if (std::sscanf(sep + 4, "%d %d %d %d %d", &t.tile_w, &t.waves_per_block, &t.bwd_mode, &t.persistent,
                                &t.chunk) != 5)
                    continue;
                sqr::TuneDev td;
                if (tuning_of(&t, td)) continue;    // (a line this library cannot run is skipped)
                found = t;                          // the last matching line wins
                hit = true;
            }
            std::fclose(f);
            if (hit) {
                *best = found;
                if (from_cache) *from_cache = 1;
                return ok();
            }
        }
    }
    int32_t bi = -1;
    if ((st = sq_batch_autotune(b, io, candidates, n_candidates, reps, &bi, nullptr, ws, ws_bytes, stream))) return st;
    *best = candidates[bi];
    if (from_cache) *from_cache = 0;
    ok();
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f || std::fprintf(f, "%s => %d %d %d %d %d\n", key.c_str(), best->tile_w, best->waves_per_block,
                               best->bwd_mode, best->persistent, best->chunk) < 0)
            fail(SQ_ERR_INVALID, "autotune cache %s not written", cache_path);   // reported, result still valid
        if (f) std::fclose(f);
    }
    return SQ_OK;
}

}  // extern "C"

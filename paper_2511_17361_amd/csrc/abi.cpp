// C ABI of the renderer: host-side validation, workspace queries and dispatch
// to the kernel launchers.  Nothing is launched for a rejected call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

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
    return std::isfinite(g->voxel) && g->voxel > 0.0f && g->nv >= 0 && g->nv <= 32767;
}

sqr::GridDev to_dev(const sq_grid* g) {
    sqr::GridDev d;
    d.lox = g->lo[0]; d.loy = g->lo[1]; d.loz = g->lo[2];
    d.inv = 1.0f / g->voxel;   // fl32(1/voxel): x86 SSE division is correctly rounded
    d.X = g->dims[0]; d.Y = g->dims[1]; d.Z = g->dims[2];
    d.nv = g->nv;
    return d;
}

int64_t nvox(const sq_grid* g) { return (int64_t)g->dims[0] * g->dims[1] * g->dims[2]; }

sq_status check_prims(const sq_prims* p, bool need_params) {
    if (!p) return fail(SQ_ERR_INVALID, "prims is NULL");
    if (p->n < 0) return fail(SQ_ERR_INVALID, "prims->n = %d < 0", p->n);
    if (p->n_classes < 1 || p->n_classes > SQ_MAX_CLASSES)
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
    if (r->n_cams < 0 || r->height < 0 || r->width < 0)
        return fail(SQ_ERR_INVALID, "negative ray dimensions");
    const int64_t n = (int64_t)r->n_cams * r->height * r->width;
    if (n > ((int64_t)1 << 31) / 32) return fail(SQ_ERR_INVALID, "too many rays (%lld)", (long long)n);
    if (n > 0 && (!r->origins || !r->dirs)) return fail(SQ_ERR_INVALID, "ray origins/dirs is NULL");
    return SQ_OK;
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
    return SQ_OK;
}

sqr::MarchDev to_dev(const sq_march* m) {
    sqr::MarchDev d;
    d.L = m->n_samples;
    d.t_near = m->t_near;
    // delta = fl32(fl32(t_far - t_near) / fl32(L - 1)), as the pinned sample sequence states
    const float span = m->t_far - m->t_near;
    d.delta = m->n_samples > 1 ? span / (float)(m->n_samples - 1) : 0.0f;
    d.K = m->ckpt_every;
    return d;
}

sq_status check_index(const sq_index* idx, bool for_render) {
    if (!idx) return fail(SQ_ERR_INVALID, "index is NULL");
    if (!idx->counts || !idx->offsets) return fail(SQ_ERR_INVALID, "index counts/offsets is NULL");
    if (idx->capacity < 0) return fail(SQ_ERR_INVALID, "index capacity < 0");
    if (idx->capacity > 0 && !idx->ids) return fail(SQ_ERR_INVALID, "index ids is NULL");
    if (!for_render && !idx->total) return fail(SQ_ERR_INVALID, "index total is NULL");
    return SQ_OK;
}

sq_status tuning_of(const sq_tuning* t, sqr::TuneDev& d) {
    sq_tuning v = t ? *t : sq_default_tuning();
    if (!(v.tile_w == 4 || v.tile_w == 8 || v.tile_w == 16))
        return fail(SQ_ERR_INVALID, "tile_w = %d not in {4, 8, 16}", v.tile_w);
    if (v.waves_per_block < 1 || v.waves_per_block > 4)
        return fail(SQ_ERR_INVALID, "waves_per_block = %d not in [1, 4]", v.waves_per_block);
    if (v.bwd_mode < SQ_BWD_AUTO || v.bwd_mode > SQ_BWD_PRIMITIVE_MAJOR)
        return fail(SQ_ERR_INVALID, "bwd_mode = %d not in {0, 1, 2}", v.bwd_mode);
    d.tile_w = v.tile_w;
    d.waves_per_block = v.waves_per_block;
    d.bwd_mode = v.bwd_mode;
    return SQ_OK;
}

sqr::PrimsDev to_dev(const sq_prims* p) {
    sqr::PrimsDev d;
    d.n = p->n; d.C = p->n_classes;
    d.means = p->means; d.quats = p->quats; d.scales = p->scales; d.eps = p->eps;
    d.opacity = p->opacity; d.logits = p->logits;
    return d;
}

sqr::RaysDev to_dev(const sq_rays* r) {
    sqr::RaysDev d;
    d.n_cams = r->n_cams; d.H = r->height; d.W = r->width;
    d.origins = r->origins; d.dirs = r->dirs;
    return d;
}

sqr::IndexDev to_dev(const sq_index* i) {
    sqr::IndexDev d;
    d.counts = i->counts; d.offsets = i->offsets; d.ids = i->ids; d.capacity = i->capacity;
    return d;
}

}  // namespace

extern "C" {

const char* sq_last_error(void) { return g_err; }

int32_t sq_version(void) { return 100; }

sq_tuning sq_default_tuning(void) {
    sq_tuning t;
    t.tile_w = 8;
    t.waves_per_block = 4;
    t.bwd_mode = SQ_BWD_AUTO;
    return t;
}

int64_t sq_index_capacity_bound(const sq_grid* grid, int32_t n) {
    if (!grid_ok(grid) || n < 0) return -1;
    int64_t per = 1;
    for (int i = 0; i < 3; ++i) {
        const int64_t side = 2 * (int64_t)grid->nv + 1;
        per *= side < grid->dims[i] ? side : grid->dims[i];
    }
    return per * n;
}

size_t sq_build_index_workspace(const sq_grid* grid, int32_t n) {
    if (!grid_ok(grid) || n < 0) return 0;
    return sqr::index_workspace_bytes(nvox(grid), n);
}

sq_status sq_build_index(const sq_grid* grid, const sq_prims* prims, sq_index* idx, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
    if (!grid_ok(grid)) return fail(SQ_ERR_INVALID, "invalid grid (dims in [1,32767], voxel > 0, nv >= 0)");
    if (!prims || prims->n < 0) return fail(SQ_ERR_INVALID, "invalid prims");
    if (prims->n > 0 && !prims->means) return fail(SQ_ERR_INVALID, "prims->means is NULL");
    sq_status s = check_index(idx, false);
    if (s) return s;
    if (nvox(grid) >= ((int64_t)1 << 31)) return fail(SQ_ERR_INVALID, "grid has >= 2^31 voxels");
    const size_t need = sqr::index_workspace_bytes(nvox(grid), prims->n);
    if (!ws || ws_bytes < need) return fail(SQ_ERR_CAPACITY, "index workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % sqr::WS_ALIGN) return fail(SQ_ERR_INVALID, "workspace must be 256-byte aligned");
    const hipError_t e = sqr::launch_build_index(to_dev(grid), prims->means, prims->n, idx->counts, idx->offsets,
                                                 idx->ids, idx->capacity, idx->total, ws, stream);
    return hip_status(e, "sq_build_index");
}

size_t sq_render_workspace(const sq_grid* grid, const sq_prims* prims, const sq_rays* rays, const sq_march* march) {
    (void)grid; (void)rays; (void)march;
    if (!prims || prims->n < 0 || prims->n_classes < 1 || prims->n_classes > SQ_MAX_CLASSES) return 0;
    return sqr::render_workspace_bytes(prims->n, prims->n_classes);
}

static sq_status check_render_common(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                                     const sq_rays* rays, const sq_march* march, void* ws, size_t ws_bytes) {
    if (!grid_ok(grid)) return fail(SQ_ERR_INVALID, "invalid grid (dims in [1,32767], voxel > 0, nv >= 0)");
    sq_status s;
    if ((s = check_index(idx, true))) return s;
    if ((s = check_prims(prims, true))) return s;
    if ((s = check_rays(rays))) return s;
    if ((s = check_march(march))) return s;
    const size_t need = sqr::render_workspace_bytes(prims->n, prims->n_classes);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(SQ_ERR_CAPACITY, "render workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % sqr::WS_ALIGN) return fail(SQ_ERR_INVALID, "workspace must be 256-byte aligned");
    return SQ_OK;
}

sq_status sq_render_fwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, const sq_rays* rays,
                        const sq_march* march, float* depth, float* sem, float* probs, float* t_final, float* ckpt,
                        int64_t* stats, const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream) {
    sq_status s = check_render_common(grid, idx, prims, rays, march, ws, ws_bytes);
    if (s) return s;
    const int64_t nr = (int64_t)rays->n_cams * rays->height * rays->width;
    if (nr > 0 && (!depth || !sem || !t_final)) return fail(SQ_ERR_INVALID, "depth/sem/t_final is NULL");
    if (ckpt && march->ckpt_every < 1) return fail(SQ_ERR_INVALID, "ckpt given but ckpt_every < 1");
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    const hipError_t e = sqr::launch_render_fwd(to_dev(grid), to_dev(idx), to_dev(prims), to_dev(rays),
                                                to_dev(march), depth, sem, probs, t_final, ckpt, stats, tune, ws,
                                                stream);
    return hip_status(e, "sq_render_fwd");
}

sq_status sq_render_bwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, const sq_rays* rays,
                        const sq_march* march, const float* ckpt, const float* g_depth, const float* g_sem,
                        const sq_grads* grads, int64_t* stats, const sq_tuning* tuning, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
    sq_status s = check_render_common(grid, idx, prims, rays, march, ws, ws_bytes);
    if (s) return s;
    if (!(march->ckpt_every == 4 || march->ckpt_every == 8 || march->ckpt_every == 16))
        return fail(SQ_ERR_INVALID, "backward needs ckpt_every in {4, 8, 16} (got %d)", march->ckpt_every);
    const int64_t nr = (int64_t)rays->n_cams * rays->height * rays->width;
    if (nr > 0 && !ckpt) return fail(SQ_ERR_INVALID, "ckpt is NULL");
    if (!grads) return fail(SQ_ERR_INVALID, "grads is NULL");
    if (prims->n > 0 && (!grads->means || !grads->quats || !grads->scales || !grads->eps || !grads->opacity ||
                         !grads->logits))
        return fail(SQ_ERR_INVALID, "a gradient output array is NULL");
    sqr::TuneDev tune;
    if ((s = tuning_of(tuning, tune))) return s;
    if (tune.bwd_mode == SQ_BWD_PRIMITIVE_MAJOR &&
        !sqr::bwd_primitive_major_ok(to_dev(grid), prims->n, march->ckpt_every, tune.waves_per_block))
        return fail(SQ_ERR_UNSUPPORTED, "primitive-major backward does not apply (ckpt_every %d, n %d)",
                    march->ckpt_every, prims->n);
    const hipError_t e = sqr::launch_render_bwd(to_dev(grid), to_dev(idx), to_dev(prims), to_dev(rays),
                                                to_dev(march), ckpt, g_depth, g_sem, grads->means, grads->quats,
                                                grads->scales, grads->eps, grads->opacity, grads->logits, stats, tune, ws,
                                                stream);
    return hip_status(e, "sq_render_bwd");
}

}  // extern "C"

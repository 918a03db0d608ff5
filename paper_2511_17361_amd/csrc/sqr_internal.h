// Host-side interface between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sqr_device.h"

namespace sqr {

constexpr size_t WS_ALIGN = 256;
inline size_t align_up(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// ---------------- index ----------------
size_t index_workspace_bytes(int64_t nvox, int n);
hipError_t launch_build_index(const GridDev& g, const float* means, int n, int32_t* counts, int32_t* offsets,
                              int32_t* ids, int64_t capacity, int64_t* total, void* ws, hipStream_t st);

// ---------------- render ----------------
struct PrimsDev {
    int n, C;
    const float *means, *quats, *scales, *eps, *opacity, *logits;
};
struct RaysDev {
    int n_cams, H, W;
    const float *origins, *dirs;
};
struct MarchDev {
    int L;
    float t_near, delta;
    int K;      // checkpoint spacing (0 = none)
};
struct IndexDev {
    const int32_t *counts, *offsets, *ids;
    int64_t capacity;
};
struct TuneDev {
    int tile_w;           // 4, 8 or 16 (tile is tile_w x 64/tile_w pixels)
    int waves_per_block;  // 1..4
    int bwd_mode;         // 0 auto, 1 sample-major, 2 primitive-major
};

// class count padded to the compiled widths
int padded_classes(int C);

size_t render_workspace_bytes(int n, int C);
hipError_t launch_render_fwd(const GridDev& g, const IndexDev& idx, const PrimsDev& pr, const RaysDev& rays,
                             const MarchDev& mr, float* depth, float* sem, float* probs, float* t_final,
                             float* ckpt, int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st);
// whether the primitive-major backward applies to these arguments
bool bwd_primitive_major_ok(const GridDev& g, int n, int K, int wpb);
hipError_t launch_render_bwd(const GridDev& g, const IndexDev& idx, const PrimsDev& pr, const RaysDev& rays,
                             const MarchDev& mr, const float* ckpt, const float* g_depth, const float* g_sem,
                             float* g_means, float* g_quats, float* g_scales, float* g_eps, float* g_opacity,
                             float* g_logits, int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st);

}  // namespace sqr

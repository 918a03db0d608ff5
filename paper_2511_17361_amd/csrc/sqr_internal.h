// Interface between the C ABI layer and the kernel launchers.
//
// Every launcher works on a batch of scenes that share one voxel grid, one ray
// march and one class count; a single-scene call is a batch of one.  All
// per-scene arrays are concatenated scene-major.  The per-scene layout lives in
// a small table (BatchDesc) that the launchers write into the workspace with a
// kernel before the render kernels read it, so a launch sequence contains no
// host->device copies and can be captured into a hipGraph.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sqr_device.h"

namespace sqr {

constexpr size_t WS_ALIGN = 256;
inline size_t align_up(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

constexpr int MAX_SCENES = 32;
constexpr int QUEUE_STRIDE = 32;      // ints between the per-XCD work counters (128 B)
constexpr int N_XCD = 8;

// One scene of a batch (device-side view).
struct SceneDev {
    int n;            // primitives of the scene
    int prim_off;     // its first primitive in the concatenated arrays
    int cams, H, W;   // its rays
    int tiles_x, tiles_y;
    int tile_off;     // its first tile in the global tile order
    int64_t ids_base; // its first slot in the concatenated id lists
    int64_t cap;      // id slots reserved for it
    int64_t ray_off;  // its first ray in the concatenated ray arrays
};

struct BatchDesc {
    int n_scenes;
    int C;            // classes
    int total_prims, total_tiles, max_n;
    int tile_w, tile_h;
    int64_t total_rays;
    SceneDev s[MAX_SCENES];
};

struct MarchDev {
    int L;
    float t_near, delta;
    int K;      // checkpoint spacing (0 = none)
    float kappa;  // early ray termination: a ray stops once T < kappa (0 = none)
};

struct TuneDev {
    int tile_w;           // 4, 8 or 16 (tile is tile_w x 64/tile_w pixels)
    int waves_per_block;  // 1..4
    int bwd_mode;         // 0 auto, 1 sample-major, 2 primitive-major
    int persistent;       // 0 static tile grid, 1 persistent waves with per-XCD work queues
};

// Device pointers of one batch call (concatenated scene-major).
struct BatchIO {
    const float *means, *quats, *scales, *eps, *opacity, *logits;
    const float *origins, *dirs;
    int32_t *counts, *offsets, *ids;
    int64_t* totals;
    float *depth, *sem, *probs, *t_final, *ckpt;
    const float *g_depth, *g_sem;
    float *g_means, *g_quats, *g_scales, *g_eps, *g_opacity, *g_logits;
    float *vox_density, *vox_sem;
    int32_t* vox_labels;
    const int32_t* sem_label;
    const float* depth_label;
    float* loss;
    int32_t* tile_stop;       // nullable: [4 + total_tiles], header then one stop per tile
    float* stash;             // nullable: per-sample forward values for the backward (StashGeom)
    int64_t stash_len;        // floats of stash
};

// Layout of the per-sample stash of a forward with checkpoints (floats from
// the start of the buffer): a header of STASH_HEAD int32 ([0] tile width,
// [1] L, [2] K, [3] 1 once a forward with checkpoints wrote it, [4] slots that
// forward asked for, [5] slots the buffer holds), the slot of every (global
// tile, chunk) as int32 (-1: none), then the pool of slots.  A slot holds, for
// the K samples of one tile's chunk and each of its 64 lanes, the density sum
// a and the class sums s[0..CP) of the sample: [K][64][4 NM] floats (the
// matrix-core class accumulators as they are in registers), then
// [K][64][2] floats (s[CP-1] when CP = 4 NM + 1, else 0; then a).
constexpr int STASH_HEAD = 16;
struct StashGeom {
    int64_t tab_off;      // int32 offset of the slot table
    int64_t pool_off;     // float offset of the pool (256-byte aligned)
    int64_t slot_floats;  // floats per slot
    int nck;              // chunks per tile
    int m_floats;         // 4 NM: class sums held in four-wide accumulators
};
StashGeom stash_geom(const BatchDesc& d, int L, int K);

// Weights of the fused loss (Eq. eq:loss); nullptr = no loss epilogue.
struct LossArgs {
    float lambda_sem, lambda_depth;
};

// class count padded to the compiled widths
int padded_classes(int C);

// Fills the tile counts and offsets of a host-side batch description.
void finish_desc(BatchDesc& d, int tile_w);

size_t batch_workspace_bytes(const GridDev& g, const BatchDesc& d);
// the front part of the same layout that the index build alone uses
size_t index_workspace_bytes(const GridDev& g, const BatchDesc& d);

hipError_t launch_batch_index(const GridDev& g, const BatchDesc& d, const BatchIO& io, void* ws, hipStream_t st);
hipError_t launch_batch_fwd(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                            int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st,
                            const LossArgs* loss = nullptr);
hipError_t launch_batch_bwd(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                            int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st);

hipError_t launch_batch_voxelise(const GridDev& g, const BatchDesc& d, const BatchIO& io, float tau, void* ws,
                                 hipStream_t st);

// Superquadric-major backward (interaction sort by primitive); `iws` is the
// caller's interaction workspace of sq_major_workspace_bytes(d, mr, capacity).
size_t sq_major_workspace_bytes(const GridDev& g, const BatchDesc& d, const MarchDev& mr, int64_t capacity);
hipError_t launch_batch_bwd_sq_major(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                                     int64_t capacity, int64_t* total, void* iws, const TuneDev& tune, void* ws,
                                     hipStream_t st);

// whether the primitive-major backward applies to these arguments
bool bwd_primitive_major_ok(const GridDev& g, int max_n, int K, int wpb);

// Records the thread's sq_last_error() message and returns `code`.
int32_t set_error(int32_t code, const char* fmt, ...);

}  // namespace sqr

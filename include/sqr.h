/*
 * sqr.h — C ABI of the MI355X (gfx950) superquadric volume renderer.
 *
 * The renderer is SQOcc-R of arXiv 2511.17361 ("SuperQuadricOcc"):
 * a voxel-indexed volume renderer that turns N superquadric primitives
 * S_i = {m, s, r, eps, sigma, c} (Sec. 3.1 "SuperQuadrics") into per-pixel
 * expected depth and semantic renders (Sec. 3.3 "Forward Pass",
 * Eq. eq:alpha_sem_sq, eq:alpha_composite, eq:depth_sem), and back-propagates
 * gradients of both renders to every primitive parameter (Sec. 3.3
 * "Backward Pass").
 *
 * Conventions for every entry point below
 *  - All array pointers are DEVICE pointers, owned by the caller, C-contiguous,
 *    float32 or int32/int64 as stated.  The library never keeps a pointer
 *    after a call returns and never allocates device memory inside a call:
 *    scratch space comes from the caller's `ws` buffer, sized by the matching
 *    *_workspace() query.
 *  - Every call is asynchronous on `stream` and performs no host<->device
 *    synchronisation, so a sequence of calls can be captured into a hipGraph.
 *  - Arguments are validated on the host before anything is launched; a
 *    rejected call launches nothing and returns a negative sq_status.
 *    sq_last_error() then returns a thread-local, human-readable message.
 *  - Behaviour on NaN/Inf inputs is unspecified (they propagate); scales and
 *    eps must be > 0.
 */
#ifndef SQR_H
#define SQR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sq_status;
#define SQ_OK              0
#define SQ_ERR_INVALID    -1  /* bad argument (detected on the host, nothing launched) */
#define SQ_ERR_CAPACITY   -2  /* workspace or index capacity too small (host-detectable) */
#define SQ_ERR_HIP        -3  /* a HIP runtime call failed; see sq_last_error() */
#define SQ_ERR_UNSUPPORTED -4 /* valid request that this library does not implement */

#define SQ_MAX_CLASSES 32     /* largest supported number of semantic classes C */
#define SQ_MAX_SCENE_PRIMS ((1 << 25) - 1) /* most primitives in one scene: the kernels
                                           * address a primitive's record and logits by
                                           * 32-bit byte offsets from the scene's base, and
                                           * a scene's logit rows (at most 128 bytes each)
                                           * by a 32-bit buffer range; more returns
                                           * SQ_ERR_UNSUPPORTED */

/* Voxel grid (Sec. 3.3 "Preliminary Construction"; bounds and resolution of
 * Sec. 4.1).  Voxel (ix,iy,iz) covers [lo + i*voxel, lo + (i+1)*voxel) per axis
 * (half-open; the upper face is outside).  The linear voxel id used by the
 * index ("hashing" of the paper) is v = (ix*dims[1] + iy)*dims[2] + iz.
 * nv is the neighbourhood half-width N_v: primitive k is listed in every voxel
 * v with max_axis |v - c_k| <= nv, where c_k is the voxel containing m_k.
 *
 * theta is the index's influence threshold (the occupancy-aware indexing of
 * the Supplement's "Limitations and Future Work"), in [0, 1).  0 gives the
 * paper's index above.  With theta > 0 primitive k is listed only in the
 * voxels of its N_v cube that meet the world-space box of
 * max(|u|,|v|,|w|) <= ln(sigma_k/theta)^(eps1_k/2), evaluated in FP64: that
 * box holds every point where p_o * sigma_k >= theta, since
 * f >= max(|u|,|v|,|w|)^(2/eps1).  A primitive with sigma_k <= theta is listed
 * nowhere.  The render then drops exactly the (sample, primitive) pairs whose
 * voxel lies outside that box, each with p_o * sigma_k < theta.  Every call
 * that takes the grid (index, renders, voxelisation) uses the same lists. */
typedef struct {
    float   lo[3];
    float   voxel;
    int32_t dims[3];
    int32_t nv;
    float   theta;
} sq_grid;

/* Superquadric -> voxel CSR lists: the paper's V_n (counts), V_f (offsets,
 * exclusive prefix sum of counts) and V_sq (ids).  counts/offsets hold
 * dims[0]*dims[1]*dims[2] int32 each; ids holds `capacity` int32.  Within each
 * voxel the ids are strictly ascending.  *total (one device int64) receives
 * E = sum(counts).  If E > capacity, ids holds only the entries below
 * `capacity` and the index must not be used (check *total after a sync). */
typedef struct {
    int32_t* counts;
    int32_t* offsets;
    int32_t* ids;
    int64_t  capacity;
    int64_t* total;
} sq_index;

/* N primitives (Sec. 3.1): means [n,3] (m), quats [n,4] (r, stored w,x,y,z,
 * need not be unit: the renderer uses r/|r|, Hamilton convention, and maps a
 * point to the local frame as x_S = R(r/|r|) (x - m)), scales [n,3]
 * (s_x,s_y,s_z > 0), eps [n,2] (eps1, eps2 > 0), opacity [n] (sigma),
 * logits [n,C] (c).  1 <= n_classes <= SQ_MAX_CLASSES, n <= SQ_MAX_SCENE_PRIMS. */
typedef struct {
    int32_t      n;
    int32_t      n_classes;
    const float* means;
    const float* quats;
    const float* scales;
    const float* eps;
    const float* opacity;
    const float* logits;
} sq_prims;

/* Rays r(t) = o + t d, one per pixel: origins/dirs [n_cams,H,W,3], |d| = 1.
 * The flat ray id is (cam*H + y)*W + x. */
typedef struct {
    int32_t      n_cams;
    int32_t      height;
    int32_t      width;
    const float* origins;
    const float* dirs;
} sq_rays;

/* L uniformly spaced samples in [t_near, t_far], endpoints included
 * (Sec. 3.3 "Preliminary Construction"): t_j = t_near + j*delta with
 * delta = (t_far - t_near)/(L-1) (t_0 = t_near if L == 1).  Sample depths,
 * sample points and their voxels are computed in float32 with every op
 * correctly rounded and no fused multiply-add:
 *   t_j = fl(t_near + fl(j*delta)), x_j = fl(o + fl(t_j*d)),
 *   i = floor(fl(fl(x_j - lo) * fl(1/voxel))).
 * ckpt_every (K) is the transmittance-checkpoint spacing used by the
 * differentiable forward and the backward; 0 = no checkpoints.
 * kappa is the early ray termination threshold (Supplement "Ray
 * Termination"): sample j is composited only while its transmittance
 * T_j >= kappa, so a ray stops once T falls below kappa; the backward
 * differentiates the truncated render (the stopping point itself carries no
 * gradient).  0 = no termination (the paper's default); requires
 * 0 <= kappa <= 1.  Requires L >= 1 and 0 <= t_near < t_far (t_near <= t_far
 * if L == 1). */
typedef struct {
    int32_t n_samples;
    float   t_near;
    float   t_far;
    int32_t ckpt_every;
    float   kappa;
} sq_march;

/* Gradient outputs (overwritten, not accumulated), shaped like sq_prims. */
typedef struct {
    float* means;    /* [n,3] */
    float* quats;    /* [n,4] */
    float* scales;   /* [n,3] */
    float* eps;      /* [n,2] */
    float* opacity;  /* [n]   */
    float* logits;   /* [n,C] */
} sq_grads;

/* Kernel launch choices.
 *  tile_w           ray-tile width in pixels: 4, 8 or 16 (a tile is 64 pixels,
 *                   one wavefront).
 *  waves_per_block  1..4.
 *  bwd_mode         SQ_BWD_AUTO picks the primitive-major backward where it
 *                   applies (checkpoint spacing 4 or 8, grid within
 *                   1023 x 1023 x 511, per-wave id bitmap within 64 KiB of LDS
 *                   per block) and the sample-major one otherwise; the other
 *                   values force one of them (forcing primitive-major where it
 *                   does not apply returns SQ_ERR_UNSUPPORTED).
 *  persistent       0: one wavefront per ray tile; 1 (default): persistent
 *                   wavefronts that take tiles from eight per-XCD work queues
 *                   (each XCD drains a contiguous range of tiles, then steals).
 *  chunk            batched calls: checkpoint spacing K (4, 8 or 16) used by
 *                   the forward's checkpoints and the backward; 0 = the
 *                   batch's march.ckpt_every.  Single-scene calls always use
 *                   march->ckpt_every.
 * Passing NULL uses sq_default_tuning(). */
#define SQ_BWD_AUTO 0
#define SQ_BWD_SAMPLE_MAJOR 1
#define SQ_BWD_PRIMITIVE_MAJOR 2
typedef struct {
    int32_t tile_w;
    int32_t waves_per_block;
    int32_t bwd_mode;
    int32_t persistent;
    int32_t chunk;
} sq_tuning;

/* Thread-local description of the last failure on this thread ("" if none). */
const char* sq_last_error(void);

/* ABI version (major*100 + minor). */
int32_t sq_version(void);

/* Defaults for sq_tuning. */
sq_tuning sq_default_tuning(void);

/* Upper bound of E for n primitives on this grid:
 * n * prod_axis min(2*nv + 1, dims[axis]).  Host-only, no launch. */
int64_t sq_index_capacity_bound(const sq_grid* grid, int32_t n);

/* Bytes of workspace sq_build_index needs (host-only). */
size_t sq_build_index_workspace(const sq_grid* grid, int32_t n);

/* Build the superquadric -> voxel lists (Sec. 3.3 "Preliminary Construction":
 * per-primitive cubic neighbourhood V_c hashed into V_sq, V_f, V_n).
 * Deterministic: the output is a pure function of (grid, means).
 * Reads prims->means only.  Writes idx->counts, offsets, ids (< capacity)
 * and *idx->total. */
sq_status sq_build_index(const sq_grid* grid, const sq_prims* prims, sq_index* idx,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace sq_render_fwd / sq_render_bwd need (host-only). */
size_t sq_render_workspace(const sq_grid* grid, const sq_prims* prims,
                           const sq_rays* rays, const sq_march* march);

/* Forward render (Sec. 3.3 "Forward Pass").  Per ray, samples front to back;
 * a sample outside the grid or in a voxel with V_n = 0 is skipped; otherwise
 *   a_j = sum_{k in Q(v_j)} p_o(x_j, S_k) sigma_k,  alpha_j = min(1, a_j),
 *   s_j = sum_k p_o(x_j, S_k) c_k                     (Eq. eq:alpha_sem_sq)
 *   w_j = T_j alpha_j, T_{j+1} = T_j (1 - alpha_j)     (Eq. eq:alpha_composite)
 *   depth = sum_j w_j t_j, sem = sum_j w_j s_j         (Eq. eq:depth_sem)
 * with p_o(x, S) = exp(-f(x_S)) (Eq. eq:sq_occupancy_prob) and
 * f = (|u|^(2/e2) + |v|^(2/e2))^(e2/e1) + |w|^(2/e1), (u,v,w) = x_S / s.
 * Outputs: depth [n_cams,H,W], sem [n_cams,C,H,W], probs (nullable;
 * softmax over classes of sem) [n_cams,C,H,W], t_final (T_L) [n_cams,H,W],
 * ckpt (nullable; needs march->ckpt_every > 0) [ceil(L/K), n_cams*H*W]:
 * ckpt[c][ray] = T at sample c*K.  `stats` (nullable, 4 device int64,
 * accumulated) counts non-empty in-grid samples, listed (sample, primitive)
 * pairs, pairs not culled, and rays; when non-NULL a counting variant of the
 * kernel runs.  A pair is culled only where float32 exp(-f) is exactly 0
 * (f >= 110, detected from max(|u|,|v|,|w|) before any transcendental). */
sq_status sq_render_fwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                        const sq_rays* rays, const sq_march* march,
                        float* depth, float* sem, float* probs, float* t_final, float* ckpt,
                        int64_t* stats, const sq_tuning* tuning,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of sq_render_fwd (Sec. 3.3 "Backward Pass") for upstream gradients
 * g_depth [n_cams,H,W] and g_sem [n_cams,C,H,W] (either may be NULL = zero).
 * Needs the checkpoints `ckpt` written by sq_render_fwd with the same
 * arguments and march->ckpt_every in {4, 8, 16}.  The ray march is replayed
 * back to front chunk by chunk from the checkpoints; nothing per sample is
 * stored.  Writes (overwrites) every array of `grads`.  Gradients are summed
 * with float atomics, so the last bits depend on scheduling order.
 * `stats` (nullable, 6 device int64, accumulated) selects a counting variant
 * that also reports, for the front-to-back recompute pass and for the adjoint
 * pass: samples visited, listed pairs, pairs not culled. */
sq_status sq_render_bwd(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                        const sq_rays* rays, const sq_march* march,
                        const float* ckpt, const float* g_depth, const float* g_sem,
                        const sq_grads* grads, int64_t* stats, const sq_tuning* tuning,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of the interaction workspace sq_render_bwd_sq_major needs for
 * `capacity` interactions (host-only; 0 on bad input). */
size_t sq_sq_major_workspace(const sq_grid* grid, const sq_prims* prims, const sq_rays* rays,
                             const sq_march* march, int64_t capacity);

/* sq_render_bwd computed superquadric-major, as the paper's Processes 1-3
 * (Sec. 3.3 "Backward Pass"): (1) per ray, replay the checkpointed chunks and
 * store dL/da_j and w_j per sample; (2) build the set of (primitive, sample)
 * interactions from the index and group it by primitive id (count, scan,
 * scatter: a counting sort); (3) reduce each primitive's group in one block,
 * without global atomics.  Same results as sq_render_bwd (to rounding).  An
 * A/B alternative to the default backward: it needs the caller's interaction
 * workspace (iws, sq_sq_major_workspace bytes) holding up to `capacity`
 * interactions; *interactions (one device int64) receives their number E; if
 * E > capacity the gradients are incomplete and the call must be repeated
 * with more (check after a sync, as for sq_build_index).  Requires
 * rays x samples < 2^32. */
sq_status sq_render_bwd_sq_major(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                                 const sq_rays* rays, const sq_march* march, const float* ckpt,
                                 const float* g_depth, const float* g_sem, const sq_grads* grads,
                                 int64_t capacity, int64_t* interactions, void* iws, size_t iws_bytes,
                                 const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* Weights of the training loss of Eq. eq:loss (Supplement "Loss
 * Formulation"): L = lambda_sem * L_sem + lambda_depth * L_depth; the paper
 * uses lambda_sem = 2, lambda_depth = 0.05. */
typedef struct {
    float lambda_sem;
    float lambda_depth;
} sq_loss_weights;

/* sq_render_fwd with the loss of Eq. eq:loss fused into the forward's
 * epilogue.  Per pixel, against the pseudo-labels sem_label [n_cams,H,W]
 * (int32 class; outside [0, C) = no label) and depth_label [n_cams,H,W]
 * (metres; a label counts where it is finite and > 0):
 *   L_sem   = mean over labelled pixels of -log softmax(sem)[label]
 *   L_depth = mean over labelled pixels of (depth - depth_label)^2
 * It writes (besides every output of sq_render_fwd) the upstream gradients
 *   g_sem   [n_cams,C,H,W] = lambda_sem / N_sem * (softmax(sem) - onehot(label))
 *   g_depth [n_cams,H,W]   = lambda_depth / N_depth * 2 (depth - depth_label)
 * (zero on unlabelled pixels) that sq_render_bwd consumes, and
 * loss[0..2] = (L, L_sem, L_depth), reduced in a fixed order (deterministic;
 * a term with no labelled pixel is 0).  Labelled pixels are counted by the
 * same call before the render. */
sq_status sq_render_fwd_loss(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                             const sq_rays* rays, const sq_march* march, const sq_loss_weights* weights,
                             const int32_t* sem_label, const float* depth_label,
                             float* depth, float* sem, float* probs, float* t_final, float* ckpt,
                             float* g_depth, float* g_sem, float* loss, const sq_tuning* tuning,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace sq_voxelise needs (host-only). */
size_t sq_voxelise_workspace(const sq_grid* grid, const sq_prims* prims);

/* Superquadric voxelisation (Supplement "SuperQuadric Voxelisation",
 * Eq. eq:voxelisation).  For every voxel v of the grid, with centre
 *   p = fl(lo + fl(fl(i + 0.5) * voxel)) per axis (float32, no FMA),
 * over the primitives listed in v (the same N_v lists as the render):
 *   density[v]  = sum_k p_o(p, S_k) sigma_k
 *   sem[c][v]   = sum_k p_o(p, S_k) c_k[c]
 *   labels[v]   = n_classes ("free") where density[v] < tau, otherwise the
 *                 smallest c with the largest sem[c][v] (compared in float32).
 * The paper uses tau = 0.05.  Outputs: density [V] (required), sem [C, V]
 * (nullable, class planes), labels [V] int32 (nullable), V = voxels in the
 * linear order of sq_grid.  Same cull as sq_render_fwd.  Deterministic: four
 * partial sums per voxel, each over a fixed part of the voxel's list in
 * ascending id, added in a fixed order. */
sq_status sq_voxelise(const sq_grid* grid, const sq_index* idx, const sq_prims* prims, float tau,
                      float* density, float* sem, int32_t* labels,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: several scenes that share one grid, one ray march and one
 * class count, with uneven primitive and camera counts, rendered by single
 * launches whose wavefronts cover the tiles of every scene.
 * ------------------------------------------------------------------------ */
#define SQ_MAX_SCENES 32

typedef struct {
    int32_t n_prims;         /* primitives of the scene */
    int32_t n_cams, height, width;
    int64_t index_capacity;  /* id slots reserved for this scene's lists */
} sq_scene;

typedef struct {
    int32_t  n_scenes;       /* 1 .. SQ_MAX_SCENES */
    int32_t  n_classes;
    sq_grid  grid;           /* shared by all scenes */
    sq_march march;          /* shared; ckpt_every = default chunk */
    sq_scene scenes[SQ_MAX_SCENES];
} sq_batch;

/* Device arrays of a batch, each concatenated scene-major in scene order:
 *  means..logits [sum n_prims, .]; origins, dirs [sum rays, 3] (each scene
 *  [n_cams, H, W, 3]); counts, offsets [n_scenes * V] (V = voxels; offsets are
 *  relative to the scene's own id region); ids [sum index_capacity];
 *  totals [n_scenes] (E per scene); depth, t_final [sum rays]; sem, probs
 *  [sum rays * C] (each scene [n_cams, C, H, W]; probs nullable); ckpt
 *  [ceil(L/K) * sum rays] (each scene [ceil(L/K), its rays]); g_depth, g_sem
 *  shaped like depth and sem (nullable = zero); g_* shaped like the
 *  parameters; vox_density, vox_labels [n_scenes * V] and vox_sem
 *  [n_scenes * C * V] (each scene as in sq_voxelise); sem_label,
 *  depth_label shaped like depth (pseudo-labels of the fused loss) and loss
 *  (3 floats).  The fused-loss calls WRITE the buffers g_depth and g_sem
 *  point to.  A call reads and writes only the members it needs. */
typedef struct {
    const float *means, *quats, *scales, *eps, *opacity, *logits;
    const float *origins, *dirs;
    int32_t *counts, *offsets, *ids;
    int64_t *totals;
    float *depth, *sem, *probs, *t_final, *ckpt;
    const float *g_depth, *g_sem;
    float *g_means, *g_quats, *g_scales, *g_eps, *g_opacity, *g_logits;
    float *vox_density, *vox_sem;
    int32_t *vox_labels;
    const int32_t *sem_label;
    const float *depth_label;
    float *loss;
    /* Where each ray tile of the last forward stopped (nullable; an
     * MI355X-side design choice, not in the paper).  A forward with
     * checkpoints writes, for every tile t of its tiling, tile_stop[4 + t] =
     * the last sample it composited before every ray of the tile was opaque
     * or out of the grid (L - 1 when the march ran to the end), behind a
     * header [tile width, L, K, 1]; a forward without checkpoints writes the
     * header with 0 in place of the 1.  The primitive-major backward, given
     * the buffer, skips the samples past each tile's stop (they add nothing);
     * when the header does not match its own tiling and march it ignores the
     * buffer.  Like the checkpoints, the buffer belongs to the last forward:
     * pass it to both calls or to neither.  tile_stop holds tile_stop_len
     * int32, at least sq_batch_tile_stop_len(); shorter: SQ_ERR_CAPACITY.
     * A backward whose chunk K or sample count L differs from the ones the
     * header records for a forward with checkpoints (the checkpoint rows are
     * laid out by that forward's K) cannot detect the mismatch on the host;
     * it writes NaN to every gradient output instead of gradients read from
     * wrongly laid-out checkpoints. */
    int32_t *tile_stop;
    int64_t  tile_stop_len;
    /* Floats that io->ckpt holds.  A call that reads or writes checkpoints
     * with chunk K needs ceil(L/K) * (sum of rays) of them; fewer:
     * SQ_ERR_CAPACITY, nothing launched. */
    int64_t  ckpt_len;
    /* Per-sample values of the last forward (nullable; an MI355X-side design
     * choice, not in the paper: it trades HBM for the backward's recompute).
     * A forward with checkpoints gives every chunk of K samples that a ray
     * tile enters one slot of the buffer's pool, in the order the tiles reach
     * their chunks, and leaves there, for each sample it composites, the
     * density sum a_j = sum_k p sigma_k and the class sums s_j = sum_k p c_k
     * of Eq. eq:alpha_sem_sq.  The primitive-major backward then takes a_j
     * and G_j = <g_S, s_j> from the slot instead of evaluating the chunk's
     * pairs a first time; a chunk without a slot (pool exhausted) is
     * recomputed as without the buffer.  Layout (int32 words at the start):
     * [0] tile width, [1] L, [2] K, [3] 1 when a forward with checkpoints
     * wrote it (a forward without checkpoints writes 0), [4] the slots that
     * forward asked for (one per chunk entered, also beyond the pool: the
     * figure to size the pool by), [5] the slots the pool holds; then the
     * slot table and the pool (sizes from sq_batch_stash_len).  The backward
     * uses it only when the header matches its own tiling, L and K; like the
     * checkpoints it belongs to the last forward: pass it to both calls or to
     * neither.  The counting variants (stats) ignore it. */
    float*   stash;
    /* Floats that io->stash holds: at least sq_batch_stash_len(batch,
     * tuning, 0) for a call with checkpoints (16 for one without); fewer:
     * SQ_ERR_CAPACITY, nothing launched.  Floats beyond that give
     * (stash_len - sq_batch_stash_len(.., 0)) / slot size slots. */
    int64_t  stash_len;
} sq_batch_io;

/* Bytes of workspace every batched call needs (host-only; 0 on bad input). */
size_t sq_batch_workspace(const sq_batch* batch);

/* Length (int32) of io->tile_stop for calls with this tuning (its tile width;
 * NULL = defaults).  Host-only; 0 on bad input. */
int64_t sq_batch_tile_stop_len(const sq_batch* batch, const sq_tuning* tuning);

/* Floats of io->stash for calls with this tuning (its tile width and chunk;
 * NULL = defaults) whose pool holds `slots` slots of one (tile, chunk) each:
 * the header and slot table, 256-byte aligned, then slots x K x 64 x (Q + 2)
 * floats, Q = the class count padded to 4, 8, 16 or 32 (16 at 17 classes).
 * Host-only; 0 on bad input (a chunk outside {4, 8, 16}, slots < 0 or above
 * INT32_MAX). */
int64_t sq_batch_stash_len(const sq_batch* batch, const sq_tuning* tuning, int64_t slots);

/* sq_build_index for every scene of the batch (Sec. 3.3 "Preliminary
 * Construction").  Writes counts, offsets, ids (below each scene's capacity)
 * and totals. */
sq_status sq_batch_build_index(const sq_batch* batch, const sq_batch_io* io,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* sq_render_fwd for every scene of the batch in one launch (Sec. 3.3
 * "Forward Pass"); checkpoints are written when io->ckpt is not NULL, which
 * needs a chunk in {4, 8, 16} (the backward's) and io->ckpt_len floats for
 * it.  `stats` as for sq_render_fwd. */
sq_status sq_batch_render_fwd(const sq_batch* batch, const sq_batch_io* io, int64_t* stats,
                              const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* sq_render_bwd for every scene of the batch in one launch (Sec. 3.3
 * "Backward Pass"); needs the checkpoints of sq_batch_render_fwd with the
 * same chunk.  `stats` as for sq_render_bwd. */
sq_status sq_batch_render_bwd(const sq_batch* batch, const sq_batch_io* io, int64_t* stats,
                              const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* sq_render_fwd_loss for every scene of the batch: the means of Eq. eq:loss
 * run over the labelled pixels of all scenes together. */
sq_status sq_batch_render_fwd_loss(const sq_batch* batch, const sq_batch_io* io, const sq_loss_weights* weights,
                                   const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* sq_voxelise for every scene of the batch in one launch (Supplement
 * "SuperQuadric Voxelisation"); needs the index (counts, offsets, ids) and the
 * primitive parameters; writes vox_density and, when not NULL, vox_sem and
 * vox_labels. */
sq_status sq_batch_voxelise(const sq_batch* batch, const sq_batch_io* io, float tau,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* One training step of the renderer: index, forward with checkpoints,
 * backward (every output of io is written). */
sq_status sq_batch_step(const sq_batch* batch, const sq_batch_io* io, const sq_tuning* tuning,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* One training step with the fused loss: index, forward with checkpoints and
 * the loss epilogue (writing g_depth, g_sem and loss), backward. */
sq_status sq_batch_train_step(const sq_batch* batch, const sq_batch_io* io, const sq_loss_weights* weights,
                              const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* Captures sq_batch_step on `stream` (not the legacy default stream) into a
 * hipGraph and instantiates it.  The graph keeps every pointer of io and ws:
 * replays read the current contents of the same buffers.  The step contains
 * no memset nodes and no host copies.  Free with sq_graph_destroy. */
typedef struct sq_graph_impl* sq_graph;
sq_status sq_batch_step_graph_create(const sq_batch* batch, const sq_batch_io* io, const sq_tuning* tuning,
                                     void* ws, size_t ws_bytes, hipStream_t stream, sq_graph* out);
/* The same for sq_batch_train_step. */
sq_status sq_batch_train_graph_create(const sq_batch* batch, const sq_batch_io* io, const sq_loss_weights* weights,
                                      const sq_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream,
                                      sq_graph* out);
sq_status sq_graph_launch(sq_graph graph, hipStream_t stream);
sq_status sq_graph_destroy(sq_graph graph);

/* Times sq_batch_step for every candidate tuning (one warm-up, then `reps`
 * timed steps, HIP events on `stream`) and returns the fastest in
 * *best_index and each candidate's mean step time in ms_per_candidate
 * (nullable, n_candidates floats).  SYNCHRONOUS: waits for the stream.  All
 * candidates are validated before the first launch, io->ckpt_len included
 * (ceil(L/K) * sum rays floats for every candidate's chunk K). */
sq_status sq_batch_autotune(const sq_batch* batch, const sq_batch_io* io, const sq_tuning* candidates,
                            int32_t n_candidates, int32_t reps, int32_t* best_index, float* ms_per_candidate,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* The autotuner behind a persistent cache (a text file, one line per workload:
 * its key, " => ", then tile_w waves_per_block bwd_mode persistent chunk).
 * The batch and the candidates are validated first, as for sq_batch_autotune.
 * Then a line of cache_path whose key equals this batch's (sq_batch_tuning_key)
 * gives *best with no launch and *from_cache = 1; otherwise the candidates
 * are timed by sq_batch_autotune, the fastest is returned with *from_cache = 0
 * and appended to the file (a file that cannot be written leaves the result
 * valid and is reported by sq_last_error only).  A missing file is an empty
 * cache, a line that does not parse is skipped; cache_path NULL times every
 * call.  A cached tuning need not be among this call's candidates. */
sq_status sq_batch_autotune_cached(const sq_batch* batch, const sq_batch_io* io, const sq_tuning* candidates,
                                   int32_t n_candidates, int32_t reps, const char* cache_path, sq_tuning* best,
                                   int32_t* from_cache, void* ws, size_t ws_bytes, hipStream_t stream);

/* The cache key of a batch: library version, the current device's
 * architecture ("nodevice" without one), scene shapes, grid, march and class
 * count, as one line of text without spaces.  Writes at most n bytes
 * including the terminating zero; returns the key's length, or -1 for a
 * NULL batch. */
int32_t sq_batch_tuning_key(const sq_batch* batch, char* buf, int32_t n);

/* ------------------------------------------------------------------------
 * Allocation-free forward, for callers that cannot allocate device memory:
 * code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc.
 * ------------------------------------------------------------------------ */
/* Bytes of the library's fixed per-GPU scratch array (16 MiB).  Every GPU the
 * library runs on holds one such array until the process ends. */
#define SQ_NOALLOC_SCRATCH_BYTES (16u << 20)

/* sq_render_fwd with no workspace argument: its scratch space (the prepared
 * primitive records, the scene table, the work counters) is the library's
 * fixed device array of SQ_NOALLOC_SCRATCH_BYTES on the current device, and
 * the call allocates nothing (no hipMalloc, no allocating library routine).
 * The caller still owns every input and output, as for sq_render_fwd, and the
 * results are those of sq_render_fwd bit for bit.  A call whose scratch need
 * (sq_render_workspace) exceeds the array returns SQ_ERR_CAPACITY before
 * touching the device.  All calls on one GPU share its array, which keeps the
 * last call's contents (each call rewrites what it reads); calls that overlap
 * on one GPU (concurrent streams or threads) race and must be serialised by
 * the caller.  The first call on a device looks the array's address up once
 * (hipGetSymbolAddress) with that device current. */
sq_status sq_render_fwd_noalloc(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                                const sq_rays* rays, const sq_march* march,
                                float* depth, float* sem, float* probs, float* t_final, float* ckpt,
                                int64_t* stats, const sq_tuning* tuning, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SQR_H */

// Forward and backward ray march of the superquadric renderer (gfx950).
//
// Mapping: one wavefront = one tile of 64 rays (tile_w x 64/tile_w pixels of
// one camera of one scene).  Rays of a tile are nearly parallel, so at a given
// sample index most lanes sit in the same voxel.  When they all do, the wave
// walks that voxel's list; otherwise it walks the union of the lists of its
// lanes' voxels (built in a per-wave LDS bitmap, ascending id) and each lane
// takes the primitives whose neighbourhood box holds its voxel -- exactly its
// own list, in the same ascending order, so the result does not depend on how
// the lanes group.  The primitive id, its prepared record and its logits are
// wave-uniform and arrive through the scalar data cache; each lane evaluates
// p_o at its own sample point.  Nothing here is a dense contraction, so there
// is no MFMA use.
//
// Tiles of all scenes of a batch form one global tile order.  Waves take tiles
// either from a static grid (one wave per tile, XCD-grouped block order) or,
// persistently, from eight per-XCD work queues (each XCD drains a contiguous
// range of the tile order first, then steals from the others); either way
// every wave exits once the tile order is exhausted.
//
// Forward (Sec. 3.3 "Forward Pass", Eq. eq:alpha_sem_sq, eq:alpha_composite,
// eq:depth_sem).  Backward (Sec. 3.3 "Backward Pass"): per ray, chunks of K
// samples are replayed back to front from the transmittance checkpoints the
// forward wrote; Q_j = alpha_j G_j + (1 - alpha_j) Q_{j+1} gives
// dL/dalpha_j = T_j (G_j - Q_{j+1}) without dividing by (1 - alpha) and
// without per-sample state outside the chunk.
#include "sqr_device.h"
#include "sqr_internal.h"
#include "sqr_launch.h"

#include <algorithm>
#include <type_traits>

namespace sqr {

// accumulator row layout (floats per primitive = AccRow<CP>::P)
constexpr int A_SIG = 0, A_E1 = 1, A_E2 = 2, A_XS = 3, A_R = 6, A_LG = 15;
template <int CP> struct AccRow { static constexpr int V = A_LG + CP; static constexpr int P = V <= 32 ? 32 : 64; };
template <int VP> struct Log2 { static constexpr int v = VP == 64 ? 6 : VP == 32 ? 5 : VP == 16 ? 4 : 0; };

int padded_classes(int C) {
    if (C <= 4) return 4;
    if (C <= 8) return 8;
    if (C <= 17) return 17;
    return 32;
}
int acc_row(int CP) { return A_LG + CP <= 32 ? 32 : 64; }

StashGeom stash_geom(const BatchDesc& d, int L, int K) {
    StashGeom g;
    const int CP = padded_classes(d.C);
    g.m_floats = CP >= 16 ? CP / 16 * 16 : CP >= 8 ? 8 : 4;
    g.nck = K > 0 ? (L + K - 1) / K : 0;
    g.tab_off = STASH_HEAD;
    g.pool_off = (STASH_HEAD + (int64_t)d.total_tiles * g.nck + 63) / 64 * 64;
    g.slot_floats = (int64_t)K * 64 * (g.m_floats + 2);
    return g;
}

// Occupancy targets (waves per SIMD) that the register allocator must meet.
// The persistent forward with checkpoints runs at 6, where it spills a few
// per-tile pointers (stored at the tile's start, reloaded for its epilogue),
// which costs less than the wave it buys; the one that writes the stash runs
// at 5, where their scratch reloads no longer wait on the stash stores ahead
// of them (one vector-memory counter, in order).
#define FWD_WPE(CP, CKPT, STATS, PERSIST, STASH) \
    ((CP) <= 8 ? 6 : (CP) > 17 ? 3 : (STATS) ? 4 : !(CKPT) ? 6 : (PERSIST) ? ((STASH) ? 5 : 6) : 4)
#define BWD_WPE(CP, KC) ((CP) <= 17 ? 4 : 3)

// Kernel parameters shared by every render kernel.
struct Ctx {
    GridDev g;
    MarchDev mr;
    int C;
    int total_tiles;
    const BatchDesc* desc;      // device copy (workspace)
    int* queue;                 // per-XCD work counters of this launch
    const int32_t *counts, *offsets, *ids;
    const float *rec, *lgp;
    const float *origins, *dirs;
    float *depth, *sem, *probs, *t_final, *ckpt;
    const float *g_depth, *g_sem;
    float* acc;
    int64_t* stats;
    int bitmap_words;           // per-wave union bitmap size (0: none)
    float tau;                  // voxelisation: free-space density threshold
    float *vox_density, *vox_sem;
    int32_t* vox_labels;
    // fused loss (Eq. eq:loss)
    const int32_t* sem_label;
    const float* depth_label;
    float *gd_out, *gs_out;     // dL/dD_hat, dL/dS_hat written by the forward
    float lam_s, lam_d;
    const int* lcount;          // labelled pixels: semantic, depth
    float* lpart;               // per-tile partial sums (cross-entropy, squared error)
    // nullable: [0] tile width, [1] L, [2] K, [3] 1 once a forward with
    // checkpoints wrote it, then per global tile the last sample its forward
    // composited
    int* tile_stop;
    // nullable: the per-sample stash (StashGeom): header, slot table, pool
    int* stash_hdr;
    int* stash_tab;
    float* stash_pool;
    int stash_slots;            // slots the pool holds
    int stash_slot_floats;
};
constexpr int STOP_HEAD = 4;

// ---------------------------------------------------------------------------
// Per-primitive preparation (all primitives of the batch)
// ---------------------------------------------------------------------------
template <int CP>
__global__ __launch_bounds__(256) void k_prep_records(int n_total, int C, const float* __restrict__ means,
                                                      const float* __restrict__ quats,
                                                      const float* __restrict__ scales,
                                                      const float* __restrict__ eps,
                                                      const float* __restrict__ opacity,
                                                      const float* __restrict__ logits, GridDev g,
                                                      float* __restrict__ rec, float* __restrict__ lgp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_total) return;
    float qw = quats[4 * k + 0], qx = quats[4 * k + 1], qy = quats[4 * k + 2], qz = quats[4 * k + 3];
    const float qinv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qinv; qx *= qinv; qy *= qinv; qz *= qinv;
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    const float is[3] = {1.0f / scales[3 * k], 1.0f / scales[3 * k + 1], 1.0f / scales[3 * k + 2]};
    const float e1 = eps[2 * k], e2 = eps[2 * k + 1];
    float* r = rec + (size_t)k * REC;
    r[0] = means[3 * k]; r[1] = means[3 * k + 1]; r[2] = means[3 * k + 2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[3 + 3 * i + j] = R[3 * i + j] * is[i];
    r[12] = 2.0f / e2;
    r[13] = 2.0f / e1;
    r[14] = e2 / e1;
    r[15] = opacity[k];
    // f >= max(|u|,|v|,|w|)^(2/eps1): culled where that bound reaches F_CULL
    r[16] = exp2f(0.5f * e1 * log2f(F_CULL));
    int box[3];
    prim_box(g, means + 3 * k, quats + 4 * k, scales + 3 * k, eps + 2 * k, opacity + k, box);
    uint32_t glo, ghi;
    box_words(box, glo, ghi);
    r[R_GLO] = __uint_as_float(glo); r[R_GHI] = __uint_as_float(ghi);
    r[R_AM1] = r[12] == 1.0f ? FLT_MIN : r[12] - 1.0f;
    r[R_BM1] = r[13] == 1.0f ? FLT_MIN : r[13] - 1.0f;
    r[R_EM1] = r[14] - 1.0f;
    r[22] = __int_as_float(box[0]); r[23] = __int_as_float(box[1]); r[24] = __int_as_float(box[2]);
    r[R_INVS] = is[0]; r[R_INVS + 1] = is[1]; r[R_INVS + 2] = is[2];
    for (int c = 0; c < CP; ++c) lgp[(size_t)k * CP + c] = c < C ? logits[(size_t)k * C + c] : 0.0f;
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Header of the per-tile stops before a forward: its tiling and march, and
// whether it writes the stops (a forward with checkpoints).
__global__ __launch_bounds__(64) void k_stop_header(int* __restrict__ tab, int tile_w, int L, int K, int written) {
    if (threadIdx.x == 0) {
        tab[0] = tile_w; tab[1] = L; tab[2] = K; tab[3] = written;
    }
}

// Header of the stash before a forward: its tiling, march and slot count, the
// request counter cleared, and whether the forward writes the stash.
__global__ __launch_bounds__(64) void k_stash_header(int* __restrict__ h, int tile_w, int L, int K, int written,
                                                     int slots) {
    if (threadIdx.x == 0) {
        h[0] = tile_w; h[1] = L; h[2] = K; h[3] = written; h[4] = 0; h[5] = slots;
    }
}

__global__ __launch_bounds__(64) void k_fill_int(int* __restrict__ p, int n, int v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(64) void k_put_desc(BatchDesc d, BatchDesc* __restrict__ dst) {
    const int* src = reinterpret_cast<const int*>(&d);
    int* out = reinterpret_cast<int*>(dst);
    constexpr int nw = (int)(sizeof(BatchDesc) / sizeof(int));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) out[i] = src[i];
}

// Labelled pixels of the fused loss: lcount[0] += semantic labels in [0, C),
// lcount[1] += finite positive depth labels (lcount zeroed before).
__global__ __launch_bounds__(256) void k_count_labels(int64_t n, int C, const int32_t* __restrict__ sem_label,
                                                      const float* __restrict__ depth_label, int* lcount) {
    __shared__ int part[2][4];
    int ns = 0, nd = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        ns += (unsigned)sem_label[i] < (unsigned)C ? 1 : 0;
        const float dl = depth_label[i];
        nd += ((dl > 0.0f) && (dl < INFINITY)) ? 1 : 0;
    }
    ns = wave_sum_int(ns);
    nd = wave_sum_int(nd);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { part[0][w] = ns; part[1][w] = nd; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { a += part[0][k]; b += part[1][k]; }
        atomicAdd(&lcount[0], a);
        atomicAdd(&lcount[1], b);
    }
}

// loss[0..2] = (total, L_sem, L_depth) from the per-tile partials, summed in
// tile order (deterministic).  One block of 256 threads.
constexpr int LOSS_THREADS = 1024;
__global__ __launch_bounds__(LOSS_THREADS) void k_loss_reduce(int tiles, const float* __restrict__ lpart,
                                                              const int* __restrict__ lcount, float lam_s,
                                                              float lam_d, float* loss) {
    __shared__ double red[2][LOSS_THREADS];
    // each thread its fixed stride of tiles, eight loads in flight; then a
    // fixed tree: the same order on every run
    const float2* lp = reinterpret_cast<const float2*>(lpart);
    double a = 0.0, b = 0.0;
#pragma unroll 8
    for (int t = threadIdx.x; t < tiles; t += LOSS_THREADS) {
        const float2 v = lp[t];
        a += (double)v.x;
        b += (double)v.y;
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int h = LOSS_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ls = lcount[0] > 0 ? red[0][0] / lcount[0] : 0.0;
        const double ld = lcount[1] > 0 ? red[1][0] / lcount[1] : 0.0;
        loss[0] = (float)(lam_s * ls + lam_d * ld);
        loss[1] = (float)ls;
        loss[2] = (float)ld;
    }
}

// ---------------------------------------------------------------------------
// Tile scheduling and lane setup
// ---------------------------------------------------------------------------
// The kernel's argument block (every render kernel takes one Ctx, at offset 0
// of the kernel argument segment) read through a pointer the compiler cannot
// see through.  Persistent loops read it once per tile: otherwise every field
// load is hoisted out of the loop and stays live in scalar registers, which
// then spill.
// (The host pass of hipcc cannot bind a constant-address-space object to the
// implicit copy constructor, so it sees a stub; only device code runs this.)
template <typename T>
__device__ __forceinline__ T kernel_arg0() {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) T* KPtr;
    KPtr p = (KPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    const T c = *p;
    return c;
#else
    return T();
#endif
}

template <bool PERSIST, typename F>
__device__ __forceinline__ void for_each_tile(const Ctx& P, F&& body) {
    const int wpb = blockDim.x >> 6;
    const int total = P.total_tiles;
    if (!PERSIST) {
        // wave-uniform by construction; readfirstlane tells the compiler so, which
        // keeps everything derived from the tile (scene, pointers) in SGPRs
        const int t = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6));
        if (t < total) body(t, P);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int xcd = blockIdx.x & (N_XCD - 1);
    const int per = (total + N_XCD - 1) / N_XCD;
    for (int q = 0; q < N_XCD; ++q) {
        const int x = (xcd + q) & (N_XCD - 1);
        const int lo = x * per, hi = min(total, lo + per);
        if (lo >= hi) continue;
        while (true) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&P.queue[x * QUEUE_STRIDE], 1);
            t = __builtin_amdgcn_readlane(t, 0);
            if (lo + t >= hi) break;
            body(lo + t, kernel_arg0<Ctx>());
        }
    }
}

__device__ __forceinline__ int find_scene(const BatchDesc* d, int tile) {
    const int ns = d->n_scenes;
    int s = 0;
    for (int i = 1; i < ns; ++i) s += (tile >= d->s[i].tile_off) ? 1 : 0;
    return s;
}

struct RayLane {
    bool valid;
    int cam, px, py;
    float ox, oy, oz, dx, dy, dz;
};

// pixel index inside the camera image, ray index inside the scene, global ray index
__device__ __forceinline__ int64_t lane_pix(const RayLane& rl, const SceneDev& S) {
    return (int64_t)rl.py * S.W + rl.px;
}
__device__ __forceinline__ int64_t lane_lray(const RayLane& rl, const SceneDev& S) {
    return ((int64_t)rl.cam * S.H + rl.py) * S.W + rl.px;
}
__device__ __forceinline__ int64_t lane_ray(const RayLane& rl, const SceneDev& S) {
    return S.ray_off + lane_lray(rl, S);
}

__device__ __forceinline__ RayLane setup_lane(const Ctx& P, const SceneDev& S, int tile) {
    RayLane rl;
    const int lane = threadIdx.x & 63;
    const int tw = P.desc->tile_w, th = P.desc->tile_h;
    const int tpc = S.tiles_x * S.tiles_y;
    rl.cam = tile / tpc;
    const int rem = tile - rl.cam * tpc;
    const int ty = rem / S.tiles_x, tx = rem - ty * S.tiles_x;
    rl.px = tx * tw + (lane % tw);
    rl.py = ty * th + (lane / tw);
    rl.valid = (rl.px < S.W) & (rl.py < S.H);
    rl.ox = rl.oy = rl.oz = rl.dx = rl.dy = rl.dz = 0.0f;
    if (rl.valid) {
        const int64_t ray = lane_ray(rl, S);
        const float* o = P.origins + 3 * ray;
        const float* d = P.dirs + 3 * ray;
        rl.ox = o[0]; rl.oy = o[1]; rl.oz = o[2];
        rl.dx = d[0]; rl.dy = d[1]; rl.dz = d[2];
    }
    return rl;
}

// Index view of one scene.
struct SceneIndex {
    const int32_t* counts;
    const int32_t* offsets;
    ci_ptr ids;
    int64_t cap;
    cf_ptr rec;     // records of the scene's primitives (local id k at rec + k*REC)
    cf_ptr lgp;
    int n;
    // Record and logit row of primitive k through a 32-bit byte offset (a
    // scene holds fewer than 2^25 primitives, so k * 4 * max(REC, CP) fits): the
    // scalar loads then take the offset in a register beside the scene's base,
    // one multiply per visit instead of a 64-bit multiply-add.
    typedef const __attribute__((address_space(4))) char* cb_ptr;
    __device__ __forceinline__ cf_ptr rec_at(int k) const {
        return (cf_ptr)((cb_ptr)rec + (uint32_t)k * (uint32_t)(REC * sizeof(float)));
    }
    template <int CP>
    __device__ __forceinline__ cf_ptr lgp_at(int k) const {
        return (cf_ptr)((cb_ptr)lgp + (uint32_t)k * (uint32_t)(CP * sizeof(float)));
    }
};

template <int CP>
__device__ __forceinline__ SceneIndex scene_index(const Ctx& P, int s, const SceneDev& S) {
    SceneIndex x;
    const int64_t nvox = (int64_t)P.g.X * P.g.Y * P.g.Z;
    x.counts = P.counts + (int64_t)s * nvox;
    x.offsets = P.offsets + (int64_t)s * nvox;
    x.ids = as_const(P.ids) + S.ids_base;
    x.cap = S.cap;
    x.rec = as_const(P.rec) + (size_t)S.prim_off * REC;
    x.lgp = as_const(P.lgp) + (size_t)S.prim_off * CP;
    x.n = S.n;
    return x;
}

// Uniform list length of voxel list (f0, n0), clamped to the scene's capacity.
__device__ __forceinline__ int clamp_list(int f0, int n0, int64_t cap) {
    if (f0 < 0) return 0;
    if ((int64_t)f0 + n0 > cap) return (int)max((int64_t)0, cap - f0);
    return n0;
}

// ---------------------------------------------------------------------------
// Per-wave union of voxel lists
//
// The index lists primitive k in voxel v exactly when v lies in k's clipped
// neighbourhood box (the packed box of its record), so a lane can test
// membership of any primitive in its own voxel's list from the record alone
// (in_box on the cell's packed word).  A per-wave LDS bitmap with one bit per
// primitive of the scene enumerates the union of several lists in ascending id.
// ---------------------------------------------------------------------------

// Visit the set bits of a per-wave bitmap in ascending order (wave-uniform);
// with CLEAR the words are zeroed as they are read.
template <bool CLEAR = false, typename F>
__device__ __forceinline__ void for_each_marked(uint32_t* bm, int nw, int lane, F&& body) {
    for (int wb = 0; wb < nw; wb += 64) {
        const uint32_t word = bm[wb + lane];
        if (CLEAR && word != 0u) bm[wb + lane] = 0u;
        uint64_t nz = wave_ballot(word != 0u);
        while (nz) {
            const int l = __builtin_ctzll(nz);
            nz &= nz - 1;
            uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)word, l);
            while (wv) {
                const int b = __builtin_ctz(wv);
                wv &= wv - 1;
                body(((wb + l) << 5) + b);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
template <int CP, bool CKPT, bool STATS, bool LOSS, bool STASH>
__device__ __forceinline__ void fwd_tile(const Ctx& P, int s, int tile, uint32_t* bm) {
    const SceneDev& S = P.desc->s[s];
    const RayLane rl = setup_lane(P, S, tile);
    const SceneIndex X = scene_index<CP>(P, s, S);
    const int lane = threadIdx.x & 63;
    const int nw = ((X.n + 31) / 32 + 63) / 64 * 64;     // bitmap words of this scene
    const int L = P.mr.L, K = P.mr.K;
    const int64_t R = (int64_t)S.cams * S.H * S.W;
    const int nck = CKPT ? (L + K - 1) / K : 0;
    float* ckpt = CKPT ? P.ckpt + (int64_t)nck * S.ray_off + lane_lray(rl, S) : nullptr;

    using CS = ClassSums<CP>;
    const LogitRows<CP> LR(X.lgp, X.n, lane);
    static_assert(CS::NX <= 1, "the stash holds at most one class beyond the four-wide accumulators");
    // the stash (forward with checkpoints): each chunk the tile enters takes a
    // slot of the pool, where the chunk's samples leave a and their class sums
    int* const stab = (CKPT && STASH && P.stash_tab) ? P.stash_tab + (int64_t)(S.tile_off + tile) * nck : nullptr;
    int stash_slot = -1;

    float T = rl.valid ? 1.0f : 0.0f;
    float D = 0.0f;
    CS Sv;
    Sv.zero();
    bool alive = rl.valid;
    int64_t st_samples = 0, st_pairs = 0, st_nz = 0;

    SamplePos nxt = pinned_sample(P.g, P.mr.t_near, P.mr.delta, 0, rl.ox, rl.oy, rl.oz, rl.dx, rl.dy, rl.dz);
    int n_nxt = 0, f_nxt = 0;
    if (alive && nxt.v >= 0) { n_nxt = X.counts[nxt.v]; f_nxt = X.offsets[nxt.v]; }
    int j_stop = L - 1;       // the last sample the tile composites

    for (int j = 0; j < L; ++j) {
        const SamplePos cur = nxt;
        const int n = n_nxt, f = f_nxt;
        if (j + 1 < L) {
            nxt = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j + 1, rl.ox, rl.oy, rl.oz, rl.dx, rl.dy, rl.dz);
            n_nxt = 0; f_nxt = 0;
            if (alive && nxt.v >= 0) { n_nxt = X.counts[nxt.v]; f_nxt = X.offsets[nxt.v]; }
        }
        if (CKPT && (j % K) == 0 && rl.valid) ckpt[(int64_t)(j / K) * R] = T;
        if (CKPT && stab && (j % K) == 0) {
            // one request per chunk, by the wave's first active lane
            const int lead = __builtin_ctzll(wave_ballot(true));
            int sl = 0;
            if (lane == lead) {
                sl = atomicAdd(P.stash_hdr + 4, 1);
                stab[j / K] = sl < P.stash_slots ? sl : -1;
            }
            sl = readlane_i(sl, lead);
            stash_slot = sl < P.stash_slots ? sl : -1;
        }
        // a ray that has left the grid for good adds nothing more; once every
        // lane has, the tile stops as it does when all rays are opaque
        if ((j & 3) == 0) alive = alive && !left_grid(P.g, cur, rl.dx, rl.dy, rl.dz);

        const bool act = alive && (cur.v >= 0) && (n > 0);
        const uint64_t am = wave_ballot(act);
        if (am != 0) {
            // Eq. eq:alpha_sem_sq: a = sum_k p_k sigma_k and s = sum_k p_k c_k over
            // the lane's own list, ascending id
            float a = 0.0f;
            CS sv;
            sv.zero();
            if (STATS && act) { ++st_samples; st_pairs += n; }
            // rr: the record of k, wave-uniform, in SGPRs; lx: its logits past
            // the matrix-core groups.  The whole wave runs each visit; lanes
            // outside it (mine false) add p = 0.  (A kept pair whose p
            // underflows to 0 leaves the sums' bits as they are, so only the
            // cull is tested.)
            auto visit = [&](int k, auto rec_words, auto lane_in) {
                constexpr int NR = decltype(rec_words)::value;
                float A[CS::NG][CS::W];
                LR.load(k, A);
                Pinned<NR> rr;
                Pinned<CS::XN> lx;
                if constexpr (CS::NX > 0) pin2(X.rec_at(k), rr, X.template lgp_at<CP>(k) + 4 * CS::NM, lx);
                else pin1(X.rec_at(k), rr);
                float p = 0.0f;
                if (lane_in(rr)) {
                    if (STATS && pair_kept(X.rec + (size_t)k * REC, cur.x, cur.y, cur.z)) ++st_nz;
                    if (eval_p_kept(rr, cur.x, cur.y, cur.z, p)) {
                        a = fmaf(p, rr[15], a);
#pragma unroll
                        for (int c = 0; c < CS::NX; ++c) sv.x[c] = fmaf(p, lx[c], sv.x[c]);
                    }
                }
                // the matrix op reads other lanes' operands, so it runs with the
                // whole wave (a uniform branch), p = 0 where no pair is kept;
                // skipped when every p is 0
                if (wave_ballot(p != 0.0f) != 0) class_mfma<CP>(sv, A, p);
            };
            const int lead = __builtin_ctzll(am);
            const int v_lead = readlane_i(cur.v, lead);
            if (wave_ballot(act && cur.v != v_lead) == 0) {
                // one voxel for every active lane: walk its list
                const int f0 = readlane_i(f, lead);
                const int n0 = clamp_list(f0, readlane_i(n, lead), X.cap);
                for (int e = 0; e < n0; ++e) {
                    const int k = X.ids[f0 + e];
                    if ((unsigned)k < (unsigned)X.n)
                        visit(k, std::integral_constant<int, 17>{}, [&](const Pinned<17>&) { return act; });
                }
            } else if (bm) {
                // several voxels: mark the union of their lists, then walk it
                bool pend = act;
                uint64_t m;
                while ((m = wave_ballot(pend)) != 0) {
                    const int g = __builtin_ctzll(m);
                    const int vg = readlane_i(cur.v, g);
                    const int fg = readlane_i(f, g);
                    const int ng = clamp_list(fg, readlane_i(n, g), X.cap);
                    for (int e = lane; e < ng; e += 64) {
                        const int k = X.ids[fg + e];
                        if ((unsigned)k < (unsigned)X.n) atomicOr(&bm[k >> 5], 1u << (k & 31));
                    }
                    pend = pend && (cur.v != vg);
                }
                wave_lds_sync();
                // the union walk runs only on grids whose cells fit the packed form
                const uint32_t cell = act ? pack_cell(cur.ix, cur.iy, cur.iz) : PV_DEAD;
                for_each_marked<true>(bm, nw, lane, [&](int k) {
                    visit(k, std::integral_constant<int, 19>{}, [&](const Pinned<19>& rr) {
                        return in_box(cell, __float_as_uint(rr[R_GLO]), __float_as_uint(rr[R_GHI]));
                    });
                });
                wave_lds_sync();
            } else {
                // several voxels, no bitmap: one voxel group at a time
                bool pend = act;
                uint64_t m;
                while ((m = wave_ballot(pend)) != 0) {
                    const int g = __builtin_ctzll(m);
                    const int vg = readlane_i(cur.v, g);
                    const int fg = readlane_i(f, g);
                    const int ng = clamp_list(fg, readlane_i(n, g), X.cap);
                    const bool mine = pend && (cur.v == vg);
                    for (int e = 0; e < ng; ++e) {
                        const int k = X.ids[fg + e];
                        if ((unsigned)k < (unsigned)X.n)
                            visit(k, std::integral_constant<int, 17>{}, [&](const Pinned<17>&) { return mine; });
                    }
                    pend = pend && !mine;
                }
            }
            if (CKPT && STASH && stash_slot >= 0 && act) {
                float* const sp = P.stash_pool + (int64_t)stash_slot * P.stash_slot_floats;
                const int jl = (j % K) * 64 + lane;
                f32x4_t* const mp = reinterpret_cast<f32x4_t*>(sp + (int64_t)jl * (4 * CS::NM));
#pragma unroll
                for (int i = 0; i < CS::NM; ++i) mp[i] = sv.m[i];
                float2 e;
                e.x = CS::NX > 0 ? sv.x[0] : 0.0f;
                e.y = a;
                reinterpret_cast<float2*>(sp + (int64_t)K * 64 * (4 * CS::NM))[jl] = e;
            }
            // Eq. eq:alpha_composite and eq:depth_sem
            const float alpha = fminf(a, 1.0f);
            const float w = T * alpha;
            D = fmaf(w, cur.t, D);
            Sv.add_scaled(w, sv);
            T = T * (1.0f - alpha);
            alive = alive && (T > 0.0f) && (T >= P.mr.kappa);
        }
        if (wave_ballot(alive) == 0) {
            // every later sample of this tile is exactly zero
            if (CKPT && rl.valid)
                for (int c = j / K + 1; c * K < L; ++c) ckpt[(int64_t)c * R] = T;
            // the chunks the tile does not enter have no slot
            if (CKPT && stab && lane == __builtin_ctzll(wave_ballot(true)))
                for (int c = j / K + 1; c < nck; ++c) stab[c] = -1;
            j_stop = j;
            break;
        }
    }
    // every lane stores the same value (no lane-divergent branch at the end of
    // the persistent tile loop's body)
    if (CKPT && P.tile_stop) P.tile_stop[STOP_HEAD + (int64_t)S.tile_off + tile] = j_stop;

    float ce = 0.0f, se = 0.0f;      // this lane's loss terms (LOSS)
    float Sc[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) Sc[c] = Sv.get(c);
    if (rl.valid) {
        const int64_t ray = lane_ray(rl, S);
        P.depth[ray] = D;
        P.t_final[ray] = T;
        const int64_t HW = (int64_t)S.H * S.W;
        const int64_t base = S.ray_off * P.C + (int64_t)rl.cam * P.C * HW + lane_pix(rl, S);
        float* semp = P.sem + base;
#pragma unroll
        for (int c = 0; c < CP; ++c)
            if (c < P.C) semp[c * HW] = Sc[c];
        if (P.probs || LOSS) {
            float mx = Sc[0];
#pragma unroll
            for (int c = 1; c < CP; ++c)
                if (c < P.C) mx = fmaxf(mx, Sc[c]);
            float e[CP];
            float sum = 0.0f;
#pragma unroll
            for (int c = 0; c < CP; ++c) {
                e[c] = c < P.C ? expf(Sc[c] - mx) : 0.0f;
                sum += e[c];
            }
            const float inv = 1.0f / sum;
            if (P.probs) {
                float* pp = P.probs + base;
#pragma unroll
                for (int c = 0; c < CP; ++c)
                    if (c < P.C) pp[c * HW] = e[c] * inv;
            }
            if (LOSS) {
                // Eq. eq:loss: cross-entropy of softmax(S_hat) against the class
                // label and squared depth error, each a mean over labelled pixels;
                // dL/dS_hat = lambda_s/N_s (softmax - onehot), dL/dD_hat = lambda_d/N_d 2 (D - D*)
                const int lab = P.sem_label[ray];
                const bool hs = (unsigned)lab < (unsigned)P.C;
                float s_lab = 0.0f;
#pragma unroll
                for (int c = 0; c < CP; ++c)
                    if (c == lab) s_lab = Sc[c];
                if (hs) ce = logf(sum) + mx - s_lab;
                const float ks = hs ? P.lam_s / (float)P.lcount[0] : 0.0f;
                float* gp = P.gs_out + base;
#pragma unroll
                for (int c = 0; c < CP; ++c)
                    if (c < P.C) gp[c * HW] = ks * (e[c] * inv - (c == lab ? 1.0f : 0.0f));
                const float dl = P.depth_label[ray];
                const bool hd = (dl > 0.0f) & (dl < INFINITY);
                const float diff = hd ? D - dl : 0.0f;
                se = diff * diff;
                P.gd_out[ray] = hd ? (P.lam_d / (float)P.lcount[1]) * 2.0f * diff : 0.0f;
            }
        }
    }
    if (LOSS) {
        // One partial per tile, written at the tile's global index, so the final
        // sum does not depend on which wave ran the tile.  Every lane stores lane
        // 0's totals: a lane-divergent branch here, at the end of the body of a
        // persistent tile loop, lets the compiler fold the branch into the
        // loop's exit mask and split the wavefront across tiles.
        ce = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_sum(ce))));
        se = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_sum(se))));
        const int64_t gt = (int64_t)S.tile_off + tile;
        P.lpart[2 * gt] = ce;
        P.lpart[2 * gt + 1] = se;
    }
    if (STATS && rl.valid) {
        atomicAdd((unsigned long long*)&P.stats[0], (unsigned long long)st_samples);
        atomicAdd((unsigned long long*)&P.stats[1], (unsigned long long)st_pairs);
        atomicAdd((unsigned long long*)&P.stats[2], (unsigned long long)st_nz);
        atomicAdd((unsigned long long*)&P.stats[3], 1ull);
    }
}

// Dynamic LDS: waves_per_block x bitmap_words words (zero bitmap_words: no
// union bitmap; mixed-voxel samples then walk one voxel group at a time).
template <int CP, bool CKPT, bool STATS, bool PERSIST, bool LOSS = false, bool STASH = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FWD_WPE(CP, CKPT, STATS, PERSIST, STASH), 8))) void k_render_fwd(Ctx P) {
    extern __shared__ uint32_t bm_all[];
    uint32_t* bm = nullptr;
    if (P.bitmap_words > 0) {
        bm = bm_all + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * P.bitmap_words;
        // the walks clear the words they read, so one clear per wave suffices
        for (int w = (int)(threadIdx.x & 63); w < P.bitmap_words; w += 64) bm[w] = 0u;
        wave_lds_sync();
    }
    for_each_tile<PERSIST>(P, [&](int t, const Ctx& Q) {
        const int s = find_scene(Q.desc, t);
        fwd_tile<CP, CKPT, STATS, LOSS, STASH>(Q, s, t - Q.desc->s[s].tile_off, bm);
    });
}

// ---------------------------------------------------------------------------
// Voxelisation (Supplement "SuperQuadric Voxelisation", Eq. eq:voxelisation)
//
// One workgroup of VOX_WAVES wavefronts per 4x4x4 block of voxels of one scene
// (blockIdx.y); in every wave one lane per voxel.  The waves mark the union of
// the block's lists in a shared LDS bitmap (wave w marks list entries w, w +
// VOX_WAVES, ...), then wave w walks the bitmap words w, w + VOX_WAVES, ... in
// ascending id; each lane takes the primitives whose box holds its voxel and
// evaluates p_o at its float32 voxel centre into partial sums
// v_d = sum p sigma, v_s = sum p c.  Wave 0 adds the other waves' partials in
// wave order (a fixed order: the result does not depend on scheduling).  The
// label is the first class maximising v_s, or C ("free") where v_d < tau.
// Without a bitmap (LDS budget exceeded) each lane walks its own list, wave w
// again taking entries w, w + VOX_WAVES, ...  Splitting a block over several
// waves shortens the dense blocks: a block's union runs to hundreds of
// primitives, visited one after another.
// ---------------------------------------------------------------------------
constexpr int VOX_WAVES = 4;
// LDS of a voxelisation workgroup: the bitmap, then the partial sums of waves
// 1 .. VOX_WAVES-1 ([wave][CP + 1][64]).
static size_t vox_lds_bytes(int words, int CP) {
    return (size_t)words * sizeof(uint32_t) + (size_t)(VOX_WAVES - 1) * (CP + 1) * 64 * sizeof(float);
}

template <int CP>
__global__ __launch_bounds__(64 * VOX_WAVES) void k_voxelise(Ctx P) {
    extern __shared__ uint32_t lds_all[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* bm = P.bitmap_words > 0 ? lds_all : nullptr;
    float* part = reinterpret_cast<float*>(lds_all + P.bitmap_words);
    for (int w = threadIdx.x; w < P.bitmap_words; w += 64 * VOX_WAVES) lds_all[w] = 0u;
    __syncthreads();
    const int nbx = (P.g.X + 3) >> 2, nby = (P.g.Y + 3) >> 2, nbz = (P.g.Z + 3) >> 2;
    const int blk = blockIdx.x;     // the grid holds exactly nbx * nby * nbz blocks
    const int s = blockIdx.y;
    const SceneDev& S = P.desc->s[s];
    const SceneIndex X = scene_index<CP>(P, s, S);
    const int nw = ((X.n + 31) / 32 + 63) / 64 * 64;
    const int bz = blk % nbz, by = (blk / nbz) % nby, bx = blk / (nbz * nby);
    const int ix = 4 * bx + (lane >> 4), iy = 4 * by + ((lane >> 2) & 3), iz = 4 * bz + (lane & 3);
    const bool valid = (ix < P.g.X) & (iy < P.g.Y) & (iz < P.g.Z);
    const int v = valid ? (ix * P.g.Y + iy) * P.g.Z + iz : 0;
    int n = 0, f = 0;
    if (valid) { n = X.counts[v]; f = X.offsets[v]; }
    const bool act = valid && n > 0;
    const float cx = pinned_voxel_centre(P.g.lox, P.g.vs, ix);
    const float cy = pinned_voxel_centre(P.g.loy, P.g.vs, iy);
    const float cz = pinned_voxel_centre(P.g.loz, P.g.vs, iz);

    float d = 0.0f;
    float sv[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) sv[c] = 0.0f;
    auto add_pair = [&](const auto& rr, const auto& lg) {
        float p;
        if (eval_p_kept(rr, cx, cy, cz, p)) {
            d = fmaf(p, rr[15], d);
#pragma unroll
            for (int c = 0; c < CP; ++c) sv[c] = fmaf(p, lg[c], sv[c]);
        }
    };
    const int n0 = act ? clamp_list(f, n, X.cap) : 0;
    if (bm) {
        // marking, sixteen of the lane's entries per round trip (the longest
        // list sets the marking's length)
        for (int e = wave; e < n0; e += 16 * VOX_WAVES) {
            int k[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int ei = e + i * VOX_WAVES;
                k[i] = ei < n0 ? X.ids[f + ei] : -1;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((unsigned)k[i] < (unsigned)X.n) atomicOr(&bm[k[i] >> 5], 1u << (k[i] & 31));
        }
        __syncthreads();
        // this wave's words of the union, ascending; the record (with its
        // per-axis box) and the logits of each primitive loaded behind one wait
        for (int jb = 0; jb * VOX_WAVES < nw; jb += 64) {
            const int wi = (jb + lane) * VOX_WAVES + wave;
            const uint32_t word = wi < nw ? bm[wi] : 0u;
            uint64_t nz = wave_ballot(word != 0u);
            while (nz) {
                const int l = __builtin_ctzll(nz);
                nz &= nz - 1;
                uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)word, l);
                const int base = ((jb + l) * VOX_WAVES + wave) << 5;
                while (wv) {
                    const int k = base + __builtin_ctz(wv);
                    wv &= wv - 1;
                    Pinned<25> rr;
                    Pinned<CP> lg;
                    pin2(X.rec_at(k), rr, X.template lgp_at<CP>(k), lg);
                    const bool mem = act && in_range(ix, __float_as_int(rr[22])) &&
                                     in_range(iy, __float_as_int(rr[23])) && in_range(iz, __float_as_int(rr[24]));
                    if (mem) add_pair(rr, lg);
                }
            }
        }
    } else {
        for (int e = wave; e < n0; e += VOX_WAVES) {
            const int k = P.ids[S.ids_base + f + e];
            if ((unsigned)k < (unsigned)X.n) add_pair(X.rec_at(k), X.template lgp_at<CP>(k));
        }
    }
    // the other waves' partials to wave 0, added in wave order
    if (wave > 0) {
        float* pw = part + (size_t)(wave - 1) * (CP + 1) * 64;
        pw[lane] = d;
#pragma unroll
        for (int c = 0; c < CP; ++c) pw[(c + 1) * 64 + lane] = sv[c];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 1; w < VOX_WAVES; ++w) {
        const float* pw = part + (size_t)(w - 1) * (CP + 1) * 64;
        d += pw[lane];
#pragma unroll
        for (int c = 0; c < CP; ++c) sv[c] += pw[(c + 1) * 64 + lane];
    }
    if (valid) {
        const int64_t nvox = (int64_t)P.g.X * P.g.Y * P.g.Z;
        const int64_t vo = (int64_t)s * nvox + v;
        P.vox_density[vo] = d;
        if (P.vox_sem) {
#pragma unroll
            for (int c = 0; c < CP; ++c)
                if (c < P.C) P.vox_sem[((int64_t)s * P.C + c) * nvox + v] = sv[c];
        }
        if (P.vox_labels) {
            int lab = P.C;
            if (!(d < P.tau)) {
                lab = 0;
                float best = sv[0];
#pragma unroll
                for (int c = 1; c < CP; ++c)
                    if (c < P.C && sv[c] > best) { best = sv[c]; lab = c; }
            }
            P.vox_labels[vo] = lab;
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of one (sample, primitive) pair through p = exp(-f) (Eq.
// eq:sq_occupancy_prob with f of Sec. "SuperQuadrics"), added to an
// accumulator row WITHOUT the primitive's constant factors; k_finalize
// multiplies each row entry by its factor once per primitive (acc_factor).
// With dfn = p dL/dp = -dL/df, base-2 logs and the quantities of eval_pair,
// which carry 1/ln 2 (B' = B/ln2, Z' = Z/ln2, r_u = (B/A) X/|u| / ln2, ...):
//   x[A_SIG]      += dL/da_j p                         (factor 1)
//   x[A_E1]       += dfn (e B' log2 A + b Z' log2|w|)  (factor  ln2^2 b / 2)
//   x[A_E2]       += dfn (B' log2 A - a S)             (factor -ln2^2 e a / 2)
//                    S = r_u |u| log2|u| + r_v |v| log2|v|
//   g = dfn (sign(u) r_u, sign(v) r_v, sign(w) q_w)    (factors -ln2 e a/s_x,
//   x[A_XS+i] += g_i, x[A_R+3i+c] += g_i (x-m)_c         -ln2 e a/s_y, -ln2 b/s_z)
// Where |u|, |v| or |w| is 0 its log2 is -inf, but the base it multiplies is
// then exactly 0, and so is the limit of the product; those products use the
// legacy multiply (0 x anything = 0), so no compare or select is needed.
// Inside the cull box r_u, r_v, q_w, B' and Z' are finite; the products with
// dfn still use the legacy multiply, so with p = 0 every term is exactly 0
// and callers need not test p.
// ---------------------------------------------------------------------------
template <int VP, typename RecT>
__device__ __forceinline__ void pair_adjoint(const RecT& r, const PairEval& ev, const float dd[3], float dfn,
                                             float da, float x[VP]) {
    const float a_ = r[12], b_ = r[13], e_ = r[14];
    const float g0 = mul0(dfn, with_sign_of(ev.ru, ev.u));
    const float g1 = mul0(dfn, with_sign_of(ev.rv, ev.v));
    const float g2 = mul0(dfn, with_sign_of(ev.qw, ev.w));
    const float bla = ev.B * ev.lA;
    const float S = mul0(ev.Xb, ev.lu) + mul0(ev.Yb, ev.lv);
    x[A_SIG] = fmaf(da, ev.p, x[A_SIG]);
    x[A_E1] = fmaf(dfn, fmaf(e_, bla, b_ * mul0(ev.Z, ev.lw)), x[A_E1]);
    x[A_E2] = fmaf(dfn, fmaf(-a_, S, bla), x[A_E2]);
    x[A_XS + 0] += g0; x[A_XS + 1] += g1; x[A_XS + 2] += g2;
    x[A_R + 0] = fmaf(g0, dd[0], x[A_R + 0]);
    x[A_R + 1] = fmaf(g0, dd[1], x[A_R + 1]);
    x[A_R + 2] = fmaf(g0, dd[2], x[A_R + 2]);
    x[A_R + 3] = fmaf(g1, dd[0], x[A_R + 3]);
    x[A_R + 4] = fmaf(g1, dd[1], x[A_R + 4]);
    x[A_R + 5] = fmaf(g1, dd[2], x[A_R + 5]);
    x[A_R + 6] = fmaf(g2, dd[0], x[A_R + 6]);
    x[A_R + 7] = fmaf(g2, dd[1], x[A_R + 7]);
    x[A_R + 8] = fmaf(g2, dd[2], x[A_R + 8]);
}

// The constant factor of accumulator entry vi of primitive record r (see
// pair_adjoint); 1 for the opacity and the logits.
__device__ __forceinline__ float acc_factor(cf_ptr r, int vi) {
    const float a_ = r[12], b_ = r[13], e_ = r[14];
    const float fu = -LN2 * e_ * a_, fw = -LN2 * b_;
    if (vi == A_E1) return 0.5f * LN2 * LN2 * b_;
    if (vi == A_E2) return -0.5f * LN2 * LN2 * e_ * a_;
    if (vi >= A_XS && vi < A_XS + 3)
        return vi == A_XS + 2 ? fw * r[R_INVS + 2] : fu * r[R_INVS + vi - A_XS];
    if (vi >= A_R && vi < A_R + 9) {
        const int i = (vi - A_R) / 3;
        return i == 2 ? fw * r[R_INVS + 2] : fu * r[R_INVS + i];
    }
    return 1.0f;
}

// ---------------------------------------------------------------------------
// Backward, sample-major (fallback): one reduction per (sample, primitive)
// ---------------------------------------------------------------------------
template <int CP, bool STATS>
__device__ __forceinline__ void bwd_sm_tile(const Ctx& P, int s, int tile, float* sw) {
    const SceneDev& S = P.desc->s[s];
    const RayLane rl = setup_lane(P, S, tile);
    const SceneIndex X = scene_index<CP>(P, s, S);
    constexpr int VP = AccRow<CP>::P;
    constexpr int V = AccRow<CP>::V;
    const int lane = threadIdx.x & 63;
    const int K = P.mr.K, L = P.mr.L;
    float* sm_a = sw;                 // a_j
    float* sm_T = sw + K * 64;        // T_j
    float* sm_G = sw + 2 * K * 64;    // G_j
    const int64_t R = (int64_t)S.cams * S.H * S.W;
    const int64_t HW = (int64_t)S.H * S.W;
    const int nck = (L + K - 1) / K;
    const float* ckpt = P.ckpt + (int64_t)nck * S.ray_off;
    float* acc = P.acc + (size_t)S.prim_off * VP;
    const float kappa = P.mr.kappa;

    const float gD = (rl.valid && P.g_depth) ? P.g_depth[lane_ray(rl, S)] : 0.0f;
    float gS[CP];
    const int64_t gbase = S.ray_off * P.C + (int64_t)rl.cam * P.C * HW + lane_pix(rl, S);
#pragma unroll
    for (int c = 0; c < CP; ++c) gS[c] = (rl.valid && P.g_sem && c < P.C) ? P.g_sem[gbase + c * HW] : 0.0f;

    float Q = 0.0f;
    int64_t st[6] = {0, 0, 0, 0, 0, 0};   // samples, listed, evaluated pairs of pass 1 and of pass 2
    for (int ci = nck - 1; ci >= 0; --ci) {
        const float Tc = rl.valid ? ckpt[(int64_t)ci * R + lane_lray(rl, S)] : 0.0f;
        if (wave_ballot((Tc > 0.0f) && (Tc >= kappa)) == 0) continue;
        const int j0 = ci * K;
        const int jn = min(K, L - j0);

        // ---- pass 1: front to back inside the chunk -------------------------
        float T = Tc;
        for (int jj = 0; jj < jn; ++jj) {
            const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j0 + jj, rl.ox, rl.oy, rl.oz,
                                               rl.dx, rl.dy, rl.dz);
            int n = 0, f = 0;
            // a sample the forward composited: T_j > 0 and T_j >= kappa (the same
            // float32 T_j, bit for bit, as the forward's)
            const bool pres = (T > 0.0f) && (T >= kappa);
            bool act = pres && (sp.v >= 0);
            if (act) { n = X.counts[sp.v]; f = X.offsets[sp.v]; act = n > 0; }
            if (STATS && act) { st[0] += 1; st[1] += n; }
            float a = 0.0f, G = 0.0f;
            bool pend = act;
            uint64_t m;
            while ((m = wave_ballot(pend)) != 0) {
                const int leader = __builtin_ctzll(m);
                const int v0 = readlane_i(sp.v, leader);
                const int f0 = readlane_i(f, leader);
                const int n0 = clamp_list(f0, readlane_i(n, leader), X.cap);
                const bool mine = pend && (sp.v == v0);
                if (mine) {
                    for (int e = 0; e < n0; ++e) {
                        const int k = X.ids[f0 + e];
                        if ((unsigned)k >= (unsigned)X.n) continue;
                        const cf_ptr r = X.rec + (size_t)k * REC;
                        const float p = eval_p(r, sp.x, sp.y, sp.z);
                        if (STATS && pair_kept(r, sp.x, sp.y, sp.z)) st[2] += 1;
                        if (p != 0.0f) {
                            a = fmaf(p, r[15], a);
                            const cf_ptr lg = X.lgp + (size_t)k * CP;
                            float gam = 0.0f;
#pragma unroll
                            for (int c = 0; c < CP; ++c) gam = fmaf(gS[c], lg[c], gam);
                            G = fmaf(p, gam, G);
                        }
                    }
                }
                pend = pend && !mine;
            }
            sm_a[jj * 64 + lane] = a;
            sm_T[jj * 64 + lane] = pres ? T : 0.0f;    // absent samples: no weight, no adjoint
            sm_G[jj * 64 + lane] = fmaf(gD, sp.t, G);
            T = T * (1.0f - fminf(a, 1.0f));
        }

        // ---- pass 2: back to front, per-pair adjoint -------------------------
        for (int jj = jn - 1; jj >= 0; --jj) {
            const float a = sm_a[jj * 64 + lane];
            const float Tj = sm_T[jj * 64 + lane];
            const float G = sm_G[jj * 64 + lane];
            const float alpha = fminf(a, 1.0f);
            const float dalpha = Tj * (G - Q);
            Q = fmaf(alpha, G, (1.0f - alpha) * Q);
            const float da = (a < 1.0f) ? dalpha : 0.0f;
            const float w = Tj * alpha;
            // (sigma_k = 0 with p > 0 still gives dL/dsigma_k = da p, so a == 0 is not a skip)
            const bool live = (Tj > 0.0f) && ((da != 0.0f) || (w != 0.0f));
            if (wave_ballot(live) == 0) continue;

            const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j0 + jj, rl.ox, rl.oy, rl.oz,
                                               rl.dx, rl.dy, rl.dz);
            int n = 0, f = 0;
            bool act = live && (sp.v >= 0);
            if (act) { n = X.counts[sp.v]; f = X.offsets[sp.v]; act = n > 0; }
            if (STATS && act) { st[3] += 1; st[4] += n; }
            bool pend = act;
            uint64_t m;
            while ((m = wave_ballot(pend)) != 0) {
                const int leader = __builtin_ctzll(m);
                const int v0 = readlane_i(sp.v, leader);
                const int f0 = readlane_i(f, leader);
                const int n0 = clamp_list(f0, readlane_i(n, leader), X.cap);
                const bool mine = pend && (sp.v == v0);
                for (int e = 0; e < n0; ++e) {
                    const int k = X.ids[f0 + e];
                    if ((unsigned)k >= (unsigned)X.n) continue;
                    const cf_ptr r = X.rec + (size_t)k * REC;
                    const cf_ptr lg = X.lgp + (size_t)k * CP;
                    float x[VP];
#pragma unroll
                    for (int i = 0; i < VP; ++i) x[i] = 0.0f;
                    bool any = false;
                    float wp = 0.0f;
                    if (mine) {
                        PairEval ev;
                        float dd[3];
                        const bool kept = eval_pair(r, sp.x, sp.y, sp.z, dd, ev);
                        if (STATS && kept) st[5] += 1;
                        if (kept && ev.p > 0.0f) {
                            any = true;
                            float gam = 0.0f;
#pragma unroll
                            for (int c = 0; c < CP; ++c) gam = fmaf(gS[c], lg[c], gam);
                            const float dfn = ev.p * fmaf(da, r[15], w * gam);
                            pair_adjoint<VP>(r, ev, dd, dfn, da, x);
                            wp = w * ev.p;
                        }
                    }
                    if (wave_ballot(any) == 0) continue;
#pragma unroll
                    for (int c = 0; c < CP; ++c) x[A_LG + c] = wp * gS[c];
                    const float tot = transpose_reduce<VP>(x, lane);
                    constexpr int shift = 6 - Log2<VP>::v;
                    const int vi = lane >> shift;
                    if (((lane & ((1 << shift) - 1)) == 0) && vi < V && (vi < A_LG || vi - A_LG < P.C))
                        atomicAdd(acc + (size_t)k * VP + vi, tot);
                }
                pend = pend && !mine;
            }
        }
    }
    if (STATS && rl.valid)
        for (int i = 0; i < 6; ++i) atomicAdd((unsigned long long*)&P.stats[i], (unsigned long long)st[i]);
}

template <int CP, bool STATS>
__global__ __launch_bounds__(256) void k_render_bwd(Ctx P) {
    extern __shared__ float smem[];   // [wave][3][K][64]
    float* sw = smem + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 3 * P.mr.K * 64;
    for_each_tile<false>(P, [&](int t, const Ctx& Q) {
        const int s = find_scene(Q.desc, t);
        bwd_sm_tile<CP, STATS>(Q, s, t - Q.desc->s[s].tile_off, sw);
    });
}

// ---------------------------------------------------------------------------
// Backward, primitive-major inside a chunk (default path)
//
// Per wavefront and chunk of KC samples:
//  1. the ids listed in the chunk's voxels are marked in a per-wave LDS bitmap
//     (one bit per primitive of the scene), which enumerates their union in
//     ascending id;
//  2. pass 1 walks that union: for each primitive k (wave-uniform, record in
//     SGPRs) every lane tests which of its KC samples lie in k's box
//     (= k is listed in the sample's voxel) and accumulates a_j += p sigma_k,
//     G_j += p <g_S, c_k>; summation order per sample is ascending id, as in
//     the forward;
//  3. compositing and its adjoint run per lane over the KC samples;
//  4. pass 2 walks the union again: each lane sums the contributions of all
//     its samples to k's parameters in registers, then the wave reduces them
//     once per (chunk, primitive) and lands them with one lane-parallel float
//     atomic.  Compared with one reduction per (sample, primitive), the
//     reductions and atomics shrink by the number of chunk samples that share
//     a primitive.
// ---------------------------------------------------------------------------
// With C = 17 the logit gradients of a (chunk, primitive) are not put through
// the 64-lane transposing reduction: each lane leaves om = sum_j w_j p_jk in LDS
// and lane (q, c) sums om x g_S[c] over the 16 lanes of row q for class c < 16,
// from a per-wave copy of g_S[0..15] in LDS written once per tile; the four
// rows are then added with two lane swaps.  Only the 15 geometric sums and
// class 16 go through the reduction (16 values instead of 32).
constexpr int LGS_STRIDE = 68;                     // floats per class row (bank-spread, 16-byte aligned)
constexpr int LGS_ZERO = 16 * LGS_STRIDE + 64;     // 16 zeros after the g_S rows and the om row
constexpr int LGS_FLOATS = LGS_ZERO + 16;
template <int CP> struct SplitLogits { static constexpr bool on = CP == 17; };

template <int CP, int KC, bool STATS>
__device__ __forceinline__ void bwd_km_tile(const Ctx& P, int s, int tile, uint32_t* bm, float* lgs) {
    const SceneDev& S = P.desc->s[s];
    const RayLane rl = setup_lane(P, S, tile);
    const SceneIndex X = scene_index<CP>(P, s, S);
    constexpr int VP = AccRow<CP>::P;
    constexpr int V = AccRow<CP>::V;
    const int lane = threadIdx.x & 63;
    // words of this scene's bitmap (its ids are local, 0 .. n-1)
    const int nw = ((X.n + 31) / 32 + 63) / 64 * 64;
    const int L = P.mr.L;
    const int64_t R = (int64_t)S.cams * S.H * S.W;
    const int64_t HW = (int64_t)S.H * S.W;
    const int nck = (L + KC - 1) / KC;
    const float* ckpt = P.ckpt + (int64_t)nck * S.ray_off;
    float* acc = P.acc + (size_t)S.prim_off * VP;
    const float kappa = P.mr.kappa;

    const float gD = (rl.valid && P.g_depth) ? P.g_depth[lane_ray(rl, S)] : 0.0f;
    float gS[CP];
    const int64_t gbase = S.ray_off * P.C + (int64_t)rl.cam * P.C * HW + lane_pix(rl, S);
#pragma unroll
    for (int c = 0; c < CP; ++c) gS[c] = (rl.valid && P.g_sem && c < P.C) ? P.g_sem[gbase + c * HW] : 0.0f;
    constexpr bool SPLIT = SplitLogits<CP>::on;
    if constexpr (SPLIT) {
#pragma unroll
        for (int c = 0; c < 16; ++c) lgs[c * LGS_STRIDE + lane] = gS[c];
    }
    // gamma_k = <g_S, c_k> for this lane's ray.  At C = 17 classes 0..15 are
    // read back from the per-wave LDS copy (the lane's column of the g_S rows),
    // which keeps 16 registers free across the chunk loop; the summation order
    // is the same either way.
    const float gS16 = gS[CP - 1];
    // lane constants of the pass-2 epilogue (C = 17): the selects of the
    // transposing reduction, the permute address of lane ^ 32, and each lane's
    // accumulator entries (the value index lane / 4: entries 0..14, class 16
    // for 15; and class lane for the 16 class sums)
    uint32_t m3 = 0u - (((uint32_t)lane >> 3) & 1u), m2 = 0u - (((uint32_t)lane >> 2) & 1u);
    asm volatile("" : "+v"(m3), "+v"(m2));
    const int bp32 = (lane ^ 32) << 2;
    const uint32_t off_tot = (lane >> 2) < 15 ? (uint32_t)(lane >> 2) : (uint32_t)(A_LG + 16);
    const uint32_t off_lgt = (uint32_t)(A_LG + (lane & 15));
    auto gamma_of = [&](const Pinned<CP>& lg) {
        float gam = 0.0f;
        if constexpr (SPLIT) {
#pragma unroll
            for (int c = 0; c < 16; ++c) gam = fmaf(lgs[c * LGS_STRIDE + lane], lg[c], gam);
            gam = fmaf(gS16, lg[16], gam);
        } else {
#pragma unroll
            for (int c = 0; c < CP; ++c) gam = fmaf(gS[c], lg[c], gam);
        }
        return gam;
    };

    int64_t st[6] = {0, 0, 0, 0, 0, 0};
    // past the sample where the forward stopped this tile every ray is opaque
    // or out of the grid: those samples add nothing
    int stop = L - 1;
    if (P.tile_stop) {
        const int* h = P.tile_stop;
        if (h[3] == 1 && h[0] == P.desc->tile_w && h[1] == L && h[2] == KC) {
            const int v = h[STOP_HEAD + (int64_t)S.tile_off + tile];
            stop = v < -1 ? -1 : v > L - 1 ? L - 1 : v;
        }
    }
    // the forward's per-sample values (stash), when that forward wrote them
    // with this tiling and chunk; the counting variant always recomputes
    const int* stab = nullptr;
    if (!STATS && P.stash_tab) {
        const int* h = P.stash_hdr;
        if (h[3] == 1 && h[0] == P.desc->tile_w && h[1] == L && h[2] == KC)
            stab = P.stash_tab + (int64_t)(S.tile_off + tile) * nck;
    }
    using CS = ClassSums<CP>;
    float Q = 0.0f;
    for (int ci = nck - 1; ci >= 0; --ci) {
        if (ci * KC > stop) continue;
        const float Tc = rl.valid ? ckpt[(int64_t)ci * R + lane_lray(rl, S)] : 0.0f;
        if (wave_ballot((Tc > 0.0f) && (Tc >= kappa)) == 0) continue;
        const int j0 = ci * KC;
        {
            // a ray that left the grid for good before the chunk adds nothing in it
            const SamplePos s0 = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j0, rl.ox, rl.oy, rl.oz, rl.dx, rl.dy,
                                               rl.dz);
            if (wave_ballot((Tc > 0.0f) && (Tc >= kappa) && !left_grid(P.g, s0, rl.dx, rl.dy, rl.dz)) == 0) continue;
        }

        // ---- chunk geometry + bitmap of the listed ids ----------------------
        // (the bitmap is clear here: cleared at the start, and pass 2 clears
        // every word it reads)
        float sx[KC], sy[KC], sz[KC];
        // packed cell of each sample (PV_DEAD: absent), two samples per 64 bits
        // so that a visit tests them in pairs (in_box2)
        CellPairs<KC> pv;
        int last_v = -1;
#pragma unroll
        for (int jj = 0; jj < KC; ++jj) {
            pv.set(jj, PV_DEAD);
            sx[jj] = sy[jj] = sz[jj] = 0.0f;
            if (j0 + jj <= stop) {
                const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j0 + jj, rl.ox, rl.oy, rl.oz,
                                                   rl.dx, rl.dy, rl.dz);
                sx[jj] = sp.x; sy[jj] = sp.y; sz[jj] = sp.z;
                int n = 0, f = 0;
                bool act = (Tc > 0.0f) && (Tc >= kappa) && (sp.v >= 0);
                if (act) { n = X.counts[sp.v]; f = X.offsets[sp.v]; act = n > 0; }
                if (act) pv.set(jj, pack_cell(sp.ix, sp.iy, sp.iz));
                bool pend = act;
                uint64_t m;
                while ((m = wave_ballot(pend)) != 0) {
                    const int leader = __builtin_ctzll(m);
                    const int v0 = readlane_i(sp.v, leader);
                    const int f0 = readlane_i(f, leader);
                    const int n0 = clamp_list(f0, readlane_i(n, leader), X.cap);
                    if (v0 != last_v) {
                        for (int e = lane; e < n0; e += 64) {
                            const int k = X.ids[f0 + e];
                            if ((unsigned)k < (unsigned)X.n) atomicOr(&bm[k >> 5], 1u << (k & 31));
                        }
                        last_v = v0;
                    }
                    pend = pend && (sp.v != v0);
                }
            }
        }
        wave_lds_sync();

        // ---- a_j and G_j: from the forward's stash, else pass 1 --------------
        float a[KC], G[KC];
#pragma unroll
        for (int jj = 0; jj < KC; ++jj) { a[jj] = 0.0f; G[jj] = 0.0f; }
        const int slot = stab ? stab[ci] : -1;
        if (slot >= 0 && slot < P.stash_slots) {
            // a_j as the forward summed it and G_j = <g_S, s_j> from its class
            // sums s_j = sum_k p c_k; samples the forward did not composite hold
            // stale values, which the compositing below never reads
            // through a buffer resource on the slot: the lane's offset in a
            // register, each sample's offset a scalar constant
            const float* const sp = P.stash_pool + (int64_t)slot * P.stash_slot_floats;
            const __amdgpu_buffer_rsrc_t srs =
                __builtin_amdgcn_make_buffer_rsrc((void*)sp, 0, (int)(KC * 64 * (4 * CS::NM + 2) * sizeof(float)),
                                                  0x00020000);
            constexpr int MB = 4 * CS::NM * (int)sizeof(float);     // class-sum bytes per lane and sample
            const uint32_t vm = (uint32_t)lane * MB, ve = (uint32_t)lane * 8u;
            // two samples per round trip (one at 32 classes, where two would
            // spill), loaded by every lane (the slot is in bounds whatever the
            // lane holds); absent samples are masked
            constexpr int NS = CP <= 17 ? 2 : 1;
#pragma unroll
            for (int j2 = 0; j2 < KC; j2 += NS) {
                __builtin_amdgcn_sched_barrier(0);
                CS cs[NS];
                float ea[NS];
#pragma unroll
                for (int h = 0; h < NS; ++h) {
                    const int jj = j2 + h;
#pragma unroll
                    for (int i = 0; i < CS::NM; ++i) {
                        const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(srs, vm, jj * 64 * MB + 16 * i, 0);
                        cs[h].m[i] = f32x4_t{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                                             __uint_as_float(v[3])};
                    }
                    const u32x2_t e = __builtin_amdgcn_raw_buffer_load_b64(srs, ve, KC * 64 * MB + jj * 64 * 8, 0);
                    if constexpr (CS::NX > 0) cs[h].x[0] = __uint_as_float(e[0]);
                    ea[h] = __uint_as_float(e[1]);
                }
                float g[NS];
#pragma unroll
                for (int h = 0; h < NS; ++h) g[h] = 0.0f;
#pragma unroll
                for (int c = 0; c < CP; ++c) {
                    float gs;
                    if constexpr (SPLIT) gs = c < 16 ? lgs[c * LGS_STRIDE + lane] : gS16;
                    else gs = gS[c];
#pragma unroll
                    for (int h = 0; h < NS; ++h) g[h] = fmaf(gs, cs[h].get(c), g[h]);
                }
#pragma unroll
                for (int h = 0; h < NS; ++h) {
                    const bool live = pv.get(j2 + h) != PV_DEAD;
                    a[j2 + h] = live ? ea[h] : 0.0f;
                    G[j2 + h] = live ? g[h] : 0.0f;
                }
            }
        } else {
            // ---- pass 1: a_j and G_j over the union, ascending id -----------
            for_each_marked(bm, nw, lane, [&](int k) {
                const cf_ptr r = X.rec_at(k);
                Pinned<19> rr;
                Pinned<CP> lg;
                pin2(r, rr, X.template lgp_at<CP>(k), lg);
                bool mem[KC];
                pv.members(__float_as_uint(rr[R_GLO]), __float_as_uint(rr[R_GHI]), mem);
                bool anym = false;
#pragma unroll
                for (int jj = 0; jj < KC; ++jj) anym |= mem[jj];
                if (wave_ballot(anym) == 0) return;
                const float sig = rr[15];
                // gamma up front: the sums are then updated inside each sample's
                // branch, and a culled pair costs no default value of p
                const float gam = gamma_of(lg);
                bool hit = false;
#pragma unroll
                for (int jj = 0; jj < KC; ++jj) {
                    if (mem[jj]) {
                        if (STATS) { st[1] += 1; if (pair_kept(r, sx[jj], sy[jj], sz[jj])) st[2] += 1; }
                        float p;
                        if (eval_p_kept(rr, sx[jj], sy[jj], sz[jj], p)) {
                            // (with p = 0 the sums keep their bits, as in the forward, which skips)
                            a[jj] = fmaf(p, sig, a[jj]);
                            G[jj] = fmaf(p, gam, G[jj]);
                            hit |= p != 0.0f;
                        }
                    }
                }
                if (wave_ballot(hit) == 0) {
                    // p = 0 for every lane and sample: the adjoint of k is 0 in this
                    // chunk, so pass 2 need not visit it
                    if (lane == 0) bm[k >> 5] &= ~(1u << (k & 31));
                }
            });
        }

        // ---- compositing and its adjoint (per lane) -------------------------
        float Tj[KC];
        {
            // the forward composited sample j only while T_j > 0 and T_j >= kappa;
            // absent samples get T_j = 0 here (no weight, no adjoint) and leave T as is
            float T = Tc;
#pragma unroll
            for (int jj = 0; jj < KC; ++jj) {
                const bool pres = (T > 0.0f) && (T >= kappa);
                Tj[jj] = pres ? T : 0.0f;
                if (pres) T = T * (1.0f - fminf(a[jj], 1.0f));
                // (an absent sample's values are not the forward's: zero them,
                // which leaves the recursion below as it is for finite ones)
                a[jj] = pres ? a[jj] : 0.0f;
                G[jj] = pres ? G[jj] : 0.0f;
            }
        }
#pragma unroll
        for (int jj = KC - 1; jj >= 0; --jj) {
            if (j0 + jj < L) {
                const float t = P.mr.t_near + (float)(j0 + jj) * P.mr.delta;
                // absent samples (T_j = 0 here) pass Q through unchanged
                const float al = Tj[jj] > 0.0f ? fminf(a[jj], 1.0f) : 0.0f;
                const float Gf = fmaf(gD, t, G[jj]);
                const float dal = Tj[jj] * (Gf - Q);
                Q = fmaf(al, Gf, (1.0f - al) * Q);
                const float da = (a[jj] < 1.0f) ? dal : 0.0f;
                const float w = Tj[jj] * al;
                if (STATS && pv.get(jj) != PV_DEAD) st[0] += 1;
                if (!(Tj[jj] > 0.0f) || (da == 0.0f && w == 0.0f)) pv.set(jj, PV_DEAD);
                if (STATS && pv.get(jj) != PV_DEAD) st[3] += 1;
                a[jj] = da;     // reuse: dL/da_j
                G[jj] = w;      // reuse: w_j
            }
        }

        // ---- pass 2: per-primitive adjoint over the union -------------------
        wave_lds_sync();
        for_each_marked<true>(bm, nw, lane, [&](int k) {
            const cf_ptr r = X.rec_at(k);
            Pinned<22> rr;
            Pinned<CP> lg;
            pin2(r, rr, X.template lgp_at<CP>(k), lg);
            bool mem[KC];
            pv.members(__float_as_uint(rr[R_GLO]), __float_as_uint(rr[R_GHI]), mem);
            bool anym = false;
#pragma unroll
            for (int jj = 0; jj < KC; ++jj) anym |= mem[jj];
            if (wave_ballot(anym) == 0) return;
            const float gam = gamma_of(lg);
            const float sig = rr[15];
            constexpr int VR = SPLIT ? 16 : VP;     // values reduced across the wave
            float x[VR];
            // At C = 17 the 16 sums start from four 16-byte LDS reads of a block
            // of zeros (no vector ALU instruction).  The block's address is made
            // opaque per visit: a hoisted read would be copied into the sums with
            // 16 moves.  The wider rows of the other class counts are cleared
            // with moves.
            if constexpr (SPLIT) {
                typedef const __attribute__((address_space(3))) f32x4_t* lds_f4;
                lds_f4 z4 = (lds_f4)(lgs + LGS_ZERO);
                asm volatile("" : "+v"(z4));
#pragma unroll
                for (int i = 0; i < VR / 4; ++i) {
                    const f32x4_t z = z4[i];
                    x[4 * i] = z[0]; x[4 * i + 1] = z[1]; x[4 * i + 2] = z[2]; x[4 * i + 3] = z[3];
                }
            } else {
#pragma unroll
                for (int i = 0; i < VR; ++i) x[i] = 0.0f;
            }
            float om = 0.0f;          // sum_j w_j p_jk
            bool anyk = false;
#pragma unroll
            for (int jj = 0; jj < KC; ++jj) {
                if (mem[jj]) {
                    PairEval ev;
                    float dd[3];
                    const bool kept = eval_pair(rr, sx[jj], sy[jj], sz[jj], dd, ev);
                    if (STATS) { st[4] += 1; if (kept) st[5] += 1; }
                    // (a kept pair whose p underflows to 0 adds exactly 0)
                    if (kept) {
                        anyk = true;
                        const float da = a[jj], w = G[jj];
                        const float dfn = ev.p * fmaf(da, sig, w * gam);
                        pair_adjoint<VR>(rr, ev, dd, dfn, da, x);
                        om = fmaf(w, ev.p, om);
                    }
                }
            }
            // a visit that kept no pair adds nothing: no reduction, no atomics
            // (with the stash, pass 2 also meets the primitives that pass 1
            // would have dropped for p = 0 throughout the chunk)
            if (wave_ballot(anyk) == 0) return;
            if constexpr (SPLIT) {
                // classes 0..15: lane (q, c) = (lane / 16, lane % 16)
                float* omr = lgs + 16 * LGS_STRIDE;
                omr[lane] = om;
                wave_lds_sync();
                const int q = lane >> 4, c = lane & 15;
                const float4* o4 = reinterpret_cast<const float4*>(omr + 16 * q);
                const float4* g4 = reinterpret_cast<const float4*>(lgs + c * LGS_STRIDE + 16 * q);
                float part = 0.0f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // one pair of 16-byte reads at a time (immediate offsets, 8 registers)
                    __builtin_amdgcn_sched_barrier(0);
                    const float4 o = o4[i], g = g4[i];
                    part = fmaf(o.x, g.x, part);
                    part = fmaf(o.y, g.y, part);
                    part = fmaf(o.z, g.z, part);
                    part = fmaf(o.w, g.w, part);
                }
                __builtin_amdgcn_sched_barrier(0);
                wave_lds_sync();
                const float lgt = row_sum4_lds(part, bp32);
                x[15] = om * gS16;
                const float tot = transpose_reduce16(x, m3, m2);
                // (the lane tests are compares per visit: held lane masks would
                // take scalar registers for the whole walk)
                float* const ak = acc + (size_t)k * VP;
                int ln = lane;
                asm volatile("" : "+v"(ln));
                if ((ln & 3) == 0) atomicAdd(ak + off_tot, tot);
                if (ln < 16) atomicAdd(ak + off_lgt, lgt);
            } else {
#pragma unroll
                for (int c = 0; c < CP; ++c) x[A_LG + c] = om * gS[c];
                const float tot = transpose_reduce<VP>(x, lane);
                constexpr int shift = 6 - Log2<VP>::v;
                const int vi = lane >> shift;
                if (((lane & ((1 << shift) - 1)) == 0) && vi < V && (vi < A_LG || vi - A_LG < P.C))
                    atomicAdd(acc + (size_t)k * VP + vi, tot);
            }
        });
    }
    if (STATS && rl.valid)
        for (int i = 0; i < 6; ++i) atomicAdd((unsigned long long*)&P.stats[i], (unsigned long long)st[i]);
}

template <int CP, int KC, bool STATS, bool PERSIST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BWD_WPE(CP, KC), 8))) void k_render_bwd_km(
    Ctx P) {
    extern __shared__ uint32_t bm_all[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* bm = bm_all + (size_t)wave * P.bitmap_words;
    // per-wave logit scratch after the block's bitmaps (C = 17 only)
    float* lgs = reinterpret_cast<float*>(bm_all + (size_t)(blockDim.x >> 6) * P.bitmap_words) +
                 (size_t)wave * LGS_FLOATS;
    // one clear per wave: every chunk's second pass clears the words it reads
    for (int w = (int)(threadIdx.x & 63); w < P.bitmap_words; w += 64) bm[w] = 0u;
    if constexpr (SplitLogits<CP>::on)
        if ((threadIdx.x & 63) < 16) lgs[LGS_ZERO + (threadIdx.x & 63)] = 0.0f;
    wave_lds_sync();
    for_each_tile<PERSIST>(P, [&](int t, const Ctx& Q) {
        const int s = find_scene(Q.desc, t);
        bwd_km_tile<CP, KC, STATS>(Q, s, t - Q.desc->s[s].tile_off, bm, lgs);
    });
}

// ---------------------------------------------------------------------------
// Superquadric-major backward (Sec. 3.3 "Backward Pass", Processes 1-3), an
// alternative to the wavefront-reduced atomics of the default backward:
//   1. per ray, replay the chunks from the checkpoints and store, per sample,
//      dL/da_j and w_j (k_sqm_replay);
//   2. build the (primitive, sample) interaction set from the index and group
//      it by primitive: count per primitive, scan, scatter sample ids into
//      contiguous per-primitive ranges (k_sqm_walk<false/true>, k_sqm_scan);
//   3. one block per primitive reduces its range: every interaction is
//      evaluated against the block's (uniform) record and the 15 + C sums are
//      reduced in registers, across the wavefront and across the block, and
//      written once -- no global atomics (k_sqm_reduce).
// ---------------------------------------------------------------------------

// Process 1: per sample dL/da_j (dA) and w_j (W), [rays x L], zero where the
// sample is absent or contributes nothing.  Chunk replay as in the
// sample-major backward (LDS per wave: a_j, T_j, G_j of one chunk).
template <int CP>
__device__ __forceinline__ void sqm_replay_tile(const Ctx& P, int s, int tile, float* sw, float* dA, float* W,
                                                float* gSr) {
    const SceneDev& S = P.desc->s[s];
    const RayLane rl = setup_lane(P, S, tile);
    const SceneIndex X = scene_index<CP>(P, s, S);
    const int lane = threadIdx.x & 63;
    const int K = P.mr.K, L = P.mr.L;
    float* sm_a = sw;
    float* sm_T = sw + K * 64;
    float* sm_G = sw + 2 * K * 64;
    const int64_t R = (int64_t)S.cams * S.H * S.W;
    const int64_t HW = (int64_t)S.H * S.W;
    const int nck = (L + K - 1) / K;
    const float* ckpt = P.ckpt + (int64_t)nck * S.ray_off;
    const float kappa = P.mr.kappa;
    const int64_t ray = rl.valid ? lane_ray(rl, S) : 0;

    const float gD = (rl.valid && P.g_depth) ? P.g_depth[ray] : 0.0f;
    float gS[CP];
    const int64_t gbase = S.ray_off * P.C + (int64_t)rl.cam * P.C * HW + lane_pix(rl, S);
#pragma unroll
    for (int c = 0; c < CP; ++c) gS[c] = (rl.valid && P.g_sem && c < P.C) ? P.g_sem[gbase + c * HW] : 0.0f;
    if (rl.valid) {
#pragma unroll
        for (int c = 0; c < CP; ++c) gSr[ray * CP + c] = gS[c];     // ray-major copy for Process 3
    }

    float Q = 0.0f;
    for (int ci = nck - 1; ci >= 0; --ci) {
        const int j0 = ci * K;
        const int jn = min(K, L - j0);
        const float Tc = rl.valid ? ckpt[(int64_t)ci * R + lane_lray(rl, S)] : 0.0f;
        if (wave_ballot((Tc > 0.0f) && (Tc >= kappa)) == 0) {
            if (rl.valid)
                for (int jj = 0; jj < jn; ++jj) { dA[ray * L + j0 + jj] = 0.0f; W[ray * L + j0 + jj] = 0.0f; }
            continue;
        }
        float T = Tc;
        for (int jj = 0; jj < jn; ++jj) {
            const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j0 + jj, rl.ox, rl.oy, rl.oz,
                                               rl.dx, rl.dy, rl.dz);
            int n = 0, f = 0;
            const bool pres = (T > 0.0f) && (T >= kappa);
            bool act = pres && (sp.v >= 0);
            if (act) { n = X.counts[sp.v]; f = X.offsets[sp.v]; act = n > 0; }
            float a = 0.0f, G = 0.0f;
            bool pend = act;
            uint64_t m;
            while ((m = wave_ballot(pend)) != 0) {
                const int leader = __builtin_ctzll(m);
                const int v0 = readlane_i(sp.v, leader);
                const int f0 = readlane_i(f, leader);
                const int n0 = clamp_list(f0, readlane_i(n, leader), X.cap);
                const bool mine = pend && (sp.v == v0);
                if (mine) {
                    for (int e = 0; e < n0; ++e) {
                        const int k = X.ids[f0 + e];
                        if ((unsigned)k >= (unsigned)X.n) continue;
                        const cf_ptr r = X.rec + (size_t)k * REC;
                        const float p = eval_p(r, sp.x, sp.y, sp.z);
                        if (p != 0.0f) {
                            a = fmaf(p, r[15], a);
                            const cf_ptr lg = X.lgp + (size_t)k * CP;
                            float gam = 0.0f;
#pragma unroll
                            for (int c = 0; c < CP; ++c) gam = fmaf(gS[c], lg[c], gam);
                            G = fmaf(p, gam, G);
                        }
                    }
                }
                pend = pend && !mine;
            }
            sm_a[jj * 64 + lane] = a;
            sm_T[jj * 64 + lane] = pres ? T : 0.0f;
            sm_G[jj * 64 + lane] = fmaf(gD, sp.t, G);
            T = T * (1.0f - fminf(a, 1.0f));
        }
        for (int jj = jn - 1; jj >= 0; --jj) {
            const float a = sm_a[jj * 64 + lane];
            const float Tj = sm_T[jj * 64 + lane];
            const float G = sm_G[jj * 64 + lane];
            const float alpha = fminf(a, 1.0f);
            const float dalpha = Tj * (G - Q);
            Q = fmaf(alpha, G, (1.0f - alpha) * Q);
            if (rl.valid) {
                dA[ray * L + j0 + jj] = (a < 1.0f) ? dalpha : 0.0f;
                W[ray * L + j0 + jj] = Tj * alpha;
            }
        }
    }
}

template <int CP>
__global__ __launch_bounds__(256) void k_sqm_replay(Ctx P, float* dA, float* W, float* gSr) {
    extern __shared__ float smem[];   // [wave][3][K][64]
    float* sw = smem + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 3 * P.mr.K * 64;
    for_each_tile<false>(P, [&](int t, const Ctx& Q) {
        const int s = find_scene(Q.desc, t);
        sqm_replay_tile<CP>(Q, s, t - Q.desc->s[s].tile_off, sw, dA, W, gSr);
    });
}

// Process 2, voxel-major.  The index lists primitive k in voxel v exactly
// when v lies in k's box, so k's interactions are the active samples (dL/da_j
// or w_j nonzero) of the voxels of its box.  Samples are bucketed by voxel
// (count, scan, scatter: one atomic per sample), then each primitive copies
// the buckets of its box, in voxel order, into its contiguous range.
// Single scene: the rays and voxels of scene 0.
template <bool SCATTER>
__global__ __launch_bounds__(256) void k_sqm_bucket(Ctx P, const float* __restrict__ dA,
                                                    const float* __restrict__ W, int* vcnt,
                                                    const int64_t* __restrict__ voff, int* vcur, uint32_t* vsamp) {
    const int L = P.mr.L;
    const int64_t n = P.desc->total_rays * (int64_t)L;
    for (int64_t sid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sid < n;
         sid += (int64_t)gridDim.x * blockDim.x) {
        if (dA[sid] == 0.0f && W[sid] == 0.0f) continue;
        const int64_t ray = sid / L;
        const int j = (int)(sid - ray * L);
        const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j, P.origins[3 * ray],
                                           P.origins[3 * ray + 1], P.origins[3 * ray + 2], P.dirs[3 * ray],
                                           P.dirs[3 * ray + 1], P.dirs[3 * ray + 2]);
        if (sp.v < 0 || P.counts[sp.v] == 0) continue;
        if (!SCATTER) {
            atomicAdd(&vcnt[sp.v], 1);
        } else {
            const int at = atomicAdd(&vcur[sp.v], 1);
            vsamp[voff[sp.v] + at] = (uint32_t)sid;
        }
    }
}

// cnt[k] = number of active samples in the voxels of k's box.
__global__ __launch_bounds__(256) void k_sqm_prim_count(Ctx P, const int* __restrict__ vcnt, int* cnt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.desc->total_prims) return;
    const float* r = P.rec + (size_t)k * REC;
    const int bx = __float_as_int(r[22]), by = __float_as_int(r[23]), bz = __float_as_int(r[24]);
    int64_t c = 0;
    if (bx != EMPTY_BOX)
        for (int ix = bx & 0xffff; ix <= (bx >> 16); ++ix)
            for (int iy = by & 0xffff; iy <= (by >> 16); ++iy) {
                const int64_t v0 = ((int64_t)ix * P.g.Y + iy) * P.g.Z;
                for (int iz = bz & 0xffff; iz <= (bz >> 16); ++iz) c += vcnt[v0 + iz];
            }
    cnt[k] = (int)min(c, (int64_t)INT_MAX);
}

// One block per primitive: copy the voxel buckets of its box into
// pairs[off[k] ...], dropping entries at or beyond capacity.
__global__ __launch_bounds__(256) void k_sqm_prim_fill(Ctx P, const int* __restrict__ vcnt,
                                                       const int64_t* __restrict__ voff,
                                                       const uint32_t* __restrict__ vsamp,
                                                       const int64_t* __restrict__ off, uint32_t* pairs,
                                                       int64_t capacity) {
    const int k = blockIdx.x;
    const float* r = P.rec + (size_t)k * REC;
    const int bx = __float_as_int(r[22]), by = __float_as_int(r[23]), bz = __float_as_int(r[24]);
    if (bx == EMPTY_BOX) return;
    int64_t pos = off[k];
    for (int ix = bx & 0xffff; ix <= (bx >> 16); ++ix)
        for (int iy = by & 0xffff; iy <= (by >> 16); ++iy) {
            const int64_t v0 = ((int64_t)ix * P.g.Y + iy) * P.g.Z;
            for (int iz = bz & 0xffff; iz <= (bz >> 16); ++iz) {
                const int nv = vcnt[v0 + iz];
                const int64_t src = voff[v0 + iz];
                for (int e = threadIdx.x; e < nv; e += blockDim.x)
                    if (pos + e < capacity) pairs[pos + e] = vsamp[src + e];
                pos += nv;
            }
        }
}

// Exclusive scan of the per-primitive counts into int64 offsets [n + 1]; one
// block; *total = off[n].
__global__ __launch_bounds__(1024) void k_sqm_scan(int n, const int* __restrict__ cnt, int64_t* off,
                                                   int64_t* total) {
    __shared__ int64_t part[1024];
    int64_t carry = 0;
    for (int base = 0; base < n; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int64_t v = i < n ? cnt[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t add = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) off[i] = carry + part[threadIdx.x] - v;
        carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        off[n] = carry;
        *total = carry;
    }
}

// Process 3: one block per primitive reduces its interaction range.
template <int CP>
__global__ __launch_bounds__(256) void k_sqm_reduce(Ctx P, const float* __restrict__ dA, const float* __restrict__ W,
                                                    const float* __restrict__ gSr, const int64_t* __restrict__ off,
                                                    const uint32_t* __restrict__ pairs, int64_t capacity) {
    constexpr int VP = AccRow<CP>::P;
    constexpr int V = AccRow<CP>::V;
    __shared__ float red[4][VP];
    const int kg = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int s = 0;
    for (int i = 1; i < P.desc->n_scenes; ++i) s += (kg >= P.desc->s[i].prim_off) ? 1 : 0;
    const SceneDev& S = P.desc->s[s];
    const cf_ptr r = as_const(P.rec) + (size_t)kg * REC;
    const cf_ptr lg = as_const(P.lgp) + (size_t)kg * CP;
    const int L = P.mr.L;
    const int64_t lo = off[kg], hi = min(off[kg + 1], capacity);
    float x[VP];
#pragma unroll
    for (int i = 0; i < VP; ++i) x[i] = 0.0f;
    float om = 0.0f;     // sum of w p over the range, for the logits
    float gsum[CP];      // sum of w p g_S per class
#pragma unroll
    for (int c = 0; c < CP; ++c) gsum[c] = 0.0f;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t sid = pairs[i];
        const int64_t ray = sid / (uint32_t)L;
        const int j = (int)(sid - (uint32_t)ray * (uint32_t)L);
        const float da = dA[sid], w = W[sid];
        const float ox = P.origins[3 * ray], oy = P.origins[3 * ray + 1], oz = P.origins[3 * ray + 2];
        const float dx = P.dirs[3 * ray], dy = P.dirs[3 * ray + 1], dz = P.dirs[3 * ray + 2];
        const SamplePos sp = pinned_sample(P.g, P.mr.t_near, P.mr.delta, j, ox, oy, oz, dx, dy, dz);
        PairEval ev;
        float dd[3];
        if (!eval_pair(r, sp.x, sp.y, sp.z, dd, ev) || !(ev.p > 0.0f)) continue;
        float gam = 0.0f;
        const float wp = w * ev.p;
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            const float g = gSr[ray * CP + c];
            gam = fmaf(g, lg[c], gam);
            gsum[c] = fmaf(wp, g, gsum[c]);
        }
        pair_adjoint<VP>(r, ev, dd, ev.p * fmaf(da, r[15], w * gam), da, x);
        om += wp;
    }
#pragma unroll
    for (int c = 0; c < CP; ++c) x[A_LG + c] = gsum[c];
    (void)om;
    const float tot = transpose_reduce<VP>(x, lane);
    constexpr int shift = 6 - Log2<VP>::v;
    const int vi = lane >> shift;
    if ((lane & ((1 << shift) - 1)) == 0 && vi < VP) red[wave][vi] = tot;
    __syncthreads();
    if ((int)threadIdx.x < VP) {
        const float v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        P.acc[(size_t)kg * VP + threadIdx.x] = (int)threadIdx.x < V ? v : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Finalize: accumulator row -> parameter gradients
//   g_m = -R^T sum(g_xs);  g_s_i = -(1/s_i) [G_R R^T]_ii  (G_R = sum g_xs (x-m)^T)
//   g_q = (I - q^ q^T)/|q| * sum_ij G_R_ij dR_ij/dq^
// ---------------------------------------------------------------------------
// With `stop` (the forward's tile-stop record, nullable): when that record
// says a forward with checkpoints ran with another sample count or chunk than
// this backward's (L, K), the checkpoint rows were laid out for the other
// chunk and every gradient written is NaN.
template <int CP>
__global__ __launch_bounds__(256) void k_finalize(int n_total, int C, const float* __restrict__ quats,
                                                  const float* __restrict__ scales, const float* __restrict__ rec,
                                                  const float* __restrict__ acc, float* g_means, float* g_quats,
                                                  float* g_scales, float* g_eps, float* g_opacity,
                                                  float* g_logits, const int* __restrict__ stop, int L, int K) {
    constexpr int VP = AccRow<CP>::P;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_total) return;
    if (stop && stop[3] == 1 && (stop[1] != L || stop[2] != K)) {
        const float nan = __int_as_float(0x7fc00000);
        for (int i = 0; i < 3; ++i) { g_means[3 * k + i] = nan; g_scales[3 * k + i] = nan; }
        for (int i = 0; i < 4; ++i) g_quats[4 * k + i] = nan;
        g_eps[2 * k] = g_eps[2 * k + 1] = nan;
        g_opacity[k] = nan;
        for (int c = 0; c < C; ++c) g_logits[(size_t)k * C + c] = nan;
        return;
    }
    // the accumulated sums carry no per-primitive constant factors (pair_adjoint)
    const cf_ptr r = as_const(rec) + (size_t)k * REC;
    float a[A_LG];
    for (int i = 0; i < A_LG; ++i) a[i] = acc[(size_t)k * VP + i] * acc_factor(r, i);
    const float q0 = quats[4 * k], q1 = quats[4 * k + 1], q2 = quats[4 * k + 2], q3 = quats[4 * k + 3];
    const float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const float w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    const float* gx = a + A_XS;
    const float* G = a + A_R;
    for (int i = 0; i < 3; ++i) g_means[3 * k + i] = -(R[i] * gx[0] + R[3 + i] * gx[1] + R[6 + i] * gx[2]);
    for (int i = 0; i < 3; ++i) {
        const float d = G[3 * i] * R[3 * i] + G[3 * i + 1] * R[3 * i + 1] + G[3 * i + 2] * R[3 * i + 2];
        g_scales[3 * k + i] = -d / scales[3 * k + i];
    }
    // sum_ij G_ij dR_ij/dq^ for the Hamilton matrix above
    const float gw = -2.f * z * G[1] + 2.f * y * G[2] + 2.f * z * G[3] - 2.f * x * G[5] - 2.f * y * G[6] +
                     2.f * x * G[7];
    const float gxq = 2.f * y * G[1] + 2.f * z * G[2] + 2.f * y * G[3] - 4.f * x * G[4] - 2.f * w * G[5] +
                      2.f * z * G[6] + 2.f * w * G[7] - 4.f * x * G[8];
    const float gy = -4.f * y * G[0] + 2.f * x * G[1] + 2.f * w * G[2] + 2.f * x * G[3] + 2.f * z * G[5] -
                     2.f * w * G[6] + 2.f * z * G[7] - 4.f * y * G[8];
    const float gz = -4.f * z * G[0] - 2.f * w * G[1] + 2.f * x * G[2] + 2.f * w * G[3] - 4.f * z * G[4] +
                     2.f * y * G[5] + 2.f * x * G[6] + 2.f * y * G[7];
    const float dot = w * gw + x * gxq + y * gy + z * gz;
    g_quats[4 * k + 0] = (gw - w * dot) / qn;
    g_quats[4 * k + 1] = (gxq - x * dot) / qn;
    g_quats[4 * k + 2] = (gy - y * dot) / qn;
    g_quats[4 * k + 3] = (gz - z * dot) / qn;
    g_eps[2 * k] = a[A_E1];
    g_eps[2 * k + 1] = a[A_E2];
    g_opacity[k] = a[A_SIG];
    for (int c = 0; c < C; ++c) g_logits[(size_t)k * C + c] = acc[(size_t)k * VP + A_LG + c];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int bitmap_words(int n) { return ((n + 31) / 32 + 63) / 64 * 64; }

void finish_desc(BatchDesc& d, int tile_w) {
    d.tile_w = tile_w;
    d.tile_h = 64 / tile_w;
    int tiles = 0, prims = 0, max_n = 0;
    int64_t rays = 0, ids = 0;
    for (int i = 0; i < d.n_scenes; ++i) {
        SceneDev& S = d.s[i];
        S.tiles_x = (S.W + d.tile_w - 1) / d.tile_w;
        S.tiles_y = (S.H + d.tile_h - 1) / d.tile_h;
        S.tile_off = tiles;
        S.prim_off = prims;
        S.ray_off = rays;
        S.ids_base = ids;
        tiles += S.cams * S.tiles_x * S.tiles_y;
        prims += S.n;
        rays += (int64_t)S.cams * S.H * S.W;
        ids += S.cap;
        max_n = std::max(max_n, S.n);
    }
    d.total_tiles = tiles;
    d.total_prims = prims;
    d.total_rays = rays;
    d.max_n = max_n;
}

struct WsSizes {
    size_t desc, queue, boxes, partials, rec, lgp, acc, lcount, lpart;
};
static WsSizes ws_sizes(const GridDev& g, const BatchDesc& d) {
    const int CP = padded_classes(d.C);
    WsSizes z;
    z.desc = align_up(sizeof(BatchDesc));
    z.queue = align_up(2 * N_XCD * QUEUE_STRIDE * sizeof(int));
    z.boxes = align_up((size_t)d.total_prims * sizeof(int4));
    z.partials = align_up(index_scratch_bytes(g, d));
    z.rec = align_up((size_t)d.total_prims * REC * sizeof(float));
    z.lgp = align_up((size_t)d.total_prims * CP * sizeof(float));
    z.acc = align_up((size_t)d.total_prims * acc_row(CP) * sizeof(float));
    z.lcount = align_up(2 * sizeof(int));
    z.lpart = align_up((size_t)d.total_tiles * 2 * sizeof(float));
    return z;
}

size_t batch_workspace_bytes(const GridDev& g, const BatchDesc& d) {
    const WsSizes z = ws_sizes(g, d);
    return z.desc + z.queue + z.boxes + z.partials + z.rec + z.lgp + z.acc + z.lcount + z.lpart;
}

size_t index_workspace_bytes(const GridDev& g, const BatchDesc& d) {
    const WsSizes z = ws_sizes(g, d);
    return z.desc + z.queue + z.boxes + z.partials;
}

WsLayout carve_ws(void* ws, const GridDev& g, const BatchDesc& d) {
    const WsSizes z = ws_sizes(g, d);
    char* p = (char*)ws;
    WsLayout l;
    l.desc = (BatchDesc*)p; p += z.desc;
    l.queue = (int*)p; p += z.queue;
    l.boxes = (int4*)p; p += z.boxes;
    l.partials = (int64_t*)p; p += z.partials;
    l.rec = (float*)p; p += z.rec;
    l.lgp = (float*)p; p += z.lgp;
    l.acc = (float*)p; p += z.acc;
    l.lcount = (int*)p; p += z.lcount;
    l.lpart = (float*)p;
    return l;
}

void put_desc(const BatchDesc& d, BatchDesc* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, st, d, dst);
}

hipError_t launch_batch_index(const GridDev& g, const BatchDesc& d, const BatchIO& io, void* ws, hipStream_t st) {
    const WsLayout l = carve_ws(ws, g, d);
    put_desc(d, l.desc, st);
    launch_index_kernels(g, d, l.desc, io, l.boxes, l.partials, st);
    return hipGetLastError();
}

static int cu_count() {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0;
        int n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n = 0;
        cached = n > 0 ? n : 256;
    }
    return cached;
}

template <typename Kern>
static void launch_tiles(Kern k, bool persistent, const Ctx& P, int wpb, size_t shm, hipStream_t st) {
    const dim3 block(64 * wpb);
    const int static_blocks = (P.total_tiles + wpb - 1) / wpb;
    if (static_blocks == 0) return;
    if (!persistent) {
        hipLaunchKernelGGL(k, dim3(static_blocks), block, shm, st, P);
        return;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, (int)block.x, shm) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const int blocks = std::min(static_blocks, per_cu * cu_count());
    hipLaunchKernelGGL(k, dim3(blocks), block, shm, st, P);
}

// One wave per tile on a static grid, with extra kernel arguments after the context.
template <typename Kern, typename... A>
static void launch_tiles_with(Kern k, const Ctx& P, int wpb, size_t shm, hipStream_t st, A... args) {
    const int static_blocks = (P.total_tiles + wpb - 1) / wpb;
    if (static_blocks == 0) return;
    hipLaunchKernelGGL(k, dim3(static_blocks), dim3(64 * wpb), shm, st, P, args...);
}

template <int CP>
static void prep_records(const BatchDesc& d, const GridDev& g, const BatchIO& io, const WsLayout& l,
                         hipStream_t st) {
    if (d.total_prims > 0)
        hipLaunchKernelGGL(k_prep_records<CP>, dim3((d.total_prims + 255) / 256), dim3(256), 0, st, d.total_prims,
                           d.C, io.means, io.quats, io.scales, io.eps, io.opacity, io.logits, g, l.rec, l.lgp);
}

static Ctx make_ctx(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                    const WsLayout& l, int64_t* stats) {
    Ctx P;
    P.g = g; P.mr = mr; P.C = d.C; P.total_tiles = d.total_tiles; P.desc = l.desc; P.queue = l.queue;
    P.counts = io.counts; P.offsets = io.offsets; P.ids = io.ids;
    P.rec = l.rec; P.lgp = l.lgp; P.origins = io.origins; P.dirs = io.dirs;
    P.depth = io.depth; P.sem = io.sem; P.probs = io.probs; P.t_final = io.t_final; P.ckpt = io.ckpt;
    P.g_depth = io.g_depth; P.g_sem = io.g_sem; P.acc = l.acc; P.stats = stats;
    P.bitmap_words = bitmap_words(d.max_n);
    P.tau = 0.0f;
    P.vox_density = io.vox_density; P.vox_sem = io.vox_sem; P.vox_labels = io.vox_labels;
    P.sem_label = io.sem_label; P.depth_label = io.depth_label;
    P.gd_out = const_cast<float*>(io.g_depth); P.gs_out = const_cast<float*>(io.g_sem);
    P.lam_s = P.lam_d = 0.0f;
    P.lcount = l.lcount; P.lpart = l.lpart;
    P.tile_stop = io.tile_stop;
    P.stash_hdr = nullptr; P.stash_tab = nullptr; P.stash_pool = nullptr;
    P.stash_slots = 0; P.stash_slot_floats = 0;
    // (a call without checkpoints only rewrites the header, marking the stash
    // as not its own)
    if (io.stash && io.stash_len >= STASH_HEAD) {
        P.stash_hdr = reinterpret_cast<int*>(io.stash);
        const StashGeom sg = stash_geom(d, mr.L, mr.K);
        if (mr.K > 0 && io.stash_len >= sg.pool_off) {
            P.stash_tab = P.stash_hdr + sg.tab_off;
            P.stash_pool = io.stash + sg.pool_off;
            P.stash_slots = (int)std::min<int64_t>((io.stash_len - sg.pool_off) / sg.slot_floats, INT32_MAX);
            P.stash_slot_floats = (int)sg.slot_floats;
        }
    }
    return P;
}

// Grids whose cells fit the packed form of in_box.
static bool cells_fit(const GridDev& g) { return g.X <= PV_MAX_XY && g.Y <= PV_MAX_XY && g.Z <= PV_MAX_Z; }
// LDS budget of the per-wave bitmaps of one block.
static bool bitmap_fits(int max_n, int wpb) {
    return (size_t)wpb * bitmap_words(max_n) * sizeof(uint32_t) <= 64 * 1024;
}
// LDS of a primitive-major backward block: the bitmaps, then (C = 17) each
// wave's logit scratch.
static size_t km_lds_bytes(int words, int wpb, int CP) {
    return (size_t)wpb * ((size_t)words * sizeof(uint32_t) + (CP == 17 ? LGS_FLOATS * sizeof(float) : 0));
}

template <int CP, bool LOSS>
static void fwd_launch(const Ctx& P, const TuneDev& t, size_t shm, hipStream_t st) {
    const int wpb = t.waves_per_block;
    const bool ck = P.ckpt != nullptr, sth = ck && P.stash_tab != nullptr;
    if (t.persistent) {
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, P.queue, N_XCD * QUEUE_STRIDE, 0);
        if (sth) launch_tiles(k_render_fwd<CP, true, false, true, LOSS, true>, true, P, wpb, shm, st);
        else if (ck) launch_tiles(k_render_fwd<CP, true, false, true, LOSS>, true, P, wpb, shm, st);
        else launch_tiles(k_render_fwd<CP, false, false, true, LOSS>, true, P, wpb, shm, st);
    } else {
        if (sth) launch_tiles(k_render_fwd<CP, true, false, false, LOSS, true>, false, P, wpb, shm, st);
        else if (ck) launch_tiles(k_render_fwd<CP, true, false, false, LOSS>, false, P, wpb, shm, st);
        else launch_tiles(k_render_fwd<CP, false, false, false, LOSS>, false, P, wpb, shm, st);
    }
}

template <int CP>
static void fwd_run(const GridDev& g, const BatchDesc& d, const BatchIO& io, const WsLayout& l, const Ctx& P0,
                    const TuneDev& t, hipStream_t st, const LossArgs* loss) {
    prep_records<CP>(d, g, io, l, st);
    const int wpb = t.waves_per_block;
    Ctx P = P0;
    // the stash serves only the primitive-major backward of this tuning; the
    // counting variant does not write it
    if (P.stash_tab && (P.stats || !(t.bwd_mode != 1 && bwd_primitive_major_ok(g, d.max_n, P.mr.K, wpb)))) {
        P.stash_tab = nullptr;
        P.stash_pool = nullptr;
    }
    if (P.tile_stop)
        hipLaunchKernelGGL(k_stop_header, dim3(1), dim3(64), 0, st, P.tile_stop, d.tile_w, P.mr.L, P.mr.K,
                           P.ckpt != nullptr && P.mr.K > 0 ? 1 : 0);
    if (P.stash_hdr)
        hipLaunchKernelGGL(k_stash_header, dim3(1), dim3(64), 0, st, P.stash_hdr, d.tile_w, P.mr.L, P.mr.K,
                           P.ckpt != nullptr && P.stash_tab != nullptr ? 1 : 0, P.stash_slots);
    // the union walk tests membership on packed cells
    if (!bitmap_fits(d.max_n, wpb) || !cells_fit(g)) P.bitmap_words = 0;
    const size_t shm = (size_t)wpb * P.bitmap_words * sizeof(uint32_t);
    const bool ck = P.ckpt != nullptr, stt = P.stats != nullptr;
    if (loss) {
        // labelled-pixel counts first: the forward's epilogue divides by them
        P.lam_s = loss->lambda_sem;
        P.lam_d = loss->lambda_depth;
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, l.lcount, 2, 0);
        if (d.total_rays > 0) {
            const int64_t blocks = std::min<int64_t>((d.total_rays + 255) / 256, 2048);
            hipLaunchKernelGGL(k_count_labels, dim3((unsigned)blocks), dim3(256), 0, st, (int64_t)d.total_rays, d.C,
                               io.sem_label, io.depth_label, l.lcount);
        }
        fwd_launch<CP, true>(P, t, shm, st);
        hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(LOSS_THREADS), 0, st, d.total_tiles, (const float*)l.lpart,
                           (const int*)l.lcount, loss->lambda_sem, loss->lambda_depth, io.loss);
        return;
    }
    if (stt) {
        if (ck) launch_tiles(k_render_fwd<CP, true, true, false>, false, P, wpb, shm, st);
        else launch_tiles(k_render_fwd<CP, false, true, false>, false, P, wpb, shm, st);
        return;
    }
    fwd_launch<CP, false>(P, t, shm, st);
}

hipError_t launch_batch_fwd(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                            int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st, const LossArgs* loss) {
    const WsLayout l = carve_ws(ws, g, d);
    put_desc(d, l.desc, st);
    const Ctx P = make_ctx(g, d, mr, io, l, stats);
    switch (padded_classes(d.C)) {
        case 4: fwd_run<4>(g, d, io, l, P, tune, st, loss); break;
        case 8: fwd_run<8>(g, d, io, l, P, tune, st, loss); break;
        case 17: fwd_run<17>(g, d, io, l, P, tune, st, loss); break;
        default: fwd_run<32>(g, d, io, l, P, tune, st, loss); break;
    }
    return hipGetLastError();
}

template <int CP>
static void vox_run(const GridDev& g, const BatchDesc& d, const BatchIO& io, const WsLayout& l, const Ctx& P0,
                    hipStream_t st) {
    prep_records<CP>(d, g, io, l, st);
    Ctx P = P0;
    // one shared bitmap per block, within the LDS budget of a block
    if (vox_lds_bytes(P.bitmap_words, CP) > 64 * 1024) P.bitmap_words = 0;
    const size_t shm = vox_lds_bytes(P.bitmap_words, CP);
    const int64_t nblk = (int64_t)((g.X + 3) / 4) * ((g.Y + 3) / 4) * ((g.Z + 3) / 4);
    const dim3 grid((unsigned)nblk, (unsigned)d.n_scenes);
    hipLaunchKernelGGL(k_voxelise<CP>, grid, dim3(64 * VOX_WAVES), shm, st, P);
}

hipError_t launch_batch_voxelise(const GridDev& g, const BatchDesc& d, const BatchIO& io, float tau, void* ws,
                                 hipStream_t st) {
    const WsLayout l = carve_ws(ws, g, d);
    put_desc(d, l.desc, st);
    MarchDev mr;
    mr.L = 1; mr.t_near = 0.0f; mr.delta = 0.0f; mr.K = 0;
    Ctx P = make_ctx(g, d, mr, io, l, nullptr);
    P.tau = tau;
    switch (padded_classes(d.C)) {
        case 4: vox_run<4>(g, d, io, l, P, st); break;
        case 8: vox_run<8>(g, d, io, l, P, st); break;
        case 17: vox_run<17>(g, d, io, l, P, st); break;
        default: vox_run<32>(g, d, io, l, P, st); break;
    }
    return hipGetLastError();
}

// ---- superquadric-major backward ------------------------------------------
// Interaction workspace (caller's): dA, W [rays x L] float; cnt [prims] int;
// off [prims + 1] int64; cur [prims] uint64; pairs [capacity + 1] uint32 (the
// last slot is a write sink for lanes without an interaction).
struct SqmLayout {
    float *dA, *W, *gSr;
    int *vcnt, *vcur;
    int64_t* voff;
    uint32_t* vsamp;
    int* cnt;
    int64_t* off;
    uint32_t* pairs;
};

static SqmLayout carve_sqm(void* iws, const GridDev& g, const BatchDesc& d, const MarchDev& mr, int64_t capacity,
                           size_t* bytes) {
    const int64_t V = (int64_t)g.X * g.Y * g.Z;
    const int64_t S = d.total_rays * (int64_t)mr.L;
    const size_t s_dw = align_up((size_t)S * sizeof(float));
    const size_t s_gs = align_up((size_t)d.total_rays * padded_classes(d.C) * sizeof(float));
    const size_t s_vc = align_up((size_t)V * sizeof(int));
    const size_t s_vo = align_up(((size_t)V + 1) * sizeof(int64_t));
    const size_t s_vs = align_up((size_t)S * sizeof(uint32_t));
    const size_t s_cnt = align_up((size_t)d.total_prims * sizeof(int));
    const size_t s_off = align_up(((size_t)d.total_prims + 1) * sizeof(int64_t));
    const size_t s_pairs = align_up(((size_t)capacity + 1) * sizeof(uint32_t));
    if (bytes) *bytes = 2 * s_dw + s_gs + 2 * s_vc + s_vo + s_vs + s_cnt + s_off + s_pairs;
    SqmLayout l{};
    char* p = (char*)iws;
    if (!p) return l;
    l.dA = (float*)p; p += s_dw;
    l.W = (float*)p; p += s_dw;
    l.gSr = (float*)p; p += s_gs;
    l.vcnt = (int*)p; p += s_vc;
    l.vcur = (int*)p; p += s_vc;
    l.voff = (int64_t*)p; p += s_vo;
    l.vsamp = (uint32_t*)p; p += s_vs;
    l.cnt = (int*)p; p += s_cnt;
    l.off = (int64_t*)p; p += s_off;
    l.pairs = (uint32_t*)p;
    return l;
}

size_t sq_major_workspace_bytes(const GridDev& g, const BatchDesc& d, const MarchDev& mr, int64_t capacity) {
    size_t b = 0;
    carve_sqm(nullptr, g, d, mr, capacity, &b);
    return b;
}

template <int CP>
static void sqm_run(const GridDev& g, const BatchDesc& d, const BatchIO& io, const WsLayout& l, const Ctx& P,
                    const SqmLayout& q, int64_t capacity, int64_t* total, int wpb, hipStream_t st) {
    prep_records<CP>(d, g, io, l, st);
    const int n = d.total_prims;
    const int V = g.X * g.Y * g.Z;
    const int64_t S = d.total_rays * (int64_t)P.mr.L;
    const unsigned sblocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((S + 255) / 256, 8192));
    const size_t shm = (size_t)wpb * 3 * P.mr.K * 64 * sizeof(float);
    launch_tiles_with(k_sqm_replay<CP>, P, wpb, shm, st, q.dA, q.W, q.gSr);                   // Process 1
    // Process 2: samples bucketed by voxel, then gathered per primitive box
    hipLaunchKernelGGL(k_fill, dim3((V + 255) / 256), dim3(256), 0, st, (float*)q.vcnt, (int64_t)V, 0.0f);
    hipLaunchKernelGGL(k_fill, dim3((V + 255) / 256), dim3(256), 0, st, (float*)q.vcur, (int64_t)V, 0.0f);
    hipLaunchKernelGGL(k_sqm_bucket<false>, dim3(sblocks), dim3(256), 0, st, P, (const float*)q.dA,
                       (const float*)q.W, q.vcnt, (const int64_t*)q.voff, q.vcur, q.vsamp);
    hipLaunchKernelGGL(k_sqm_scan, dim3(1), dim3(1024), 0, st, V, (const int*)q.vcnt, q.voff, q.voff + V);
    hipLaunchKernelGGL(k_sqm_bucket<true>, dim3(sblocks), dim3(256), 0, st, P, (const float*)q.dA,
                       (const float*)q.W, q.vcnt, (const int64_t*)q.voff, q.vcur, q.vsamp);
    if (n > 0)
        hipLaunchKernelGGL(k_sqm_prim_count, dim3((n + 255) / 256), dim3(256), 0, st, P, (const int*)q.vcnt, q.cnt);
    hipLaunchKernelGGL(k_sqm_scan, dim3(1), dim3(1024), 0, st, n, (const int*)q.cnt, q.off, total);
    if (n > 0) {
        hipLaunchKernelGGL(k_sqm_prim_fill, dim3((unsigned)n), dim3(256), 0, st, P, (const int*)q.vcnt,
                           (const int64_t*)q.voff, (const uint32_t*)q.vsamp, (const int64_t*)q.off, q.pairs,
                           capacity);
        hipLaunchKernelGGL(k_sqm_reduce<CP>, dim3((unsigned)n), dim3(256), 0, st, P, (const float*)q.dA,
                           (const float*)q.W, (const float*)q.gSr, (const int64_t*)q.off,
                           (const uint32_t*)q.pairs, capacity);                                      // Process 3
        hipLaunchKernelGGL(k_finalize<CP>, dim3((n + 255) / 256), dim3(256), 0, st, n, d.C, io.quats, io.scales,
                           (const float*)l.rec, (const float*)l.acc, io.g_means, io.g_quats, io.g_scales,
                           io.g_eps, io.g_opacity, io.g_logits, (const int*)nullptr, P.mr.L, P.mr.K);
    }
}

hipError_t launch_batch_bwd_sq_major(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                                     int64_t capacity, int64_t* total, void* iws, const TuneDev& tune, void* ws,
                                     hipStream_t st) {
    const WsLayout l = carve_ws(ws, g, d);
    put_desc(d, l.desc, st);
    const SqmLayout q = carve_sqm(iws, g, d, mr, capacity, nullptr);
    Ctx P = make_ctx(g, d, mr, io, l, nullptr);
    const int wpb = tune.waves_per_block;
    switch (padded_classes(d.C)) {
        case 4: sqm_run<4>(g, d, io, l, P, q, capacity, total, wpb, st); break;
        case 8: sqm_run<8>(g, d, io, l, P, q, capacity, total, wpb, st); break;
        case 17: sqm_run<17>(g, d, io, l, P, q, capacity, total, wpb, st); break;
        default: sqm_run<32>(g, d, io, l, P, q, capacity, total, wpb, st); break;
    }
    return hipGetLastError();
}

// The primitive-major backward needs the chunk in registers (K <= 8), a
// per-wave bitmap that fits the LDS budget, and voxel coordinates that fit the
// packed form.  Otherwise the sample-major backward runs.
bool bwd_primitive_major_ok(const GridDev& g, int max_n, int K, int wpb) {
    if (!(K == 4 || K == 8)) return false;
    if (!cells_fit(g)) return false;
    // sized for the largest per-wave scratch (C = 17), whatever C is
    return km_lds_bytes(bitmap_words(max_n), wpb, 17) <= 64 * 1024;
}

template <int CP, int KC>
static void bwd_km_launch(const Ctx& P, const TuneDev& t, hipStream_t st) {
    const int wpb = t.waves_per_block;
    const size_t shm = km_lds_bytes(P.bitmap_words, wpb, CP);
    if (P.stats) {
        launch_tiles(k_render_bwd_km<CP, KC, true, false>, false, P, wpb, shm, st);
    } else if (t.persistent) {
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, P.queue, N_XCD * QUEUE_STRIDE, 0);
        launch_tiles(k_render_bwd_km<CP, KC, false, true>, true, P, wpb, shm, st);
    } else {
        launch_tiles(k_render_bwd_km<CP, KC, false, false>, false, P, wpb, shm, st);
    }
}

template <int CP>
static void bwd_run(const GridDev& g, const BatchDesc& d, const BatchIO& io, const WsLayout& l, const Ctx& P,
                    const TuneDev& t, hipStream_t st) {
    prep_records<CP>(d, g, io, l, st);
    const int64_t nacc = (int64_t)d.total_prims * AccRow<CP>::P;
    if (nacc > 0)
        hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((nacc + 255) / 256, 4096)), dim3(256), 0, st,
                           l.acc, nacc, 0.0f);
    const int wpb = t.waves_per_block;
    const bool km = t.bwd_mode != 1 && bwd_primitive_major_ok(g, d.max_n, P.mr.K, wpb);
    if (km) {
        if (P.mr.K == 4) bwd_km_launch<CP, 4>(P, t, st);
        else bwd_km_launch<CP, 8>(P, t, st);
    } else {
        const size_t shm = (size_t)wpb * 3 * P.mr.K * 64 * sizeof(float);
        if (P.stats) launch_tiles(k_render_bwd<CP, true>, false, P, wpb, shm, st);
        else launch_tiles(k_render_bwd<CP, false>, false, P, wpb, shm, st);
    }
    if (d.total_prims > 0)
        hipLaunchKernelGGL(k_finalize<CP>, dim3((d.total_prims + 255) / 256), dim3(256), 0, st, d.total_prims, d.C,
                           io.quats, io.scales, (const float*)l.rec, (const float*)l.acc, io.g_means,
                           io.g_quats, io.g_scales, io.g_eps, io.g_opacity, io.g_logits,
                           (const int*)io.tile_stop, P.mr.L, P.mr.K);
}

hipError_t launch_batch_bwd(const GridDev& g, const BatchDesc& d, const MarchDev& mr, const BatchIO& io,
                            int64_t* stats, const TuneDev& tune, void* ws, hipStream_t st) {
    const WsLayout l = carve_ws(ws, g, d);
    put_desc(d, l.desc, st);
    Ctx P = make_ctx(g, d, mr, io, l, stats);
    P.queue = l.queue + N_XCD * QUEUE_STRIDE;   // the backward's own counters
    switch (padded_classes(d.C)) {
        case 4: bwd_run<4>(g, d, io, l, P, tune, st); break;
        case 8: bwd_run<8>(g, d, io, l, P, tune, st); break;
        case 17: bwd_run<17>(g, d, io, l, P, tune, st); break;
        default: bwd_run<32>(g, d, io, l, P, tune, st); break;
    }
    return hipGetLastError();
}

}  // namespace sqr

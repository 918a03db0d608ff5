// Superquadric -> voxel lists (Sec. 3.3 "Preliminary Construction").
//
// The paper builds, per primitive, the voxel coordinates of its cubic
// neighbourhood of half-width N_v (V_c) and "hashes" them into three dense
// per-voxel tensors: V_n (count), V_f (first offset) and V_sq (ids).  Here:
//
//   k_prep_boxes    one thread per primitive: pinned float32 centre voxel and
//                   the clipped box, packed lo|hi<<16 per axis.
//   k_tile_lists    one workgroup per voxel tile.  The workgroup streams the
//                   boxes of all primitives in ascending id, keeps the ones
//                   that overlap the tile (ordered compaction into LDS), and
//                   every thread (= one voxel of the tile) walks that ordered
//                   candidate batch.  Count mode writes V_n; write mode appends
//                   ids at V_f[v] in ascending order.  No atomics, no sort:
//                   the output is deterministic by construction.
//   k_scan_*        exclusive prefix sum V_f = scan(V_n) and E = sum(V_n).
#include "sqr_device.h"
#include "sqr_internal.h"
#include "sqr_launch.h"

namespace sqr {

constexpr int TILE_THREADS = 256;
constexpr int CAND_CAP = 2048;      // LDS candidate batch (id + packed box = 16 B each)

__global__ __launch_bounds__(256) void k_prep_boxes(const float* __restrict__ means, const float* __restrict__ quats,
                                                    const float* __restrict__ scales, const float* __restrict__ eps,
                                                    const float* __restrict__ opacity, int n, GridDev g,
                                                    int4* __restrict__ boxes) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int b[3];
    prim_box(g, means + 3 * k, quats + 4 * k, scales + 3 * k, eps + 2 * k, opacity + k, b);
    boxes[k] = make_int4(b[0], b[1], b[2], 0);
}

__device__ __forceinline__ bool box_has(int bx, int i) {
    return (i >= (bx & 0xffff)) & (i <= (bx >> 16));
}
__device__ __forceinline__ bool box_overlaps(int bx, int lo, int hi) {
    return ((bx & 0xffff) <= hi) & ((bx >> 16) >= lo);
}

struct TileShape {
    int tx, ty, tz;       // tile extent in voxels
    int ntx, nty, ntz;    // tiles per axis
};

template <bool WRITE>
__global__ __launch_bounds__(TILE_THREADS) void k_tile_lists(const BatchDesc* __restrict__ desc,
                                                              const int4* __restrict__ boxes_all, GridDev g,
                                                              TileShape ts, int32_t* __restrict__ counts_all,
                                                              const int32_t* __restrict__ offsets_all,
                                                              int32_t* __restrict__ ids_all) {
    __shared__ int4 cand[CAND_CAP];
    __shared__ int wave_cnt[TILE_THREADS / 64];
    __shared__ int batch_n;

    const int scene = blockIdx.y;
    const SceneDev& S = desc->s[scene];
    const int n = S.n;
    const int4* boxes = boxes_all + S.prim_off;
    const int64_t nvox = (int64_t)g.X * g.Y * g.Z;
    int32_t* counts = counts_all + (int64_t)scene * nvox;
    const int32_t* offsets = WRITE ? offsets_all + (int64_t)scene * nvox : nullptr;
    int32_t* ids = WRITE ? ids_all + S.ids_base : nullptr;
    const int64_t capacity = S.cap;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int t = blockIdx.x;
    const int tzi = t % ts.ntz; t /= ts.ntz;
    const int tyi = t % ts.nty; t /= ts.nty;
    const int txi = t;
    const int x0 = txi * ts.tx, y0 = tyi * ts.ty, z0 = tzi * ts.tz;
    const int x1 = min(x0 + ts.tx, g.X) - 1, y1 = min(y0 + ts.ty, g.Y) - 1, z1 = min(z0 + ts.tz, g.Z) - 1;

    // this thread's voxel (z fastest inside the tile)
    const int lz = tid % ts.tz, ly = (tid / ts.tz) % ts.ty, lx = tid / (ts.tz * ts.ty);
    const int ix = x0 + lx, iy = y0 + ly, iz = z0 + lz;
    const bool mine = (lx < ts.tx) & (ix <= x1) & (iy <= y1) & (iz <= z1);
    const int v = mine ? ((ix * g.Y + iy) * g.Z + iz) : 0;
    int cnt = 0;
    int64_t cursor = 0;
    if (WRITE && mine) cursor = offsets[v];

    if (tid == 0) batch_n = 0;
    __syncthreads();
    for (int base = 0; base < n; base += TILE_THREADS) {
        const int k = base + tid;
        int4 b = make_int4(EMPTY_BOX, EMPTY_BOX, EMPTY_BOX, 0);
        if (k < n) b = boxes[k];
        const bool keep = (k < n) && box_overlaps(b.x, x0, x1) && box_overlaps(b.y, y0, y1) &&
                          box_overlaps(b.z, z0, z1);
        const uint64_t m = wave_ballot(keep);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int before = batch_n;
        for (int w = 0; w < wave; ++w) before += wave_cnt[w];
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (keep) cand[before + rank] = make_int4(k, b.x, b.y, b.z);
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < TILE_THREADS / 64; ++w) tot += wave_cnt[w];
            batch_n += tot;
        }
        __syncthreads();
        const int nb = batch_n;
        const bool last = base + TILE_THREADS >= n;
        if (nb > CAND_CAP - TILE_THREADS || last) {
            if (mine) {
                for (int c = 0; c < nb; ++c) {
                    const int4 cb = cand[c];
                    if (box_has(cb.y, ix) & box_has(cb.z, iy) & box_has(cb.w, iz)) {
                        if (WRITE) {
                            // (the host keeps every offset within int32 and the
                            // capacity; the guard holds whatever offsets hold)
                            if (cursor >= 0 && cursor < capacity) ids[cursor] = cb.x;
                            ++cursor;
                        } else {
                            ++cnt;
                        }
                    }
                }
            }
            __syncthreads();
            if (tid == 0) batch_n = 0;
            __syncthreads();
        }
    }
    if (!WRITE && mine) counts[v] = cnt;
}

// ---------------------------------------------------------------------------
// Exclusive scan over the voxel counts of each scene (three passes over
// 2048-element blocks; blockIdx.y = scene).
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_PER_THREAD;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t val, int64_t* sh, int64_t& total) {
    // Hillis-Steele over 256 threads in LDS (int64 to detect E >= 2^31)
    const int tid = threadIdx.x;
    sh[tid] = val;
    __syncthreads();
    for (int d = 1; d < SCAN_BLOCK; d <<= 1) {
        const int64_t add = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    total = sh[SCAN_BLOCK - 1];
    const int64_t incl = sh[tid];
    __syncthreads();
    return incl - val;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_partials(const int32_t* __restrict__ counts_all, int64_t nvox,
                                                              int nparts, int64_t* __restrict__ partials_all) {
    __shared__ int64_t sh[SCAN_BLOCK];
    const int32_t* counts = counts_all + (int64_t)blockIdx.y * nvox;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; ++i)
        if (base + i < nvox) s += counts[base + i];
    int64_t tot;
    block_exclusive_scan(s, sh, tot);
    if (threadIdx.x == 0) partials_all[(int64_t)blockIdx.y * nparts + blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_top(int64_t* __restrict__ partials_all, int nparts,
                                                         int64_t* __restrict__ totals) {
    __shared__ int64_t sh[SCAN_BLOCK];
    int64_t* partials = partials_all + (int64_t)blockIdx.x * nparts;
    int64_t carry = 0;
    for (int base = 0; base < nparts; base += SCAN_BLOCK) {
        const int i = base + threadIdx.x;
        const int64_t v = i < nparts ? partials[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, sh, tot);
        if (i < nparts) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(const int32_t* __restrict__ counts_all, int64_t nvox,
                                                           int nparts, const int64_t* __restrict__ part_off_all,
                                                           int32_t* __restrict__ offsets_all) {
    __shared__ int64_t sh[SCAN_BLOCK];
    const int32_t* counts = counts_all + (int64_t)blockIdx.y * nvox;
    int32_t* offsets = offsets_all + (int64_t)blockIdx.y * nvox;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int32_t c[SCAN_PER_THREAD];
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; ++i) {
        c[i] = (base + i < nvox) ? counts[base + i] : 0;
        s += c[i];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan(s, sh, tot) + part_off_all[(int64_t)blockIdx.y * nparts + blockIdx.x];
    for (int i = 0; i < SCAN_PER_THREAD; ++i) {
        if (base + i < nvox) offsets[base + i] = (int32_t)run;
        run += c[i];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static TileShape pick_tile(const GridDev& g) {
    TileShape ts;
    ts.tz = g.Z < 16 ? g.Z : 16;
    int rest = TILE_THREADS / ts.tz;   // columns per tile
    int side = 1;
    while ((side * 2) * (side * 2) <= rest) side *= 2;
    ts.tx = side;
    ts.ty = rest / side;
    if (ts.ty > side * 2) ts.ty = side * 2;
    ts.ntx = (g.X + ts.tx - 1) / ts.tx;
    ts.nty = (g.Y + ts.ty - 1) / ts.ty;
    ts.ntz = (g.Z + ts.tz - 1) / ts.tz;
    return ts;
}

int scan_parts(const GridDev& g) {
    const int64_t nvox = (int64_t)g.X * g.Y * g.Z;
    return (int)((nvox + SCAN_TILE - 1) / SCAN_TILE);
}

void launch_index_kernels(const GridDev& g, const BatchDesc& d, const BatchDesc* desc_dev, const BatchIO& io,
                          int4* boxes, int64_t* partials, hipStream_t st) {
    const int64_t nvox = (int64_t)g.X * g.Y * g.Z;
    const int np = scan_parts(g);
    const int S = d.n_scenes;
    if (d.total_prims > 0)
        hipLaunchKernelGGL(k_prep_boxes, dim3((d.total_prims + 255) / 256), dim3(256), 0, st, io.means, io.quats,
                           io.scales, io.eps, io.opacity, d.total_prims, g, boxes);
    const TileShape ts = pick_tile(g);
    const int ntiles = ts.ntx * ts.nty * ts.ntz;
    hipLaunchKernelGGL(k_tile_lists<false>, dim3(ntiles, S), dim3(TILE_THREADS), 0, st, desc_dev,
                       (const int4*)boxes, g, ts, io.counts, (const int32_t*)nullptr, (int32_t*)nullptr);
    hipLaunchKernelGGL(k_scan_partials, dim3(np, S), dim3(SCAN_BLOCK), 0, st, (const int32_t*)io.counts, nvox, np,
                       partials);
    hipLaunchKernelGGL(k_scan_top, dim3(S), dim3(SCAN_BLOCK), 0, st, partials, np, io.totals);
    hipLaunchKernelGGL(k_scan_final, dim3(np, S), dim3(SCAN_BLOCK), 0, st, (const int32_t*)io.counts, nvox, np,
                       (const int64_t*)partials, io.offsets);
    hipLaunchKernelGGL(k_tile_lists<true>, dim3(ntiles, S), dim3(TILE_THREADS), 0, st, desc_dev,
                       (const int4*)boxes, g, ts, io.counts, (const int32_t*)io.offsets, io.ids);
}

}  // namespace sqr

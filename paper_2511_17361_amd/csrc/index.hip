// Superquadric -> voxel lists (Sec. 3.3 "Preliminary Construction").
//
// The paper builds, per primitive, the voxel coordinates of its cubic
// neighbourhood of half-width N_v (V_c) and "hashes" them into three dense
// per-voxel tensors: V_n (count), V_f (first offset) and V_sq (ids).  Here:
//
//   k_prep_boxes    one thread per primitive: pinned float32 centre voxel and
//                   the clipped box, packed lo|hi<<16 per axis.
//   k_bin_*         binning of the primitives by voxel tile: every primitive
//                   counts the tiles its box overlaps, an exclusive scan gives
//                   each tile's slice of a candidate array, and every primitive
//                   writes its id into the slices of its tiles (in any order).
//   k_tile_lists    one workgroup per voxel tile.  In count mode it sorts its
//                   tile's candidate slice in LDS (ascending id) and writes it
//                   back; both modes then stream that sorted slice, keep the
//                   boxes that overlap the tile (ordered compaction into LDS),
//                   and every thread (= one voxel of the tile) walks that
//                   ordered candidate batch.  Count mode writes V_n; write mode
//                   appends ids at V_f[v] in ascending order.  Work and traffic
//                   are O(N x tiles per box + E).  A tile whose slice exceeds
//                   the LDS sort streams every primitive of the scene instead,
//                   in ascending id.  Either way the lists are ascending and
//                   the output is deterministic: no atomic decides an order.
//   k_scan_*        exclusive prefix sum V_f = scan(V_n) and E = sum(V_n).
#include <algorithm>
#include <climits>

#include "sqr_device.h"
#include "sqr_internal.h"
#include "sqr_launch.h"

namespace sqr {

constexpr int TILE_THREADS = 256;
constexpr int CAND_CAP = 2048;      // LDS candidate batch (id + packed box = 16 B each)
constexpr int SORT_CAP = 4096;      // largest tile slice sorted in LDS (4 B per id)

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

// Scene of a global primitive index (scenes are few; a linear scan).
__device__ __forceinline__ int scene_of_prim(const BatchDesc* d, int k) {
    int s = 0;
    for (int i = 1; i < d->n_scenes; ++i) s += (k >= d->s[i].prim_off) ? 1 : 0;
    return s;
}

// Tile range of a packed box along one axis (empty: lo > hi).
__device__ __forceinline__ void tile_range(int bx, int t, int& lo, int& hi) {
    lo = (bx & 0xffff) / t;
    hi = (bx >> 16) / t;
}

// Tiles overlapped by primitive k's box; calls f(linear tile) for each.
template <typename F>
__device__ __forceinline__ void for_each_tile_of(const int4& b, const TileShape& ts, F&& f) {
    if (b.x == EMPTY_BOX) return;
    int x0, x1, y0, y1, z0, z1;
    tile_range(b.x, ts.tx, x0, x1);
    tile_range(b.y, ts.ty, y0, y1);
    tile_range(b.z, ts.tz, z0, z1);
    for (int x = x0; x <= x1; ++x)
        for (int y = y0; y <= y1; ++y)
            for (int z = z0; z <= z1; ++z) f((x * ts.nty + y) * ts.ntz + z);
}

// tile_cnt[scene][tile] += 1 for every tile each primitive's box overlaps
__global__ __launch_bounds__(256) void k_bin_count(const BatchDesc* __restrict__ desc,
                                                   const int4* __restrict__ boxes, int n_total, TileShape ts,
                                                   int* __restrict__ tile_cnt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_total) return;
    const int ntiles = ts.ntx * ts.nty * ts.ntz;
    int* cnt = tile_cnt + (int64_t)scene_of_prim(desc, k) * ntiles;
    for_each_tile_of(boxes[k], ts, [&](int t) { atomicAdd(&cnt[t], 1); });
}

// Exclusive scan of each scene's tile counts (one block per scene); the
// cursors start at the offsets.  Scene s's slices start at prim_off(s) x the
// most tiles one box overlaps, so the scenes' regions of the candidate array
// are disjoint.
__global__ __launch_bounds__(256) void k_bin_scan(const BatchDesc* __restrict__ desc, const int* __restrict__ tile_cnt,
                                                  int ntiles, int64_t tiles_per_box, int64_t* __restrict__ tile_off,
                                                  int64_t* __restrict__ tile_cur) {
    __shared__ int64_t sh[256];
    const int s = blockIdx.x;
    const int* cnt = tile_cnt + (int64_t)s * ntiles;
    int64_t* off = tile_off + (int64_t)s * ntiles;
    int64_t* cur = tile_cur + (int64_t)s * ntiles;
    int64_t carry = (int64_t)desc->s[s].prim_off * tiles_per_box;
    for (int base = 0; base < ntiles; base += 256) {
        const int i = base + threadIdx.x;
        const int64_t v = i < ntiles ? cnt[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int64_t add = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) {
            off[i] = carry + sh[threadIdx.x] - v;
            cur[i] = carry + sh[threadIdx.x] - v;
        }
        carry += sh[255];
        __syncthreads();
    }
}

// Every primitive writes its (scene-local) id into the slice of each tile its
// box overlaps (order within a slice is arbitrary; the list kernel sorts).
__global__ __launch_bounds__(256) void k_bin_fill(const BatchDesc* __restrict__ desc,
                                                  const int4* __restrict__ boxes, int n_total, TileShape ts,
                                                  int64_t* __restrict__ tile_cur, int32_t* __restrict__ cand) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_total) return;
    const int ntiles = ts.ntx * ts.nty * ts.ntz;
    const int s = scene_of_prim(desc, k);
    int64_t* cur = tile_cur + (int64_t)s * ntiles;
    const int local = k - desc->s[s].prim_off;
    for_each_tile_of(boxes[k], ts, [&](int t) {
        const int64_t pos = atomicAdd((unsigned long long*)&cur[t], 1ull);
        cand[pos] = local;
    });
}

// Ascending sort of n ints in LDS by the block (bitonic, padded to a power of two).
__device__ void block_sort(int* a, int n) {
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = n + (int)threadIdx.x; i < m; i += blockDim.x) a[i] = INT_MAX;
    __syncthreads();
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (m >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int x = a[lo], y = a[hi];
                if ((x > y) == up) { a[lo] = y; a[hi] = x; }
            }
            __syncthreads();
        }
    }
}

template <bool WRITE>
__global__ __launch_bounds__(TILE_THREADS) void k_tile_lists(const BatchDesc* __restrict__ desc,
                                                              const int4* __restrict__ boxes_all, GridDev g,
                                                              TileShape ts, int32_t* __restrict__ counts_all,
                                                              const int32_t* __restrict__ offsets_all,
                                                              int32_t* __restrict__ ids_all,
                                                              const int* __restrict__ tile_cnt,
                                                              const int64_t* __restrict__ tile_off,
                                                              int32_t* __restrict__ bin) {
    __shared__ int4 cand[CAND_CAP];
    __shared__ int sorted[SORT_CAP];
    __shared__ int wave_cnt[TILE_THREADS / 64];
    __shared__ int batch_n;

    const int scene = blockIdx.y;
    const SceneDev& S = desc->s[scene];
    const int4* boxes = boxes_all + S.prim_off;
    // this tile's slice of the binned candidates (scene-local ids); count mode
    // sorts it in place, write mode reads it sorted
    const int ntiles = ts.ntx * ts.nty * ts.ntz;
    const int nbin = tile_cnt[(int64_t)scene * ntiles + blockIdx.x];
    const int64_t boff = tile_off[(int64_t)scene * ntiles + blockIdx.x];
    const bool binned = nbin <= SORT_CAP;
    if (binned) {
        for (int i = threadIdx.x; i < nbin; i += blockDim.x) sorted[i] = bin[boff + i];
        __syncthreads();
        if (!WRITE) {
            block_sort(sorted, nbin);
            for (int i = threadIdx.x; i < nbin; i += blockDim.x) bin[boff + i] = sorted[i];
        }
        __syncthreads();
    }
    // the stream of candidates: the sorted slice, or every primitive of the scene
    const int n = binned ? nbin : S.n;
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
        const int idx = base + tid;
        const int k = idx < n ? (binned ? sorted[idx] : idx) : 0;
        int4 b = make_int4(EMPTY_BOX, EMPTY_BOX, EMPTY_BOX, 0);
        if (idx < n) b = boxes[k];
        const bool keep = (idx < n) && box_overlaps(b.x, x0, x1) && box_overlaps(b.y, y0, y1) &&
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

// Most voxel tiles one primitive's box can overlap (its N_v cube spans at most
// 2 N_v + 1 cells per axis).
static int64_t tiles_per_box(const GridDev& g, const TileShape& ts) {
    const int span = 2 * g.nv + 1;
    auto ax = [&](int t, int nt) { return std::min<int64_t>(nt, (span + t - 1) / t + 1); };
    return ax(ts.tx, ts.ntx) * ax(ts.ty, ts.nty) * ax(ts.tz, ts.ntz);
}

// Index scratch: scan partials [S x parts] int64, then the tile binning:
// counts [S x tiles] int, offsets and cursors [S x tiles] int64, candidates
// [total prims x tiles per box] int32.
struct IndexScratch {
    int64_t* partials;
    int* tile_cnt;
    int64_t *tile_off, *tile_cur;
    int32_t* bin;
};
static size_t a256(size_t b) { return (b + 255) / 256 * 256; }
static IndexScratch carve_index(void* base, const GridDev& g, const BatchDesc& d, size_t* bytes) {
    const TileShape ts = pick_tile(g);
    const int64_t nt = (int64_t)d.n_scenes * ts.ntx * ts.nty * ts.ntz;
    const size_t s_p = a256((size_t)d.n_scenes * scan_parts(g) * sizeof(int64_t));
    const size_t s_c = a256((size_t)nt * sizeof(int));
    const size_t s_o = a256((size_t)nt * sizeof(int64_t));
    const size_t s_b = a256((size_t)std::max<int64_t>(1, (int64_t)d.total_prims * tiles_per_box(g, ts)) * sizeof(int32_t));
    if (bytes) *bytes = s_p + s_c + 2 * s_o + s_b;
    IndexScratch x{};
    char* p = (char*)base;
    if (!p) return x;
    x.partials = (int64_t*)p; p += s_p;
    x.tile_cnt = (int*)p; p += s_c;
    x.tile_off = (int64_t*)p; p += s_o;
    x.tile_cur = (int64_t*)p; p += s_o;
    x.bin = (int32_t*)p;
    return x;
}

size_t index_scratch_bytes(const GridDev& g, const BatchDesc& d) {
    size_t b = 0;
    carve_index(nullptr, g, d, &b);
    return b;
}

__global__ __launch_bounds__(256) void k_bin_zero(int* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

void launch_index_kernels(const GridDev& g, const BatchDesc& d, const BatchDesc* desc_dev, const BatchIO& io,
                          int4* boxes, void* scratch, hipStream_t st) {
    const int64_t nvox = (int64_t)g.X * g.Y * g.Z;
    const int np = scan_parts(g);
    const int S = d.n_scenes;
    const IndexScratch x = carve_index(scratch, g, d, nullptr);
    const TileShape ts = pick_tile(g);
    const int ntiles = ts.ntx * ts.nty * ts.ntz;
    const int64_t nbins = (int64_t)S * ntiles;
    hipLaunchKernelGGL(k_bin_zero, dim3((unsigned)std::min<int64_t>((nbins + 255) / 256, 1024)), dim3(256), 0, st,
                       x.tile_cnt, nbins);
    if (d.total_prims > 0) {
        const dim3 pg((d.total_prims + 255) / 256);
        hipLaunchKernelGGL(k_prep_boxes, pg, dim3(256), 0, st, io.means, io.quats, io.scales, io.eps, io.opacity,
                           d.total_prims, g, boxes);
        hipLaunchKernelGGL(k_bin_count, pg, dim3(256), 0, st, desc_dev, (const int4*)boxes, d.total_prims, ts,
                           x.tile_cnt);
    }
    hipLaunchKernelGGL(k_bin_scan, dim3(S), dim3(256), 0, st, desc_dev, (const int*)x.tile_cnt, ntiles,
                       tiles_per_box(g, ts), x.tile_off, x.tile_cur);
    if (d.total_prims > 0)
        hipLaunchKernelGGL(k_bin_fill, dim3((d.total_prims + 255) / 256), dim3(256), 0, st, desc_dev,
                           (const int4*)boxes, d.total_prims, ts, x.tile_cur, x.bin);
    hipLaunchKernelGGL(k_tile_lists<false>, dim3(ntiles, S), dim3(TILE_THREADS), 0, st, desc_dev,
                       (const int4*)boxes, g, ts, io.counts, (const int32_t*)nullptr, (int32_t*)nullptr,
                       (const int*)x.tile_cnt, (const int64_t*)x.tile_off, x.bin);
    hipLaunchKernelGGL(k_scan_partials, dim3(np, S), dim3(SCAN_BLOCK), 0, st, (const int32_t*)io.counts, nvox, np,
                       x.partials);
    hipLaunchKernelGGL(k_scan_top, dim3(S), dim3(SCAN_BLOCK), 0, st, x.partials, np, io.totals);
    hipLaunchKernelGGL(k_scan_final, dim3(np, S), dim3(SCAN_BLOCK), 0, st, (const int32_t*)io.counts, nvox, np,
                       (const int64_t*)x.partials, io.offsets);
    hipLaunchKernelGGL(k_tile_lists<true>, dim3(ntiles, S), dim3(TILE_THREADS), 0, st, desc_dev,
                       (const int4*)boxes, g, ts, io.counts, (const int32_t*)io.offsets, io.ids,
                       (const int*)x.tile_cnt, (const int64_t*)x.tile_off, x.bin);
}

}  // namespace sqr

// Device-side building blocks shared by the gfx950 renderer kernels.
//
// Everything here runs on CDNA4 wavefronts of 64 lanes.  The renderer maps one
// wavefront to a tile of 64 rays; per sample, lanes that fall into the same
// voxel walk that voxel's primitive list together, so the primitive id, its
// prepared record and its logits are wave-uniform and are fetched with scalar
// loads into SGPRs (no LDS traffic, no per-lane gathers).
#pragma once

#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

namespace sqr {

// ---------------------------------------------------------------------------
// Prepared per-primitive record (float[REC]), written by k_prep_records.
//   [0..2]   m                       centre
//   [3..11]  R' = diag(1/s) R(q/|q|)  row-major, so (u,v,w) = R'(x - m)
//   [12]     a = 2/eps2   [13] b = 2/eps1   [14] e = eps2/eps1
//   [15]     sigma
//   [16]     r_cull: max(|u|,|v|,|w|) >= r_cull  =>  f >= F_CULL
//   [17..18] the clipped box of [22..24] in the packed-cell form of box_words
//            (int bits; meaningful on grids within PV_MAX_XY x PV_MAX_XY x PV_MAX_Z)
//   [19..21] a - 1, b - 1 (each FLT_MIN where it is 0), e - 1 (the
//            exponents of the ratios the adjoint evaluates, eval_pair)
//   [22..24] clipped neighbourhood box per axis, int bits lo | hi << 16
//            (the primitive is listed in voxel v iff v lies in this box)
//   [25..27] 1/s
// The forward walks read [0..18], the adjoint [0..21].
// ---------------------------------------------------------------------------
constexpr int R_GLO = 17, R_GHI = 18, R_AM1 = 19, R_BM1 = 20, R_EM1 = 21, R_INVS = 25;
constexpr int REC = 28;
constexpr int EMPTY_BOX = 0x7fff7fff;
constexpr float F_CULL = 110.0f;          // exp(-110) = 1.7e-48: 0 in float32
constexpr float LN2 = 0.6931471805599453f;

// Read-only views in the constant address space.  The kernels store floats
// (checkpoints, atomics) while they read records and logits; through these
// pointers the compiler knows the reads are invariant and keeps wave-uniform
// ones on the scalar path (s_load into SGPRs) instead of vector loads.
typedef const __attribute__((address_space(4))) float* cf_ptr;
typedef const __attribute__((address_space(4))) int* ci_ptr;
__device__ __forceinline__ cf_ptr as_const(const float* p) { return (cf_ptr)p; }
__device__ __forceinline__ ci_ptr as_const(const int* p) { return (ci_ptr)p; }

// Hardware base-2 transcendentals (v_log_f32 / v_exp_f32).
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Pinned float32 discrete decisions: every op correctly rounded, no FMA, so the
// sample depth, the sample point and its voxel match the oracle bit for bit.
// ---------------------------------------------------------------------------
struct GridDev {
    float lox, loy, loz;
    float inv;          // fl(1/voxel), computed on the host
    int X, Y, Z;
    int nv;
    float vs;           // voxel edge length
    float theta;        // influence threshold of the index (0: the N_v cube)
    float fX, fY, fZ;   // X, Y, Z as floats (exact), set on the host: uniform
                        // operands rather than per-lane conversions
};

struct SamplePos {
    float t, x, y, z;
    int v;              // linear voxel id, or -1 outside the grid
    int ix, iy, iz;     // voxel coordinates (valid when v >= 0)
};

__device__ __forceinline__ SamplePos pinned_sample(const GridDev& g, float t_near, float delta, int j,
                                                   float ox, float oy, float oz,
                                                   float dx, float dy, float dz) {
#pragma clang fp contract(off)
    SamplePos s;
    s.t = t_near + (float)j * delta;
    s.x = ox + s.t * dx;
    s.y = oy + s.t * dy;
    s.z = oz + s.t * dz;
    const float qx = (s.x - g.lox) * g.inv;
    const float qy = (s.y - g.loy) * g.inv;
    const float qz = (s.z - g.loz) * g.inv;
    const bool in = (qx >= 0.0f) & (qx < g.fX) & (qy >= 0.0f) & (qy < g.fY) & (qz >= 0.0f) & (qz < g.fZ);
    // q >= 0 here, so truncation is floor
    s.ix = in ? (int)qx : 0;
    s.iy = in ? (int)qy : 0;
    s.iz = in ? (int)qz : 0;
    s.v = in ? ((s.ix * g.Y + s.iy) * g.Z + s.iz) : -1;
    return s;
}

// Sample s lies outside the grid along an axis on which the ray moves away from
// (or parallel to) the grid: every later sample of the ray lies outside too.
// Each step of pinned_sample is a monotone function of j (of t, then of x for
// a fixed sign of d), so a cell coordinate that has left [0, dims) in the
// direction of travel never comes back.  The same op sequence as
// pinned_sample, so the test sees the very q it classified.
__device__ __forceinline__ bool left_grid(const GridDev& g, const SamplePos& s, float dx, float dy, float dz) {
#pragma clang fp contract(off)
    const float qx = (s.x - g.lox) * g.inv;
    const float qy = (s.y - g.loy) * g.inv;
    const float qz = (s.z - g.loz) * g.inv;
    return ((qx >= g.fX) & (dx >= 0.0f)) | ((qx < 0.0f) & (dx <= 0.0f)) |
           ((qy >= g.fY) & (dy >= 0.0f)) | ((qy < 0.0f) & (dy <= 0.0f)) |
           ((qz >= g.fZ) & (dz >= 0.0f)) | ((qz < 0.0f) & (dz <= 0.0f));
}

// Centre of voxel i along one axis in float32, fl(lo + fl(fl(i + 0.5) * voxel))
// with no fused multiply-add (the point the voxelisation evaluates).
__device__ __forceinline__ float pinned_voxel_centre(float lo, float vs, int i) {
#pragma clang fp contract(off)
    const float h = (float)i + 0.5f;
    return lo + h * vs;
}

// Centre voxel of a primitive along one axis, bounded before conversion.
// (The same op sequence as the index build, so boxes agree bit for bit.)
__device__ __forceinline__ int pinned_centre_axis(float m, float lo, float inv, float bound) {
#pragma clang fp contract(off)
    float q = (m - lo) * inv;
    q = fminf(fmaxf(q, -bound), bound);   // NaN -> -bound (covers nothing)
    return (int)floorf(q);
}

// N wave-uniform floats (a primitive's record, its logits) held in SGPRs for
// as long as a walk uses them.  The empty asm makes each value opaque, so the
// compiler keeps it in its register instead of re-issuing the scalar load
// (and waiting for it) at every use, and the loads of one group are issued
// together behind a single wait.  The forward's pair evaluation needs the
// record's first 17 entries, 19 with the packed-cell box words; the adjoint 22.
template <int N>
struct Pinned {
    float v[N];
    __device__ __forceinline__ float operator[](int i) const { return v[i]; }
};
template <int N>
__device__ __forceinline__ Pinned<N> pin(cf_ptr r) {
    Pinned<N> o;
#pragma unroll
    for (int i = 0; i < N; ++i) o.v[i] = r[i];
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+s"(o.v[i]));
    return o;
}
// A group of N wave-uniform floats in flight: for 16 < N < 32 the last 16 as
// one 16-dword tuple.  Loaded element by element, a group's trailing words
// (used last: r_cull, the last logit) end up in single-dword loads that the
// scheduler sinks below the wait for the others, so a visit waits twice;
// inside the tuple they share the load of words used first.
typedef float f32x16_t __attribute__((ext_vector_type(16), aligned(4)));
typedef const __attribute__((address_space(4))) f32x16_t* cf16_ptr;
template <int N>
struct GroupLoad {
    static constexpr bool TUPLE = N > 16 && N < 32;
    static constexpr int H = TUPLE ? N - 16 : N;    // words loaded one by one
    float head[H];
    f32x16_t tail;
    __device__ __forceinline__ void issue(cf_ptr r) {
#pragma unroll
        for (int i = 0; i < H; ++i) head[i] = r[i];
        if constexpr (TUPLE) tail = *(cf16_ptr)(r + H);
    }
    __device__ __forceinline__ void pin(float (&v)[N]) {
        if constexpr (TUPLE) asm volatile("" : "+s"(tail));
#pragma unroll
        for (int i = 0; i < H; ++i) asm volatile("" : "+s"(head[i]));
#pragma unroll
        for (int i = 0; i < H; ++i) v[i] = head[i];
        if constexpr (TUPLE) {
#pragma unroll
            for (int i = 0; i < 16; ++i) v[H + i] = tail[i];
        }
    }
};
// Two groups (a record and the logits): every load issued, then one wait.
template <int N, int M>
__device__ __forceinline__ void pin2(cf_ptr r, Pinned<N>& a, cf_ptr q, Pinned<M>& b) {
    GroupLoad<N> ga;
    GroupLoad<M> gb;
    ga.issue(r);
    gb.issue(q);
    // both tuples in one statement: neither load can sink below the other's wait
    if constexpr (GroupLoad<N>::TUPLE && GroupLoad<M>::TUPLE) asm volatile("" : "+s"(ga.tail), "+s"(gb.tail));
    // a tuple and one word (a record and its last logit): likewise
    if constexpr (GroupLoad<N>::TUPLE && M == 1) asm volatile("" : "+s"(ga.tail), "+s"(gb.head[0]));
    ga.pin(a.v);
    gb.pin(b.v);
}

// One group: a record alone.
template <int N>
__device__ __forceinline__ void pin1(cf_ptr r, Pinned<N>& a) {
    GroupLoad<N> ga;
    ga.issue(r);
    ga.pin(a.v);
}

// ---------------------------------------------------------------------------
// Per-lane class sums s_c += p c_k[c] (Eq. eq:alpha_sem_sq) on the matrix cores
//
// The 16-block 4x4x1 f32 MFMA forms, in every group of four lanes 4b..4b+3,
// D[i][j] += A[i] B[j] with A[i] read from lane 4b+i and B[j] from lane 4b+j,
// and leaves D[i][j] in register i of lane 4b+j.  With B = p (each lane its
// own sample's value) and A = four logits of primitive k spread over the four
// lanes of each group, register i of every lane L gains p_L c_k[class of i]:
// four classes of the whole wave in one instruction instead of four FMAs.
// A visit reads k's logit row with one vector load per group of 4W classes:
// the lane with L % 4 = i reads the W classes that start at 4W G + W i, so
// register i of accumulator (G, q) holds class 4W G + W i + q.  Classes past
// the last full group (the 17th of 17) stay on FMAs with a scalar logit.
// A lane that takes no part in a visit passes p = 0 and adds exact zeros.
// ---------------------------------------------------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <int CP>
struct ClassSums {
    static constexpr int W = CP >= 16 ? 4 : CP >= 8 ? 2 : 1;   // logits a lane loads per group
    static constexpr int NG = CP >= 16 ? CP / 16 : 1;          // groups of 4W classes
    static constexpr int NM = NG * W;                          // accumulators of four classes
    static constexpr int NX = CP - 4 * NM;                     // classes summed by FMAs
    static constexpr int XN = NX > 0 ? NX : 1;
    f32x4_t m[NM];
    float x[XN];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int j = 0; j < NM; ++j) m[j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < XN; ++c) x[c] = 0.0f;
    }
    // class c (a constant once the caller's loop is unrolled)
    __device__ __forceinline__ float get(int c) const {
        if (c >= 4 * NM) return x[c - 4 * NM];
        const int r = c % (4 * W);
        return m[(c / (4 * W)) * W + r % W][r / W];
    }
    // this += w * o, class by class
    __device__ __forceinline__ void add_scaled(float w, const ClassSums& o) {
#pragma unroll
        for (int j = 0; j < NM; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) m[j][i] = fmaf(w, o.m[j][i], m[j][i]);
#pragma unroll
        for (int c = 0; c < NX; ++c) x[c] = fmaf(w, o.x[c], x[c]);
    }
};

// The logit rows of one scene seen through a buffer resource: a visit's
// vector loads take the row's byte offset as their scalar offset.
template <int CP>
struct LogitRows {
    using CS = ClassSums<CP>;
    __amdgpu_buffer_rsrc_t rs;
    uint32_t voff;      // this lane's byte offset inside a group: 4W (L % 4)
    __device__ __forceinline__ LogitRows(cf_ptr lgp, int n, int lane) {
        const uint64_t bytes = (uint64_t)n * CP * sizeof(float);
        rs = __builtin_amdgcn_make_buffer_rsrc((void*)(const float*)lgp, 0, (int)(uint32_t)(bytes < 0xFFFFFFFFull ? bytes : 0xFFFFFFFFull),
                                               0x00020000);
        voff = (uint32_t)(lane & 3) * CS::W * sizeof(float);
    }
    // the groups of primitive k's row, A[G][q] = class 4W G + W (L % 4) + q
    __device__ __forceinline__ void load(int k, float (&A)[CS::NG][CS::W]) const {
        // (unsigned: a row's byte offset reaches 2^32 - 128 at the largest scenes)
        const uint32_t row = (uint32_t)k * (uint32_t)(CP * sizeof(float));
#pragma unroll
        for (int G = 0; G < CS::NG; ++G) {
            const int so = (int)(row + (uint32_t)(G * 4 * CS::W * sizeof(float)));
            if constexpr (CS::W == 4) {
                const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) A[G][q] = __uint_as_float(v[q]);
            } else if constexpr (CS::W == 2) {
                const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, so, 0);
                A[G][0] = __uint_as_float(v[0]);
                A[G][1] = __uint_as_float(v[1]);
            } else {
                A[G][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, so, 0));
            }
        }
    }
};

// s += p * c_k over the wave (every lane active; p = 0 where a lane adds nothing)
template <int CP>
__device__ __forceinline__ void class_mfma(ClassSums<CP>& s, const float (&A)[ClassSums<CP>::NG][ClassSums<CP>::W],
                                           float p) {
    using CS = ClassSums<CP>;
#pragma unroll
    for (int G = 0; G < CS::NG; ++G)
#pragma unroll
        for (int q = 0; q < CS::W; ++q)
            s.m[G * CS::W + q] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[G][q], p, s.m[G * CS::W + q], 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Pair evaluation p_o(x, S_k) = exp(-f(R(x - m)/s)) (Eq. eq:sq_occupancy_prob).
// ---------------------------------------------------------------------------
// log2(1 / ln 2): 2^(x + L2_LOG2E) = 2^x / ln 2
constexpr float L2_LOG2E = 0.5287663729448977f;

// 0 * anything = 0 (v_mul_legacy_f32): the products below whose first factor
// vanishes exactly where the second is infinite (a power times the log or the
// reciprocal of its base) take their limit, 0, with no compare or select.
extern "C" __device__ float sqr_fmul_legacy(float, float) __asm("llvm.amdgcn.fmul.legacy");
__device__ __forceinline__ float mul0(float zero_wins, float x) { return sqr_fmul_legacy(zero_wins, x); }
// |q| with the sign of x (q >= 0)
__device__ __forceinline__ float with_sign_of(float q, float x) {
    return __uint_as_float(__float_as_uint(q) | (__float_as_uint(x) & 0x80000000u));
}

// The sum A = |u|^a + |v|^a is formed in the log domain.  Its terms
// underflow float32 long before the power B = A^e (e = eps2/eps1) becomes
// negligible: at eps2 = 0.1 (a = 20) |u|^a is 0 below |u| = 0.006 while
// A^e ~ max(|u|, |v|)^(2/eps1) is still of order |u| when eps1 is near 2, and
// at the far end of the cull box |u|^a overflows where A^e is still finite.
// With l_m = max(log2|u|, log2|v|) and d = min(log2|u|, log2|v|) - l_m <= 0,
//   log2 A = a l_m + log2(1 + 2^(a d)),     log2 B = b l_m + e log2(1 + 2^(a d))
// (b = a e), which stays finite and exact to rounding at any scale.  l_m is
// floored at -LOG_FLOOR so that u = v = 0 (a sample on the primitive's third
// axis) gives d = -inf and a finite, vanishing B instead of -inf - -inf.
constexpr float LOG_FLOOR = 256.0f;

// Evaluation for the adjoint.  Besides p it keeps the ratios the derivative
// chain needs, each as one power of two with no reciprocal, and all of them
// (with B and Z) divided by ln 2 through the exponent, like eval_p's:
//   r_u = (B/A) |u|^a / |u| / ln2 = 2^((e-1) log2 A + (a-1) log2|u| + log2(1/ln2)),
//   r_v likewise, q_w = |w|^(b-1) / ln2, Z = q_w |w|, and B = A^e / ln2 as
// r_u |u| + r_v |v| = (B/A)(X + Y) / ln2 (no power of its own), so
// p = 2^-(B + Z) takes no multiply; k_finalize puts ln 2 back into the
// factors (acc_factor).  p agrees with eval_p's to rounding (not bit for
// bit).  At a base that is exactly 0 (a sample on a principal plane) its log
// is -inf.  The record stores a - 1 and b - 1 as FLT_MIN where they are 0
// (eps = 2), so (a-1) log2|u| is -inf there too and r_u = 0, the symmetric
// subgradient of |u| at its kink, with a plain FMA (likewise q_w).  So r_u,
// r_v and q_w stay finite for a, b >= 1 (eps1, eps2 <= 2, the paper's
// parameter range); log2 A is finite by the floor above.  Inside the cull box
// every field is finite.
// Returns false when the pair is culled (float32 exp(-f) would be exactly 0).
struct PairEval {
    float u, v, w;         // canonical coordinates x_S / s
    float lu, lv, lw;      // log2 |u|, log2 |v|, log2 |w|
    float ru, rv, qw;      // (B/A) X/|u|, (B/A) Y/|v|, |w|^(b-1), each / ln 2
    float Xb, Yb;          // r_u |u| = (B/A) X / ln 2, r_v |v| = (B/A) Y / ln 2
    float lA, B, Z;        // log2 A, A^e / ln 2 = Xb + Yb, |w|^b / ln 2
    float p;
};

constexpr float LOG2E = 1.4426950408889634f;

template <typename RecT>
__device__ __forceinline__ bool eval_pair(const RecT& rec, float x, float y, float z,
                                          float dxyz[3], PairEval& e) {
    const float dx = x - rec[0], dy = y - rec[1], dz = z - rec[2];
    dxyz[0] = dx; dxyz[1] = dy; dxyz[2] = dz;
    e.u = fmaf(rec[3], dx, fmaf(rec[4], dy, rec[5] * dz));
    e.v = fmaf(rec[6], dx, fmaf(rec[7], dy, rec[8] * dz));
    e.w = fmaf(rec[9], dx, fmaf(rec[10], dy, rec[11] * dz));
    const float au = fabsf(e.u), av = fabsf(e.v), aw = fabsf(e.w);
    const float mx = fmaxf(fmaxf(au, av), aw);
    if (!(mx < rec[16])) return false;
    e.lu = hw_log2(au);
    e.lv = hw_log2(av);
    e.lw = hw_log2(aw);
    const float lm = fmaxf(fmaxf(e.lu, e.lv), -LOG_FLOOR);
    const float d = fminf(e.lu, e.lv) - lm;
    e.lA = fmaf(rec[12], lm, hw_log2(1.0f + hw_exp2(rec[12] * d)));
    const float c = fmaf(rec[R_EM1], e.lA, L2_LOG2E);  // log2(B/A / ln 2)
    e.ru = hw_exp2(fmaf(rec[R_AM1], e.lu, c));
    e.rv = hw_exp2(fmaf(rec[R_AM1], e.lv, c));
    e.Xb = e.ru * au;
    e.Yb = e.rv * av;
    e.B = e.Xb + e.Yb;
    e.qw = hw_exp2(fmaf(rec[R_BM1], e.lw, L2_LOG2E));
    e.Z = e.qw * aw;
    e.p = hw_exp2(-(e.B + e.Z));
    return true;
}

// Cull test alone (used by the counting variants of the kernels).
__device__ __forceinline__ bool pair_kept(cf_ptr rec, float x, float y, float z) {
    const float dx = x - rec[0], dy = y - rec[1], dz = z - rec[2];
    const float u = fmaf(rec[3], dx, fmaf(rec[4], dy, rec[5] * dz));
    const float v = fmaf(rec[6], dx, fmaf(rec[7], dy, rec[8] * dz));
    const float w = fmaf(rec[9], dx, fmaf(rec[10], dy, rec[11] * dz));
    return fmaxf(fmaxf(fabsf(u), fabsf(v)), fabsf(w)) < rec[16];
}

// Evaluation of p alone (0 when culled): B and Z divided by ln 2 through the
// exponent, so p = 2^-(Bs + Zs) takes no multiply; B in the log form above.
// The forward, the backward's recompute and the voxelisation all call this,
// so they agree bit for bit.
// eval_p_kept: false for a culled pair (p untouched), else p.
template <typename RecT>
__device__ __forceinline__ bool eval_p_kept(const RecT& rec, float x, float y, float z, float& p) {
    const float dx = x - rec[0], dy = y - rec[1], dz = z - rec[2];
    const float u = fmaf(rec[3], dx, fmaf(rec[4], dy, rec[5] * dz));
    const float v = fmaf(rec[6], dx, fmaf(rec[7], dy, rec[8] * dz));
    const float w = fmaf(rec[9], dx, fmaf(rec[10], dy, rec[11] * dz));
    const float au = fabsf(u), av = fabsf(v), aw = fabsf(w);
    const float mx = fmaxf(fmaxf(au, av), aw);
    if (!(mx < rec[16])) return false;
    const float a = rec[12], b = rec[13], ee = rec[14];
    const float lu = hw_log2(au), lv = hw_log2(av);
    const float lm = fmaxf(fmaxf(lu, lv), -LOG_FLOOR);
    const float d = fminf(lu, lv) - lm;
    const float l1 = hw_log2(1.0f + hw_exp2(a * d));
    const float Zs = hw_exp2(fmaf(b, hw_log2(aw), L2_LOG2E));
    const float Bs = hw_exp2(fmaf(ee, l1, fmaf(b, lm, L2_LOG2E)));
    p = hw_exp2(-(Bs + Zs));
    return true;
}
template <typename RecT>
__device__ __forceinline__ float eval_p(const RecT& rec, float x, float y, float z) {
    float p = 0.0f;
    eval_p_kept(rec, x, y, z, p);
    return p;
}

// ---------------------------------------------------------------------------
// Wavefront helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Sum over the 64 lanes of a wavefront (butterfly; a fixed order, so the
// result does not depend on scheduling).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Order the LDS accesses of one wavefront (LDS is private to the wave here).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_QUAD_SWAP2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_QUAD_SWAP1 = 0xB1;   // quad_perm [1,0,3,2]

// Sum VP (16, 32 or 64) values over the 64 lanes of a wavefront with a
// transposing butterfly: at each level a lane keeps half of its values and
// adds its partner's partial sums of that half.  Levels use
// v_permlane32_swap, v_permlane16_swap, DPP row_mirror, row_half_mirror and
// two quad permutes, so no LDS is touched; once one value is left, the
// remaining levels are plain sums over the quad.  On return lane l holds the
// total of value index l >> (6 - log2 VP).  All 64 lanes must be active.
template <int VP>
__device__ __forceinline__ float transpose_reduce(float (&x)[VP], int lane) {
    static_assert(VP == 16 || VP == 32 || VP == 64, "VP must be 16, 32 or 64");
    constexpr int h1 = VP / 2, h2 = h1 / 2, h3 = h2 / 2, h4 = h3 / 2, h5 = h4 / 2;
#pragma unroll
    for (int i = 0; i < h1; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[h1 + i]),
                                                        false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < h2; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[h2 + i]),
                                                        false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const auto sel = [lane](int bit, float hi, float lo) {
        uint32_t m = 0u - (((uint32_t)lane >> bit) & 1u);
        asm("" : "+v"(m));
        return __uint_as_float((__float_as_uint(hi) & m) | (__float_as_uint(lo) & ~m));
    };
#pragma unroll
    for (int i = 0; i < h3; ++i) {
        const float lo = x[i] + dpp_f<DPP_ROW_MIRROR>(x[i]);
        const float hi = x[h3 + i] + dpp_f<DPP_ROW_MIRROR>(x[h3 + i]);
        x[i] = sel(3, hi, lo);
    }
#pragma unroll
    for (int i = 0; i < h4; ++i) {
        const float lo = x[i] + dpp_f<DPP_ROW_HALF_MIRROR>(x[i]);
        const float hi = x[h4 + i] + dpp_f<DPP_ROW_HALF_MIRROR>(x[h4 + i]);
        x[i] = sel(2, hi, lo);
    }
    if constexpr (VP == 16) {
        const float t = x[0] + dpp_f<DPP_QUAD_SWAP2>(x[0]);
        return t + dpp_f<DPP_QUAD_SWAP1>(t);
    } else {
#pragma unroll
        for (int i = 0; i < h5; ++i) {
            const float lo = x[i] + dpp_f<DPP_QUAD_SWAP2>(x[i]);
            const float hi = x[h5 + i] + dpp_f<DPP_QUAD_SWAP2>(x[h5 + i]);
            x[i] = sel(1, hi, lo);
        }
        if constexpr (VP == 64) {
            const float lo = x[0] + dpp_f<DPP_QUAD_SWAP1>(x[0]);
            const float hi = x[1] + dpp_f<DPP_QUAD_SWAP1>(x[1]);
            return sel(0, hi, lo);
        } else {
            return x[0] + dpp_f<DPP_QUAD_SWAP1>(x[0]);
        }
    }
}

// The 16-value transposing reduction with the lane-bit selects given as
// vector masks computed once by the caller (m3, m2: all ones where lane bit 3,
// respectively 2, is set), so that no mask is rebuilt or copied per call.
// Same levels and summation order as transpose_reduce<16>.
__device__ __forceinline__ float transpose_reduce16(float (&x)[16], uint32_t m3, uint32_t m2) {
    const auto sel = [](uint32_t m, float hi, float lo) {
        float r;    // one bitfield insert: (hi & m) | (lo & ~m)
        asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(hi), "v"(lo));
        return r;
    };
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[8 + i]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[4 + i]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float lo = x[i] + dpp_f<DPP_ROW_MIRROR>(x[i]);
        const float hi = x[2 + i] + dpp_f<DPP_ROW_MIRROR>(x[2 + i]);
        x[i] = sel(m3, hi, lo);
    }
    {
        const float lo = x[0] + dpp_f<DPP_ROW_HALF_MIRROR>(x[0]);
        const float hi = x[1] + dpp_f<DPP_ROW_HALF_MIRROR>(x[1]);
        x[0] = sel(m2, hi, lo);
    }
    const float t = x[0] + dpp_f<DPP_QUAD_SWAP2>(x[0]);
    return t + dpp_f<DPP_QUAD_SWAP1>(t);
}

// Sum of v over the four 16-lane rows, through the LDS crossbar (no vector ALU
// move or swap): a swizzle that exchanges 16-lane halves of each 32-lane group,
// then a permute across the 32-lane halves (bp32: this lane's byte address of
// lane ^ 32).  Every lane gets the total of its position in the row; the sum
// is (v_l + v_l^16) + (v_l^32 + v_l^48).
__device__ __forceinline__ float row_sum4_lds(float v, int bp32) {
    const float s = v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    return s + __int_as_float(__builtin_amdgcn_ds_bpermute(bp32, __float_as_int(s)));
}

// Sum of v over the four 16-lane rows: every lane gets the total of its
// position in the row (v_permlane32_swap, v_permlane16_swap).
__device__ __forceinline__ float row_sum4(float v) {
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// works on one contiguous range of logical blocks (neighbouring ray tiles share
// voxel lists and primitive records in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return (xcd < rem) ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Clipped box of a primitive, packed lo | hi << 16 per axis.  An empty box is
// stored as lo = hi = 0x7fff on every axis: no voxel index reaches 0x7fff
// (dims <= 32767), so every containment / overlap test fails.
//
// With an influence threshold theta > 0 the N_v cube is further clipped to the
// voxels meeting the world box of max(|u|,|v|,|w|) <= r = ln(sigma/theta)^(eps1/2)
// (x - m = R^T diag(s) u, so its half-extent along axis a is
// r (|R_0a| s_0 + |R_1a| s_1 + |R_2a| s_2)); empty where sigma <= theta.  That
// part runs in FP64 with a fixed operation order and no contraction, so the
// index build and the render's record preparation, which both call this
// function on the same inputs, get the same box.
__device__ __forceinline__ int clamp_cell(double c, int big) {
    if (!(c >= -(double)big)) return -big;      // also NaN
    if (c > (double)big) return big;
    return (int)c;
}
// q, s, eps, sigma point at the primitive's quaternion, scales, (eps1, eps2)
// and opacity; they are read only when theta > 0.
__device__ __forceinline__ void prim_box(const GridDev& g, const float* m, const float* q, const float* s,
                                         const float* eps, const float* sigma, int out[3]) {
    const int dims[3] = {g.X, g.Y, g.Z};
    const float lo[3] = {g.lox, g.loy, g.loz};
    const float bound = (float)(max(max(g.X, g.Y), g.Z) + g.nv + 2);
    int blo[3], bhi[3];
    bool empty = false;
    for (int ax = 0; ax < 3; ++ax) {
        const int c = pinned_centre_axis(m[ax], lo[ax], g.inv, bound);
        blo[ax] = max(c - g.nv, 0);
        bhi[ax] = min(c + g.nv, dims[ax] - 1);
    }
    if (g.theta > 0.0f) {
#pragma clang fp contract(off)
        const double th = (double)g.theta, sg = (double)sigma[0];
        if (!(sg > th)) {
            empty = true;
        } else {
            double w = q[0], x = q[1], y = q[2], z = q[3];
            const double nrm = sqrt(w * w + x * x + y * y + z * z);
            w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
            const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                                 2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                                 2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
            const double r = exp(0.5 * (double)eps[0] * log(log(sg / th)));
            const double vs = (double)g.vs;
            const int big = max(max(g.X, g.Y), g.Z) + g.nv + 2;
            for (int ax = 0; ax < 3; ++ax) {
                const double h = r * (fabs(R[ax]) * (double)s[0] + fabs(R[3 + ax]) * (double)s[1] +
                                      fabs(R[6 + ax]) * (double)s[2]);
                const double mm = (double)m[ax], l = (double)lo[ax];
                const int slo = clamp_cell(floor(((mm - h) - l) / vs), big);
                const int shi = clamp_cell(floor(((mm + h) - l) / vs), big);
                blo[ax] = max(blo[ax], slo);
                bhi[ax] = min(bhi[ax], shi);
            }
        }
    }
    for (int ax = 0; ax < 3; ++ax) {
        if (blo[ax] > bhi[ax]) empty = true;
        out[ax] = (blo[ax] & 0xffff) | (bhi[ax] << 16);
    }
    if (empty) out[0] = out[1] = out[2] = EMPTY_BOX;
}

// lo <= i <= hi for a packed axis range (one subtract, one unsigned compare)
__device__ __forceinline__ bool in_range(int i, int packed) {
    const int lo = packed & 0xffff, hi = packed >> 16;
    return (unsigned)(i - lo) <= (unsigned)(hi - lo);
}

// Voxel cells packed into one word, x | y << 11 | z << 22, with a guard bit
// above each field (bits 10, 21, 31).  The three-axis box test then takes two
// additions and one three-input bit operation: for a cell word c with clear
// guards,
//   c + (G - lo)       keeps a field's guard bit set exactly when c_f >= lo_f,
//   c + (G - (hi + 1)) sets it exactly when c_f > hi_f,
// and no carry crosses a guard or leaves the word.  Grids up to PV_MAX_XY x
// PV_MAX_XY x PV_MAX_Z cells fit; PV_DEAD (every field at its maximum, above any
// cell of such a grid) lies in no box.  Two cells packed in 64 bits are tested
// with two 64-bit additions (in_box2): neither half carries into the other.
constexpr uint32_t PV_GUARDS = (1u << 10) | (1u << 21) | (1u << 31);
constexpr uint32_t PV_ONES = 1u | (1u << 11) | (1u << 22);
constexpr int PV_MAX_XY = 1023, PV_MAX_Z = 511;
constexpr uint32_t PV_DEAD = 0x3ffu | (0x3ffu << 11) | (0x1ffu << 22);

__device__ __forceinline__ uint32_t pack_cell(int ix, int iy, int iz) {
    return (uint32_t)ix | ((uint32_t)iy << 11) | ((uint32_t)iz << 22);
}
// The record words of a per-axis box (prim_box's output): G - lo and
// G - (hi + 1).  An empty box gets lo above hi in every field, which no cell
// satisfies.
__device__ __forceinline__ void box_words(const int box[3], uint32_t& glo, uint32_t& ghi) {
    int lo[3], hi[3];
    bool empty = false;
    const int cap[3] = {PV_MAX_XY, PV_MAX_XY, PV_MAX_Z};
    for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = box[ax] & 0xffff;
        hi[ax] = box[ax] >> 16;
        empty |= box[ax] == EMPTY_BOX || lo[ax] > hi[ax] || hi[ax] >= cap[ax];
    }
    const uint32_t plo = empty ? PV_DEAD : pack_cell(lo[0], lo[1], lo[2]);
    const uint32_t phi = empty ? 0u : pack_cell(hi[0], hi[1], hi[2]);
    glo = PV_GUARDS - plo;
    ghi = PV_GUARDS - (phi + PV_ONES);
}
// Guards of a = c + glo all set and of b = c + ghi all clear.
__device__ __forceinline__ bool box_guards(uint32_t a, uint32_t b) {
    return (a & ~b & PV_GUARDS) == PV_GUARDS;
}
// Cell word c (guards clear) inside the box of record words glo, ghi?
__device__ __forceinline__ bool in_box(uint32_t c, uint32_t glo, uint32_t ghi) {
    return box_guards(c + glo, c + ghi);
}
// Two cells c2 = c0 | c1 << 32 against one box (glo2 = glo | glo << 32, and
// likewise ghi2).
__device__ __forceinline__ void in_box2(uint64_t c2, uint64_t glo2, uint64_t ghi2, bool& m0, bool& m1) {
    // one 64-bit add each (left to itself the compiler splits them into a
    // 64-bit multiply-add and a 32-bit add)
    uint64_t a, b;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(a) : "v"(c2), "s"(glo2));
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(b) : "v"(c2), "s"(ghi2));
    m0 = box_guards((uint32_t)a, (uint32_t)b);
    m1 = box_guards((uint32_t)(a >> 32), (uint32_t)(b >> 32));
}
// K packed cells held in pairs (K even); get/set take a constant index once the
// caller's loop is unrolled.
template <int K>
struct CellPairs {
    uint64_t w[K / 2];
    __device__ __forceinline__ uint32_t get(int j) const { return (uint32_t)(w[j >> 1] >> (32 * (j & 1))); }
    __device__ __forceinline__ void set(int j, uint32_t c) {
        const int sh = 32 * (j & 1);
        w[j >> 1] = (w[j >> 1] & ~(0xffffffffull << sh)) | ((uint64_t)c << sh);
    }
    // mem[j]: cell j inside the box of record words glo, ghi
    __device__ __forceinline__ void members(uint32_t glo, uint32_t ghi, bool (&mem)[K]) const {
        const uint64_t glo2 = glo | ((uint64_t)glo << 32), ghi2 = ghi | ((uint64_t)ghi << 32);
#pragma unroll
        for (int i = 0; i < K / 2; ++i) in_box2(w[i], glo2, ghi2, mem[2 * i], mem[2 * i + 1]);
    }
};

}  // namespace sqr

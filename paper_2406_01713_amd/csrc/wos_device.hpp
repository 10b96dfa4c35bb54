// wos_device.hpp -- device building blocks of the Walk-on-Spheres walk kernels
// for gfx950: counter-based Philox random numbers, uniform directions on the
// sphere, the distance-to-boundary loop over wave-uniform obstacle tables,
// closest points and boundary data, the screening-weight series and one walk
// iteration.  Internal to libwos.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wos_params.hpp"

namespace wos {

// Read-only tables are accessed through the constant address space: with a
// wave-uniform index the compiler turns every read into a scalar load (one
// fetch per wave through the scalar cache, operands in SGPRs).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> to_const(const T* p)
{
    return (cptr<T>)p;
}

// An empty asm that claims to rewrite a scalar value.  Placed right before a
// use, it stops the compiler from hoisting the loads (or key schedule) that
// depend on the value out of the walk loop and pinning them in scalar
// registers for the whole loop; they are re-read from the scalar cache
// instead, which keeps the hot obstacle loop free of scalar-register spills.
template <typename T>
__device__ __forceinline__ cptr<T> fresh(cptr<T> p)
{
    asm volatile("" : "+s"(p));
    return p;
}

__device__ __forceinline__ uint32_t fresh(uint32_t v)
{
    asm volatile("" : "+s"(v));
    return v;
}

template <typename T>
using cenv = cptr<EnvP<T>>;

// ------------------------------------------------------------------------
// Precision-specific math.  FP32 uses the hardware instructions directly
// (v_sqrt_f32, v_rcp_f32, v_rsq_f32, v_log_f32 = log2, v_sin/v_cos_f32 whose
// argument is in turns); FP64 uses the device math library.
// ------------------------------------------------------------------------
template <typename T>
struct Math;

template <>
struct Math<float> {
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float min(float a, float b) { return __builtin_fminf(a, b); }
    static __device__ __forceinline__ float max(float a, float b) { return __builtin_fmaxf(a, b); }
    static __device__ __forceinline__ float abs(float a) { return __builtin_fabsf(a); }
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
    static __device__ __forceinline__ float log(float x) { return __logf(x); }
    static __device__ __forceinline__ float pow(float x, float y) { return __expf(y * __logf(x)); }
    // sin and cos of x radians: x in turns, reduced to [-1/2, 1/2], on the
    // hardware sine and cosine (no wide-range reduction code)
    static __device__ __forceinline__ void sincos(float x, float& s, float& c)
    {
        float t = x * 0.15915494309189535f;
        t -= __builtin_rintf(t);
        s = __builtin_amdgcn_sinf(t);
        c = __builtin_amdgcn_cosf(t);
    }
    // Box-Muller radius sqrt(-2 ln u) with ln u = ln 2 * log2 u
    static __device__ __forceinline__ float bm_radius(float u)
    {
        return __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u));
    }
    // sin and cos of 2 pi t
    static __device__ __forceinline__ void sincos_turns(float t, float& s, float& c)
    {
        s = __builtin_amdgcn_sinf(t);
        c = __builtin_amdgcn_cosf(t);
    }
    // (2 (x >> 9) + 1) 2^-24: the bits 0x3F800000 | (x >> 9) (one v_alignbit
    // of 0x7F:x) are 1 + (x >> 9) 2^-23, and subtracting 1 - 2^-24 is exact
    // (Sterbenz: both lie in [1/2, 2])
    static __device__ __forceinline__ float uniform(uint32_t x)
    {
        return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
    }
};

template <>
struct Math<double> {
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double min(double a, double b) { return __builtin_fmin(a, b); }
    static __device__ __forceinline__ double max(double a, double b) { return __builtin_fmax(a, b); }
    static __device__ __forceinline__ double abs(double a) { return __builtin_fabs(a); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double pow(double x, double y) { return ::pow(x, y); }
    static __device__ __forceinline__ void sincos(double x, double& s, double& c) { ::sincos(x, &s, &c); }
    static __device__ __forceinline__ double bm_radius(double u) { return ::sqrt(-2.0 * ::log(u)); }
    static __device__ __forceinline__ void sincos_turns(double t, double& s, double& c)
    {
        ::sincospi(2.0 * t, &s, &c);
    }
    static __device__ __forceinline__ double uniform(uint32_t x)
    {
        return (double)(2u * (x >> 9) + 1u) * 0x1p-24;
    }
};

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products on words 0 and 2, word swap and xor with the round
// key; the key is bumped by the Weyl constants after each round.  The key is
// wave-uniform, so its schedule stays in scalar registers.
// ------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64-bit product per word (v_mad_u64_u32) gives both
        // halves; each three-way xor is one v_bitop3_b32 (truth table 0x96)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = y0;
        c1 = (uint32_t)p1;
        c2 = y2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform direction on S^{D-1} for step k of walk (w, q, env) (Sec. IV: the
// next point is uniform on the sphere of the largest empty ball).  Block j of
// the step uses counter (2k + j, w, q, env); Box-Muller pair p uses words
// 2p, 2p + 1; the normal vector is scaled to unit length.
template <typename T, int D>
__device__ __forceinline__ void direction(uint32_t k, uint32_t w, uint32_t q, uint32_t env,
                                          uint32_t key0, uint32_t key1, T (&v)[D])
{
    constexpr int NP = (D + 1) / 2;
    constexpr int NB = (NP + 1) / 2;
    uint32_t words[4 * NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        uint32_t c0 = 2u * k + (uint32_t)j, c1 = w, c2 = q, c3 = env;
        philox4x32_10(c0, c1, c2, c3, fresh(key0), fresh(key1));
        words[4 * j + 0] = c0;
        words[4 * j + 1] = c1;
        words[4 * j + 2] = c2;
        words[4 * j + 3] = c3;
    }
    T n[2 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const T rho = Math<T>::bm_radius(Math<T>::uniform(words[2 * p]));
        T s, c;
        Math<T>::sincos_turns(Math<T>::uniform(words[2 * p + 1]), s, c);
        n[2 * p] = rho * c;
        n[2 * p + 1] = rho * s;
    }
    T n2 = n[0] * n[0];
#pragma unroll
    for (int i = 1; i < D; ++i) n2 = Math<T>::fma(n[i], n[i], n2);
    const T inv = Math<T>::rsqrt(n2);
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = n[i] * inv;
}

// ------------------------------------------------------------------------
// Distance to the boundary (Sec. V).  The obstacle loops are the hot loop of
// the method: every walk step scans all obstacles of its environment.
// ------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ T sq_dist(const T (&x)[D], cptr<T> c)
{
    T t = x[0] - c[0];
    T acc = t * t;
#pragma unroll
    for (int i = 1; i < D; ++i) {
        t = x[i] - c[i];
        acc = Math<T>::fma(t, t, acc);
    }
    return acc;
}

template <typename T, int D>
__device__ __forceinline__ T sphere_dist(const T (&x)[D], cptr<T> row)
{
    return Math<T>::sqrt(sq_dist<T, D>(x, row)) - row[D];
}

template <typename T, int D>
__device__ __forceinline__ T box_dist(const T (&x)[D], cptr<T> row)
{
    // signed distance: |max(q, 0)| + min(max_i q_i, 0), q = |x - c| - h
    T out2 = 0, inside = -Math<T>::inf();
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const T q = Math<T>::abs(x[i] - row[i]) - row[D + i];
        const T qp = Math<T>::max(q, T(0));
        out2 = Math<T>::fma(qp, qp, out2);
        inside = Math<T>::max(inside, q);
    }
    return Math<T>::sqrt(out2) + Math<T>::min(inside, T(0));
}

#ifndef WOS_SPHERE_UNROLL
#define WOS_SPHERE_UNROLL 8
#endif

template <typename T, int D>
__device__ __forceinline__ T spheres_min(cptr<T> sph, int n, const T (&x)[D])
{
    constexpr int S = sph_stride(D);
    T best = Math<T>::inf();
#pragma unroll WOS_SPHERE_UNROLL
    for (int j = 0; j < n; ++j) best = Math<T>::min(best, sphere_dist<T, D>(x, sph + j * S));
    return best;
}

template <typename T, int D>
__device__ __forceinline__ T boxes_min(cptr<T> box, int n, const T (&x)[D])
{
    constexpr int S = box_stride(D);
    T best = Math<T>::inf();
#pragma unroll 2
    for (int j = 0; j < n; ++j) best = Math<T>::min(best, box_dist<T, D>(x, box + j * S));
    return best;
}

template <typename T, int D>
__device__ __forceinline__ T outer_dist(cenv<T> p, const T (&x)[D])
{
    if (p->outer_kind == 0) {
        T m = Math<T>::min(x[0] - p->lo[0], p->hi[0] - x[0]);
#pragma unroll
        for (int i = 1; i < D; ++i) m = Math<T>::min(m, Math<T>::min(x[i] - p->lo[i], p->hi[i] - x[i]));
        return m;
    }
    T t = x[0] - p->oc[0];
    T acc = t * t;
#pragma unroll
    for (int i = 1; i < D; ++i) {
        t = x[i] - p->oc[i];
        acc = Math<T>::fma(t, t, acc);
    }
    return p->orad - Math<T>::sqrt(acc);
}

// ------------------------------------------------------------------------
// Cluster culling.  For a cluster with bounding sphere (C, rho), every member
// distance (sphere: |x - c_j| - r_j; box SDF, which is at least
// |x - c_j| - |h_j|) is, in exact arithmetic, at least |x - C| - rho when
// rho >= |c_j - C| + r_j (or + |h_j|).  The computed bound
//     lb = |x - C| (1 - m) - rho',   rho' = rho (1 + 2m) rounded up,
// with m = 2^-16 (FP32) or 2^-45 (FP64), i.e. 256 units of rounding, is below
// the computed member distance by more than every rounding error of either
// value (each a few units relative to |x - C| + 2 rho).  So lb > t proves that
// every member's computed distance exceeds t.
// ------------------------------------------------------------------------
template <typename T>
struct Cull;
template <>
struct Cull<float> {
    static constexpr float shrink = 1.0f - 0x1p-16f;
};
template <>
struct Cull<double> {
    static constexpr double shrink = 1.0 - 0x1p-45;
};

template <typename T, int D>
__device__ __forceinline__ T cluster_bound(const T (&x)[D], cptr<T> b)
{
    return Math<T>::fma(Math<T>::sqrt(sq_dist<T, D>(x, b)), Cull<T>::shrink, -b[D]);
}

template <typename T, int D, bool BOX>
__device__ __forceinline__ T cluster_members_min(const T (&x)[D], cptr<T> r, T best)
{
    constexpr int S = BOX ? box_stride(D) : sph_stride(D);
#pragma unroll
    for (int j = 0; j < kCluster; ++j)
        best = Math<T>::min(best, BOX ? box_dist<T, D>(x, r + j * S) : sphere_dist<T, D>(x, r + j * S));
    return best;
}

// Min over the members of the clusters that some active lane of the wave may
// need: a cluster is evaluated (all kCluster rows, for every active lane) unless
// its bound exceeds thr or the running min on every active lane.  thr
// is a distance this lane's result cannot exceed (the goal, outer and box
// distances already computed), so a skipped member is never the minimum and
// never ties it.  Bounds are taken two clusters at a time (the second against
// the running min before the first cluster's members, which only culls
// less); the bound table's spare row stands in for a missing second cluster.
// NaN bounds never cull.  Lanes with live false (idle lanes that run along)
// never demand a cluster.  n_eval (wave-uniform) counts the member distances
// each lane evaluated.
template <typename T, int D, bool BOX>
__device__ __forceinline__ T cluster_min(cptr<T> rows, cptr<T> bnd, int n_cl, const T (&x)[D], T thr,
                                         bool live, uint32_t& n_eval)
{
    constexpr int S = BOX ? box_stride(D) : sph_stride(D);
    constexpr int SB = sph_stride(D);
    T best = Math<T>::inf();
    for (int g = 0; g < n_cl; g += 2) {
        const T lb0 = cluster_bound<T, D>(x, bnd + g * SB);
        const T lb1 = cluster_bound<T, D>(x, bnd + (g + 1) * SB);
        const bool need1 = live && !(lb1 > thr || lb1 > best);
        if (__ballot(live && !(lb0 > thr || lb0 > best)) != 0) {  // wave-uniform
            best = cluster_members_min<T, D, BOX>(x, rows + g * (kCluster * S), best);
            n_eval += kCluster;
        }
        if (g + 1 < n_cl && __ballot(need1) != 0) {
            best = cluster_members_min<T, D, BOX>(x, rows + (g + 1) * (kCluster * S), best);
            n_eval += kCluster;
        }
    }
    return best;
}

// ------------------------------------------------------------------------
// Cluster test on the matrix cores (FP32).  The walker and cluster feature
// vectors (see kMfmaTile) make the test a 12-term dot product per (walker,
// cluster) pair: three v_mfma_f32_16x16x4f32 per tile of 16 walkers x 16
// clusters.  Requires every lane of the wave to be active (the callers step
// all lanes); lanes with live false get a huge feature 8 and never demand a
// cluster.
// ------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));

// Walker features transposed into the A operands: A[s][t] is the operand of
// K-step s (features 4s..4s+3) for the row tile of walkers 16t..16t+15; lane
// 16h + i holds feature 4s + h of walker 16t + i.  Two permlane16 swaps then
// two permlane32 swaps transpose (feature, 16-lane row) blocks.
template <int D>
__device__ __forceinline__ void mfma_walker_operands(const float (&x)[D], float thr, bool live, float (&A)[3][4])
{
    float f[kMfmaFeat];
    float xx = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        f[i] = i < D ? x[i < D ? i : 0] : 0.0f;
        if (i < D) xx = __builtin_fmaf(f[i], f[i], xx);
    }
    const float m = 0x1p-12f;
    f[8] = live ? __builtin_fmaf(xx, 1.0f - m, -m * thr * thr) : 1e30f;
    f[9] = 1.0f;
    f[10] = thr * thr;
    f[11] = thr;
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        unsigned r0 = __float_as_uint(f[4 * st]), r1 = __float_as_uint(f[4 * st + 1]);
        unsigned r2 = __float_as_uint(f[4 * st + 2]), r3 = __float_as_uint(f[4 * st + 3]);
        const auto p01 = __builtin_amdgcn_permlane16_swap(r0, r1, false, false);
        const auto p23 = __builtin_amdgcn_permlane16_swap(r2, r3, false, false);
        const auto q02 = __builtin_amdgcn_permlane32_swap(p01[0], p23[0], false, false);
        const auto q13 = __builtin_amdgcn_permlane32_swap(p01[1], p23[1], false, false);
        A[st][0] = __uint_as_float(q02[0]);
        A[st][1] = __uint_as_float(q13[0]);
        A[st][2] = __uint_as_float(q02[1]);
        A[st][3] = __uint_as_float(q13[1]);
    }
}

// Min over the members of the clusters some live walker of the wave may need,
// deciding 16 clusters at a time on the matrix cores: D[i][j] (walker i,
// cluster j) lands in lane j + 16 (i / 4), register i % 4, so the clusters
// any walker keeps are the low 16 bits of the OR of the four register votes
// folded over the lane groups.  NaN never skips.  thr as for cluster_min.
template <int D, bool BOX>
__device__ __forceinline__ float cluster_min_mfma(cptr<float> rows, const float* __restrict__ mf, int n_cl,
                                                  const float (&x)[D], float thr, bool live, uint32_t& n_eval)
{
    constexpr int S = BOX ? box_stride(D) : sph_stride(D);
    float A[3][4];
    mfma_walker_operands<D>(x, thr, live, A);
    const mf4* tab = reinterpret_cast<const mf4*>(mf) + (threadIdx.x & (kWave - 1));
    const int n_tiles = (n_cl + kMfmaTile - 1) / kMfmaTile;
    float best = Math<float>::inf();
    // the next tile's features load while this tile is tested (the table
    // ends with a spare tile that is never used)
    mf4 bn = tab[0];
    for (int t = 0; t < n_tiles; ++t) {
        const mf4 b = bn;
        bn = tab[(t + 1) * kWave];
        uint64_t keep = 0;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            mf4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0][rt], b[0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[1][rt], b[1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[2][rt], b[2], acc, 0, 0, 0);
            keep |= __ballot(!(acc[0] > 0.0f)) | __ballot(!(acc[1] > 0.0f)) | __ballot(!(acc[2] > 0.0f)) |
                    __ballot(!(acc[3] > 0.0f));
        }
        keep |= keep >> 32;
        keep |= keep >> 16;
        uint32_t mask = (uint32_t)keep & 0xFFFFu;
        while (mask) {  // wave-uniform
            const int j = __builtin_ctz(mask);
            mask &= mask - 1u;
            best = cluster_members_min<float, D, BOX>(x, rows + (t * kMfmaTile + j) * (kCluster * S), best);
            n_eval += kCluster;
        }
    }
    return best;
}

// Planar arm (Sec. V-A): the task-plane distance between the obstacle points
// and the links at joint angles x (link i turns by x_0 + ... + x_i, base joint
// at the origin), times 1 / K, a lower bound of the joint-space distance to
// collision.
template <typename T, int D>
__device__ __forceinline__ T arm_dist(cenv<T> p, const T (&x)[D])
{
    cptr<T> pts = to_const(p->arm_pts);
    const int n = p->n_arm;
    T ax = 0, ay = 0, th = 0, best = Math<T>::inf();  // squared distance
#pragma unroll
    for (int i = 0; i < D; ++i) {
        th += x[i];
        T sn, cs;
        Math<T>::sincos(th, sn, cs);
        const T sx = p->arm_l[i] * cs, sy = p->arm_l[i] * sn;
        const T ss = Math<T>::fma(sx, sx, sy * sy);
        const T inv = ss > T(0) ? T(1) / ss : T(0);
        for (int j = 0; j < n; ++j) {
            const T px = pts[2 * j] - ax, py = pts[2 * j + 1] - ay;
            const T t = Math<T>::min(Math<T>::max(Math<T>::fma(px, sx, py * sy) * inv, T(0)), T(1));
            const T ex = px - t * sx, ey = py - t * sy;
            best = Math<T>::min(best, Math<T>::fma(ex, ex, ey * ey));
        }
        ax += sx;
        ay += sy;
    }
    return Math<T>::sqrt(best) * p->arm_invK;
}

// ------------------------------------------------------------------------
// Pair-compacted member scan (FP32).  The matrix-core test gives, per tile,
// one ballot per (row tile, register): bit j + 16 g of ballot (rt, r) says
// walker 16 rt + 4 g + r may need cluster 16 t + j.  Instead of every lane
// scanning the members of every cluster some lane needs, each needed
// (walker, cluster) pair is queued in LDS and the wave evaluates pairs 64 at
// a time, lane k taking pair k: it fetches the walker's position from that
// walker's lane, scans the cluster's members with vector loads, and folds the
// result into the walker's minimum with an LDS atomic min.  Every lane's
// result is the minimum over the same member distances a scan of its needed
// clusters computes, so R and every walk are unchanged.
// ------------------------------------------------------------------------

// Order-preserving map between FP32 values and uint32 (LDS atomic min of
// signed distances): non-negative values set the sign bit, negative ones
// flip every bit.
__device__ __forceinline__ uint32_t ord_of(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_of_ord(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Obstacle distances evaluated, summed over the live lanes of a wave: the
// scans are wave-uniform, so every lane evaluates the same rows, and the
// tally is one wave-level count for the work statistics.  Callers run the
// step on every lane of the wave (idle lanes with live false), so the tally
// is updated in wave-uniform control flow.  pairs: the wave's LDS slice of
// kPairLds words for the pair-compacted scan (kPairCap entries of the first
// queue, kBoxQueue of the member queue, both cluster << 6 | walker, then the
// 64 walkers' minima), owned by the kernel.  cbox: cluster bounding boxes
// tested (pair-compacted scan only).
struct WorkCount {
    uint64_t sph = 0, box = 0, cbox = 0;
    uint32_t* pairs;
    __device__ explicit WorkCount(uint32_t* p) : pairs(p) {}
};

// Walker lane of a queue entry: its walker field q = 16 rt + 4 r + g (see
// cluster_min_pairs) names lane 16 rt + 4 g + r.
__device__ __forceinline__ int entry_walker(uint32_t e)
{
    const uint32_t q = e & (kWave - 1);
    return (int)((q & 0x30u) | ((q & 3u) << 2) | ((q >> 2) & 3u));
}

// Evaluate queue entries [base, base + count), count <= 64, one per lane; a
// round of at most 32 (16, 8) entries gives each entry 2 (4, 8) lanes, which
// split its members (lane sub of an entry takes members sub, sub + 2^sh, ...),
// so a part-filled round, such as a step's last, costs a half (a quarter, an
// eighth) of a full one.  The minimum is the same: every member is evaluated
// once and folds into its walker's slot.  All lanes of the wave take part
// (the walker positions move by lane shuffles).
template <int D, bool BOX>
__device__ __forceinline__ void pair_round(cptr<float> rows, int n_cl, const uint32_t* queue, int base, int count,
                                           const float (&x)[D], uint32_t* best)
{
    constexpr int S = BOX ? box_stride(D) : sph_stride(D);
    const int lane = threadIdx.x & (kWave - 1);
    const int sh = count > 32 ? 0 : count > 16 ? 1 : count > 8 ? 2 : 3;  // wave-uniform
    const int slot = lane >> sh;
    const bool act = slot < count;
    const uint32_t e = act ? queue[base + slot] : 0u;
    const int w = entry_walker(e);
    int c = (int)(e >> 6);
    c = c < n_cl ? c : n_cl - 1;  // an entry never points past the table
    float xw[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xw[i] = __shfl(x[i], w, kWave);
    if (act) {
        cptr<float> r = rows + (int64_t)c * (kCluster * S);
        float m = Math<float>::inf();
        if (sh == 0) {
            // two members per iteration: the rows arrive in vector registers,
            // so a full unroll would hold all eight clusters' members at once
#pragma unroll 2
            for (int j = 0; j < kCluster; ++j)
                m = Math<float>::min(m, BOX ? box_dist<float, D>(xw, r + j * S) : sphere_dist<float, D>(xw, r + j * S));
        } else {
            r += (lane & ((1 << sh) - 1)) * S;
            const int n = kCluster >> sh;
            for (int j = 0; j < n; ++j)
                m = Math<float>::min(m, BOX ? box_dist<float, D>(xw, r + (j << sh) * S)
                                            : sphere_dist<float, D>(xw, r + (j << sh) * S));
        }
        atomicMin(&best[w], ord_of(m));
    }
}

// Bounding-box test of queue entries [base, base + count), count <= 64, one
// per lane: an entry passes unless the distance from its walker to its
// cluster's box, times Cull<float>::shrink, exceeds thr0 = max(thr, 0) of
// that walker; passing entries are appended to the member queue mq (mqn
// entries, fewer than 64 on entry, wave-uniform).
//
// Soundness (FP32, unit roundoff u = 2^-24): the stored box contains the
// members' box enlarged by delta = 2^-16 times its diagonal in every
// direction, so a walker at distance L from the members' box is at most
// max(0, L - delta) from the stored one.  The computed box distance is
// within (D / 2 + 4) u of that relatively, the shrink takes 2^-16 off, and a
// member's computed distance is at most (D + 4) u (L + diagonal) below its
// exact distance, itself >= L; so a skipped entry's members all have computed
// distances above max(thr, 0), and none attains or ties the minimum.  Inside
// the stored box the computed distance is exactly 0 (every clamped
// difference rounds to a value <= 0) and the entry passes.  A NaN walker
// gives distance 0 or NaN and passes.
template <int D>
__device__ __forceinline__ void box_round(const float* __restrict__ cb, int n_cl, const uint32_t* queue, int base,
                                          int count, const float (&x)[D], float thr0, uint32_t* mq, int& mqn)
{
    const int lane = threadIdx.x & (kWave - 1);
    const bool act = lane < count;
    const uint32_t e = act ? queue[base + lane] : 0u;
    const int w = entry_walker(e);
    int c = (int)(e >> 6);
    c = c < n_cl ? c : n_cl - 1;  // an entry never points past the table
    float xw[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xw[i] = __shfl(x[i], w, kWave);
    const float tw = __shfl(thr0, w, kWave);
    const mf4* r = reinterpret_cast<const mf4*>(cb + (int64_t)c * kClusterBox);
    const mf4 lo0 = r[0], hi0 = r[2];
    mf4 lo1 = lo0, hi1 = hi0;
    if (D > 4) {
        lo1 = r[1];
        hi1 = r[3];
    }
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float lo = i < 4 ? lo0[i & 3] : lo1[i & 3];
        const float hi = i < 4 ? hi0[i & 3] : hi1[i & 3];
        const float t = __builtin_fmaxf(__builtin_fmaxf(lo - xw[i], xw[i] - hi), 0.0f);
        acc = __builtin_fmaf(t, t, acc);
    }
    const bool pass = act && !(__builtin_amdgcn_sqrtf(acc) * Cull<float>::shrink > tw);
    const uint64_t m = __builtin_amdgcn_ballot_w64(pass);
    if (pass) {
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        mq[mqn + (int)rank] = e;
    }
    mqn += __popcll(m);
}

// Inclusive prefix sum over the 64 lanes of a wave: DPP row shifts by 1, 2,
// 4 and 8 sum within each row of 16 lanes, then the broadcasts of lane 15
// (into rows 1 and 3) and lane 31 (into rows 2 and 3) carry the row totals.
// Lanes whose source is outside the row or masked off add 0.  All lanes must
// be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)x;
}

// Min over the members of the clusters each lane may need (thr as for
// cluster_min), with the cluster test on the matrix cores, a bounding-box
// test of the pairs it keeps (BOXT), and the members of the pairs that pass
// both scanned pair by pair.  Requires every lane of the wave to be active; lds is
// the wave's kPairLds-word slice (first queue, member queue, minima).  evals:
// member distances evaluated by the wave; boxes: bounding boxes tested.
//
// Per tile each lane gathers its 16 needs (bit 4 rt + r: walker 16 rt + 4 g +
// r, g = lane / 16, needs cluster 16 t + lane % 16) into one mask; a wave
// prefix sum of the popcounts gives every lane its queue slots, so a tile's
// pairs are queued in one pass.  A tile whose pairs would overflow the queue
// first tests the pairs already waiting, then goes two need bits at a time
// (at most 128 pairs each).
template <int D, bool BOX, bool BOXT>
__device__ __forceinline__ float cluster_min_pairs(cptr<float> rows, const float* __restrict__ mf,
                                                   const float* __restrict__ cb, int n_cl, const float (&x)[D],
                                                   float thr, bool live, uint64_t& evals, uint64_t& boxes,
                                                   uint32_t* lds)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t* queue = lds;
    uint32_t* mq = lds + kPairCap;
    uint32_t* best = mq + kBoxQueue;
    best[lane] = ord_of(Math<float>::inf());
    float A[3][4];
    mfma_walker_operands<D>(x, thr, live, A);
    const mf4* tab = reinterpret_cast<const mf4*>(mf) + lane;
    const int n_tiles = (n_cl + kMfmaTile - 1) / kMfmaTile;
    // queue entry: cluster << 6 | q, where the need bit 4 rt + r of lane
    // 16 g + j (walker 16 rt + 4 g + r, cluster 16 t + j) gives
    // q = (bit << 2) | g = 16 rt + 4 r + g, so each entry is one shift-or of
    // the bit index into the lane's constant part
    const uint32_t lane_e = ((uint32_t)(lane & (kMfmaTile - 1)) << 6) | (uint32_t)(lane >> 4);
    const float thr0 = __builtin_fmaxf(thr, 0.0f);  // the box test's threshold
    int qn = 0;   // first-queue pairs (wave-uniform), < 64 between tiles
    int mqn = 0;  // member-queue pairs (wave-uniform), < 64 between rounds
    uint32_t tested = 0, pairs = 0;
    // box-test first-queue entries [base, base + count); a full member queue
    // evaluates its last 64.  Without the box test the entries go straight to
    // a member round.
    auto test_round = [&](int base, int count) {
        if constexpr (!BOXT) {
            pairs += (uint32_t)count;
            pair_round<D, BOX>(rows, n_cl, queue, base, count, x, best);
        } else {
            box_round<D>(cb, n_cl, queue, base, count, x, thr0, mq, mqn);
            tested += (uint32_t)count;
            if (mqn >= kWave) {
                mqn -= kWave;
                pairs += kWave;
                pair_round<D, BOX>(rows, n_cl, mq, mqn, kWave, x, best);
            }
        }
    };
    // the next tile's features load while this tile is tested and queued (the
    // table ends with a spare tile that is never used)
    mf4 bn = tab[0];
    for (int t = 0; t < n_tiles; ++t) {
        const mf4 b = bn;
        bn = tab[(t + 1) * kWave];
        // need bit = the test value's sign bit, shifted in from the top
        // (rt = 3, r = 3 first) with one v_alignbit per value: a value >= +0
        // is skipped, which the margin makes as sound as > 0 (the rounding is
        // far below m times the sum of squares); NaN (a non-finite walker)
        // with the sign clear skips too
        uint32_t nm = 0;
#pragma unroll
        for (int rt = 3; rt >= 0; --rt) {
            mf4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0][rt], b[0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[1][rt], b[1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[2][rt], b[2], acc, 0, 0, 0);
#pragma unroll
            for (int r = 3; r >= 0; --r) nm = __builtin_amdgcn_alignbit(nm, __float_as_uint(acc[r]), 31u);
        }
        uint32_t cnt = (uint32_t)__builtin_popcount(nm);
        uint32_t incl = wave_incl_scan(cnt);
        int total = __builtin_amdgcn_readlane((int)incl, kWave - 1);
        uint32_t chunk = 0xFFFFu;  // the needs queued in this pass
        if (qn + total > kPairCap) {
            if (qn > 0) {
                test_round(0, qn);
                qn = 0;
            }
            chunk = 0x3u;
        }
        const uint32_t tile_e = (uint32_t)(t * kMfmaTile) << 6;
        for (;;) {  // wave-uniform: one pass, or one per two need bits
            uint32_t m = nm & chunk;
            if (chunk != 0xFFFFu) {
                cnt = (uint32_t)__builtin_popcount(m);
                incl = wave_incl_scan(cnt);
                total = __builtin_amdgcn_readlane((int)incl, kWave - 1);
            }
            uint32_t pos = (uint32_t)qn + incl - cnt;
            while (m) {  // per lane: its own needs, in bit order
                const uint32_t bit = (uint32_t)__builtin_ctz(m);
                m &= m - 1u;
                queue[pos++] = (bit << 2) | (tile_e + lane_e);
            }
            qn += total;
            while (qn >= kWave) {  // the last 64 queued go first
                qn -= kWave;
                test_round(qn, kWave);
            }
            if (chunk & 0x8000u) break;
            chunk <<= 2;
        }
    }
    // the step's last pairs: when the waiting ones of both queues fit one
    // member round, they go together without their box test (that round runs
    // anyway unless every box test fails, and a skipped test only adds member
    // distances, which never change the minimum)
    if constexpr (!BOXT) {
        if (qn > 0) test_round(0, qn);
    } else {
        if (qn + mqn <= kWave) {
            if (lane < qn) mq[mqn + lane] = queue[lane];
            mqn += qn;
        } else {
            test_round(0, qn);
        }
        if (mqn > 0) pair_round<D, BOX>(rows, n_cl, mq, 0, mqn, x, best);
    }
    evals += ((uint64_t)pairs + (uint64_t)mqn) * kCluster;
    boxes += tested;
    return float_of_ord(best[lane]);
}

// R = distance to the boundary; cls = first component attaining it in the
// order goal, spheres, boxes, outer.  The goal and outer distances come first
// and bound the box scan, whose result then bounds the sphere scan; ub, any
// value at or above the R a scan of every obstacle computes (the walker's
// bound from its previous step, +inf when it has none), bounds both scans as
// well.  Culled clusters leave R and cls as a scan of every obstacle gives
// them.
template <typename T, int D>
__device__ __forceinline__ T distance(cenv<T> p, const T (&x)[D], int& cls, WorkCount& wc, bool live,
                                      T ub = Math<T>::inf())
{
    T dg = Math<T>::inf();
    if (p->has_goal) {
        T t = x[0] - p->goal_c[0];
        T acc = t * t;
#pragma unroll
        for (int i = 1; i < D; ++i) {
            t = x[i] - p->goal_c[i];
            acc = Math<T>::fma(t, t, acc);
        }
        dg = Math<T>::sqrt(acc) - p->goal_r;
    }
    // extruded geometry: obstacles and the outer boundary see the leading
    // geom_d coordinates only (their stored centres are zero beyond them)
    T xg[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xg[i] = (i < p->geom_d) ? x[i] : T(0);
    const T dout = outer_dist<T, D>(fresh(p), xg);
    p = fresh(p);
    // the arm bound (joint coordinates, never extruded) tightens the scans
    const T da = p->n_arm ? arm_dist<T, D>(p, x) : Math<T>::inf();
    const T dga = Math<T>::min(dg, Math<T>::min(da, dout));
    const T tg = Math<T>::min(dga, ub);  // the scans' threshold before the box result
    p = fresh(p);
    T db;
    uint32_t nb, ns;         // member distances per lane (wave-uniform scans)
    uint64_t eb = 0, es = 0;  // member distances of the wave (pair-compacted scans)
    uint64_t cbt = 0;         // cluster bounding boxes tested by the wave
    if (p->n_cl_box) {
        nb = 0;
        bool done = false;
        if constexpr (sizeof(T) == 4) {
            if (p->use_mfma == 2) {
                if (p->box_test)
                    db = cluster_min_pairs<D, true, true>(to_const(fresh(p)->box_cl), fresh(p)->box_mf,
                                                          fresh(p)->box_cb, fresh(p)->n_cl_box, xg, tg, live, eb,
                                                          cbt, wc.pairs);
                else
                    db = cluster_min_pairs<D, true, false>(to_const(fresh(p)->box_cl), fresh(p)->box_mf,
                                                           fresh(p)->box_cb, fresh(p)->n_cl_box, xg, tg, live, eb,
                                                           cbt, wc.pairs);
                done = true;
            } else if (p->use_mfma) {
                db = cluster_min_mfma<D, true>(to_const(p->box_cl), fresh(p)->box_mf, fresh(p)->n_cl_box, xg,
                                               tg, live, nb);
                done = true;
            }
        }
        if (!done)
            db = cluster_min<T, D, true>(to_const(fresh(p)->box_cl), to_const(fresh(p)->box_bnd), fresh(p)->n_cl_box, xg,
                                         tg, live, nb);
    } else {
        db = boxes_min<T, D>(to_const(p->box), fresh(p)->n_box, xg);
        nb = (uint32_t)fresh(p)->n_box;
    }
    p = fresh(p);
    T ds;
    if (p->n_cl_sph) {
        ns = 0;
        bool done = false;
        if constexpr (sizeof(T) == 4) {
            if (p->use_mfma == 2) {
                if (p->box_test)
                    ds = cluster_min_pairs<D, false, true>(to_const(fresh(p)->sph_cl), fresh(p)->sph_mf,
                                                           fresh(p)->sph_cb, fresh(p)->n_cl_sph, xg,
                                                           Math<T>::min(tg, db), live, es, cbt, wc.pairs);
                else
                    ds = cluster_min_pairs<D, false, false>(to_const(fresh(p)->sph_cl), fresh(p)->sph_mf,
                                                            fresh(p)->sph_cb, fresh(p)->n_cl_sph, xg,
                                                            Math<T>::min(tg, db), live, es, cbt, wc.pairs);
                done = true;
            } else if (p->use_mfma) {
                ds = cluster_min_mfma<D, false>(to_const(p->sph_cl), fresh(p)->sph_mf, fresh(p)->n_cl_sph, xg,
                                                Math<T>::min(tg, db), live, ns);
                done = true;
            }
        }
        if (!done)
            ds = cluster_min<T, D, false>(to_const(fresh(p)->sph_cl), to_const(fresh(p)->sph_bnd), fresh(p)->n_cl_sph,
                                          xg, Math<T>::min(tg, db), live, ns);
    } else {
        ds = spheres_min<T, D>(to_const(p->sph), fresh(p)->n_sph, xg);
        ns = (uint32_t)fresh(p)->n_sph;
    }
    const uint64_t lanes = (uint64_t)__popcll(__ballot(live));
    wc.sph += lanes * ns + es;
    wc.box += lanes * nb + eb;
    wc.cbox += cbt;
    const T ao = Math<T>::min(da, dout);
    const T bo = Math<T>::min(db, ao);
    const T rest = Math<T>::min(ds, bo);
    cls = (dg <= rest) ? kGoal : (ds <= bo) ? kSphere : (db <= ao) ? kBox : (da <= dout) ? kArm : kOuter;
    return Math<T>::min(dg, rest);
}

// Closest boundary point xbar on the absorbing component (Fig. 2), in the
// coordinates the component depends on.  Sphere and box indices are
// recovered by rescanning with the same distance code.
template <typename T, int D>
__device__ __forceinline__ void closest_point_in(cenv<T> p, const T (&x)[D], int cls, T (&xb)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) xb[i] = x[i];
    if (cls == kOuter && p->outer_kind == 0) {
        int im = 0;
        bool hif = false;
        T m = Math<T>::inf();
        for (int i = 0; i < D; ++i) {
            const T a = x[i] - p->lo[i], b = p->hi[i] - x[i];
            if (a < m) { m = a; im = i; hif = false; }
            if (b < m) { m = b; im = i; hif = true; }
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (i == im) xb[i] = hif ? p->hi[i] : p->lo[i];
        return;
    }
    T c[D];
    T r;
    if (cls == kBox) {
        constexpr int S = box_stride(D);
        cptr<T> tab = to_const(p->box);
        int jm = 0;
        T best = Math<T>::inf();
        for (int j = 0; j < p->n_box; ++j) {
            const T dj = box_dist<T, D>(x, tab + j * S);
            if (dj < best) { best = dj; jm = j; }
        }
        cptr<T> row = tab + jm * S;
        bool inside = true;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (Math<T>::abs(x[i] - row[i]) > row[D + i]) inside = false;
        if (!inside) {
#pragma unroll
            for (int i = 0; i < D; ++i)
                xb[i] = Math<T>::min(Math<T>::max(x[i], row[i] - row[D + i]), row[i] + row[D + i]);
            return;
        }
        int im = 0;
        T qm = -Math<T>::inf();
        for (int i = 0; i < D; ++i) {
            const T q = Math<T>::abs(x[i] - row[i]) - row[D + i];
            if (q > qm) { qm = q; im = i; }
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (i == im) xb[i] = row[i] + (x[i] >= row[i] ? row[D + i] : -row[D + i]);
        return;
    }
    if (cls == kSphere) {
        constexpr int S = sph_stride(D);
        cptr<T> tab = to_const(p->sph);
        int jm = 0;
        T best = Math<T>::inf();
        for (int j = 0; j < p->n_sph; ++j) {
            const T dj = sphere_dist<T, D>(x, tab + j * S);
            if (dj < best) { best = dj; jm = j; }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) c[i] = tab[jm * S + i];
        r = tab[jm * S + D];
    } else if (cls == kGoal) {
#pragma unroll
        for (int i = 0; i < D; ++i) c[i] = p->goal_c[i];
        r = p->goal_r;
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) c[i] = p->oc[i];
        r = p->orad;
    }
    T n2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) n2 = Math<T>::fma(x[i] - c[i], x[i] - c[i], n2);
    if (n2 == T(0)) {
#pragma unroll
        for (int i = 0; i < D; ++i) xb[i] = c[i];
        xb[0] = c[0] + r;
        return;
    }
    const T s = r / Math<T>::sqrt(n2);
#pragma unroll
    for (int i = 0; i < D; ++i) xb[i] = c[i] + s * (x[i] - c[i]);
}

// Closest boundary point of an extruded component (obstacle or outer
// boundary with geom_d < d): the projection acts on the leading geom_d
// coordinates and keeps the others.
template <typename T, int D>
__device__ __forceinline__ void closest_point(cenv<T> p, const T (&x)[D], int cls, T (&xb)[D])
{
    if (cls == kArm) {  // the arm bound names no boundary point (class data only)
#pragma unroll
        for (int i = 0; i < D; ++i) xb[i] = x[i];
        return;
    }
    const int k = (cls == kGoal) ? D : p->geom_d;
    T xg[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xg[i] = (i < k) ? x[i] : T(0);
    closest_point_in<T, D>(p, xg, cls, xb);
#pragma unroll
    for (int i = 0; i < D; ++i)
        if (i >= k) xb[i] = x[i];
}

// Boundary data g at the closest point of the absorbing component.
template <typename T, int D>
__device__ __forceinline__ T boundary_value(cenv<T> p, const T (&x)[D], int cls)
{
    if (p->mode == 0) return cls == kGoal ? p->g_goal : (cls == kOuter ? p->g_outer : p->g_obs);
    T xb[D];
    closest_point<T, D>(p, x, cls, xb);
    T s = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) s = Math<T>::fma(p->ak[i], xb[i], s);
    return p->mode == 1 ? s + p->b : Math<T>::exp(s);
}

// 0F1(; b; y) by Horner's rule on the host-computed coefficients, four
// terms per iteration (one 16-byte scalar load).  The tables are zero beyond
// nt and hold kMaxTerms (a multiple of 4) entries, so the sum starts at up to
// three zero coefficients above the top term: fma(0, y, c) = c exactly, and
// the value is bit for bit that of a loop over nt terms.
static_assert(kMaxTerms % 4 == 0, "Horner tables are read four terms at a time");
template <typename T, typename C>
__device__ __forceinline__ T horner(const C& c, int nt, T y)
{
    T acc = T(0);
    for (int i = ((nt + 3) & ~3) - 4; i >= 0; i -= 4) {
        acc = Math<T>::fma(acc, y, c[i + 3]);
        acc = Math<T>::fma(acc, y, c[i + 2]);
        acc = Math<T>::fma(acc, y, c[i + 1]);
        acc = Math<T>::fma(acc, y, c[i]);
    }
    return acc;
}

// ------------------------------------------------------------------------
// Point source (Sec. VI: a unit impulse at the goal point with zero boundary
// data; Sec. IV-A: the volume term of a step whose ball holds the source and
// the c_imp grad G term of the first-sphere gradient).  nu = d/2 - 1; G_B is
// the Green's function of (-Laplacian + sigma) on the ball of radius R with
// zero data on its sphere, between the centre and a point at distance r:
//   G_B = Phi(r) - Phi(R) p(r) / p(R),  Phi(s) = phi_c s^-nu K_nu(sqrt(sigma) s),
//   p(s) = 0F1(; nu+1; sigma s^2 / 4);
// its centre gradient towards the point has length
//   grad_c r^-nu [K_{nu+1}(sqrt(sigma) r) - K_{nu+1}(sqrt(sigma) R) (r/R)^(nu+1) p1(r) / p1(R)],
//   p1(s) = 0F1(; nu+2; sigma s^2 / 4);
// at sigma = 0 both take their Laplace forms.
// ------------------------------------------------------------------------

// K_nu(z) and K_{nu+1}(z), z > 0, together: the trapezoidal rule on the
// integral of exp(-z cosh t) cosh(nu t) over t >= 0, with step
// min(1/4, 1/(2 sqrt(z))) (the integrand's width near 0 shrinks like
// 1/sqrt(z)), summed until the terms are past their peak and below the
// precision's rounding.  cosh(nu t) exp(-z cosh t) is formed as
// (exp(a + nu t) + exp(a - nu t)) / 2, a = -z cosh t, with the exponent capped
// so that a source closer than about 1e-9 cannot overflow FP32.
template <typename T>
__device__ __forceinline__ void bessel_k_pair(T nu, T z, T& k0, T& k1)
{
    if (!(z > T(0))) {
        k0 = k1 = Math<T>::inf();
        return;
    }
    const T tol = sizeof(T) == 4 ? T(1e-8) : T(1e-17);
    const T cap = T(80);
    const T h = Math<T>::min(T(0.25), T(0.5) * Math<T>::rsqrt(z));
    const T e0 = Math<T>::exp(-z);
    T s0 = T(0.5) * e0, s1 = T(0.5) * e0;
    for (int j = 1; j < 4096; ++j) {
        const T t = T(j) * h;
        const T et = Math<T>::exp(t);
        const T iet = Math<T>::rcp(et);
        const T a = -z * T(0.5) * (et + iet);
        const T u0 = T(0.5) * (Math<T>::exp(Math<T>::min(a + nu * t, cap)) + Math<T>::exp(a - nu * t));
        const T u1 = T(0.5) * (Math<T>::exp(Math<T>::min(a + (nu + T(1)) * t, cap)) + Math<T>::exp(a - (nu + T(1)) * t));
        s0 += u0;
        s1 += u1;
        if (z * T(0.5) * (et - iet) > nu + T(1) && u1 <= tol * s1) break;
    }
    k0 = h * s0;
    k1 = h * s1;
}

template <typename T>
struct SourceTerm {
    T G;    // G_B(r; R)
    T gm;   // length of the centre gradient
    T dG;   // d G_B / d sigma (sigma > 0; NaN at sigma = 0)
};

template <typename T, int D, bool BWD>
__device__ __noinline__ SourceTerm<T> ball_green(cenv<T> p, T r, T R)
{
    SourceTerm<T> o;
    if (p->sigma > T(0)) {
        const T nu = p->nu, sq = p->sqrt_sigma;
        T Kr, K1r, KR, K1R;
        bessel_k_pair<T>(nu, sq * r, Kr, K1r);
        bessel_k_pair<T>(nu, sq * R, KR, K1R);
        const T yr = p->qsigma * r * r, yR = p->qsigma * R * R;
        const T pr = horner<T>(p->cC, p->nt_C, yr), pR = horner<T>(p->cC, p->nt_C, yR);
        const T p1r = horner<T>(p->cC1, p->nt_C1, yr), p1R = horner<T>(p->cC1, p->nt_C1, yR);
        const T rn = Math<T>::pow(r, -nu), Rn = Math<T>::pow(R, -nu);
        const T ratio = pr / pR;
        o.G = p->phi_c * (rn * Kr - Rn * KR * ratio);
        o.gm = p->grad_c * rn * (K1r - K1R * Math<T>::pow(r / R, nu + T(1)) * (p1r / p1R));
        if (BWD) {
            // d Phi(s) / d sigma = phi_c s^-nu [(nu / sigma) K_nu - s / (2 sqrt(sigma)) K_{nu+1}]
            // d p(s) / d sigma = (s^2 / 4) p1(s) / (nu + 1)
            const T is = T(1) / p->sigma, ih = T(0.5) / sq;
            const T dPr = p->phi_c * rn * (nu * is * Kr - r * ih * K1r);
            const T dPR = p->phi_c * Rn * (nu * is * KR - R * ih * K1R);
            const T inv = T(1) / (nu + T(1));
            const T dpr = T(0.25) * r * r * p1r * inv, dpR = T(0.25) * R * R * p1R * inv;
            const T dratio = (dpr * pR - pr * dpR) / (pR * pR);
            o.dG = dPr - dPR * ratio - p->phi_c * Rn * KR * dratio;
        } else {
            o.dG = T(0);
        }
    } else {
        if (D == 2) {
            o.G = p->phi_c * Math<T>::log(R / r);
            o.gm = p->grad_c * (T(1) / r - r / (R * R));
        } else {
            o.G = p->phi_c * (Math<T>::pow(r, T(2 - D)) - Math<T>::pow(R, T(2 - D)));
            o.gm = p->grad_c * (Math<T>::pow(r, T(1 - D)) - r * Math<T>::pow(R, T(-D)));
        }
        o.dG = __builtin_nan("");
    }
    return o;
}

// ------------------------------------------------------------------------
// One walk (Sec. IV-A).  State lives in registers; an iteration makes one
// distance evaluation and either absorbs (eps-shell, Fig. 2) or applies the
// step's weight and jumps to a uniform point on the sphere of radius R.
// ------------------------------------------------------------------------
template <typename T, int D>
struct Walker {
    T x[D];    // current point x_k
    T v0[D];   // first direction
    T W;       // prod_{i < k} C(R_i): weight of u_hat(x_0)
    T W1;      // prod_{1 <= i < k} C(R_i): weight of u_hat(x_1)
    T gfac;    // (d / R_0) C1(R_0)
    T S;       // sum_{i < k} d ln C(R_i) / d sigma
    T src;     // point source: sum_{i < k} W_i amp G_B(x_i): source part of u_hat(x_0)
    T src1;    // the same with weights W1_i, i >= 1: of u_hat(x_1)
    T srcS;    // sum_i W_i amp (S_i G_B + d G_B / d sigma)
    T gs0;     // c_imp amp |grad G_B(x_0, z)| / |z - x_0| (the first ball holds z)
    uint32_t k;
    uint32_t w;
    int32_t ex;  // W, W1, src, src1 and srcS hold their values times 2^-ex (FP32 only)
    T rb;        // bound on this step's R from the previous one (+inf on a walk's first step)
};

template <typename T>
struct WalkEnd {
    T u;        // u_hat(x_0)
    T gs;       // gradient = gs * v0 (+ gs0 (z - x_0) with a point source)
    T S;        // sum of d ln C / d sigma over the weighted steps
    T goal_w;   // W 1{goal}
    T gs0;      // point source: coefficient of z - x_0 in the gradient
    T ubd;      // point source: boundary part of u_hat(x_0), W g
    T srcS;     // point source: source part of d u_hat / d sigma
    uint32_t steps;
    int32_t status, cls;
    int32_t ex;  // u, gs, goal_w, ubd and srcS hold their values times 2^-ex
};

template <typename T, int D, int DA>
__device__ __forceinline__ void walker_start(Walker<T, DA>& s, const T (&xq)[DA], uint32_t w)
{
#pragma unroll
    for (int i = 0; i < D; ++i) s.x[i] = xq[i];
#pragma unroll
    for (int i = 0; i < DA; ++i) s.v0[i] = T(0);
    s.W = T(1);
    s.W1 = T(1);
    s.gfac = T(0);
    s.S = T(0);
    s.src = T(0);
    s.src1 = T(0);
    s.srcS = T(0);
    s.gs0 = T(0);
    s.k = 0;
    s.w = w;
    s.ex = 0;
    s.rb = Math<T>::inf();
}

// FP32 walks: the weight product of a long walk at a large screening
// coefficient leaves the FP32 range (1/I_0(sqrt(sigma) R) per step in d = 2,
// so a walk whose radii sum to 50 weighs under 2^-200 at sigma = 10).  Once W
// drops below 2^-32 its binary exponent moves into s.ex and W, W1 and the
// source sums are scaled by the same power of two, which is exact; the
// accumulators apply 2^ex in FP64.  The rescale is skipped when it would lift
// one of the other terms past 2^100: they then outweigh every later
// contribution by more than FP32 resolves.  The path never depends on W.
template <bool SRC, bool BWD, int DA>
__device__ __forceinline__ void renormalize(Walker<float, DA>& s)
{
    if (s.W < 0x1p-32f) {
        int e;
        const float m = ::frexpf(s.W, &e);
        float big = s.W1;
        if (SRC) big = ::fmaxf(big, ::fmaxf(::fabsf(s.src), ::fabsf(s.src1)));
        if (SRC && BWD) big = ::fmaxf(big, ::fabsf(s.srcS));
        if (::ldexpf(big, -e) < 0x1p100f) {
            s.W = m;
            s.W1 = ::ldexpf(s.W1, -e);
            if (SRC) {
                s.src = ::ldexpf(s.src, -e);
                s.src1 = ::ldexpf(s.src1, -e);
            }
            if (SRC && BWD) s.srcS = ::ldexpf(s.srcS, -e);
            s.ex += e;
        }
    }
}

template <bool SRC, bool BWD, int DA>
__device__ __forceinline__ void renormalize(Walker<double, DA>&) {}

// Returns true when the walk ended (e is then filled in).  (key0, key1) is
// the Philox key of the launch, q the query's index in its environment.  The
// walker may store DA >= D coordinates; only the first D are used.
template <typename T, int D, bool BWD, int DA = D, bool SRC = false>
__device__ __forceinline__ bool walker_step(cenv<T> p0, Walker<T, DA>& s, uint32_t q, uint32_t key0,
                                            uint32_t key1, WalkEnd<T>& e, WorkCount& wc, bool live)
{
    static_assert(DA >= D, "walker storage narrower than the dimension");
    const T(&x)[D] = reinterpret_cast<const T(&)[D]>(s.x);
    int cls;
    // the step-to-step bound, in the dimensions where it culls (kStepBoundMaxDim)
    constexpr bool kBound = D <= kStepBoundMaxDim;
    const T R = distance<T, D>(fresh(p0), x, cls, wc, live, kBound ? s.rb : Math<T>::inf());
    cenv<T> p = fresh(p0);
    // R(x) is a minimum of distances, each 1-Lipschitz, and the walker moves
    // R: the next R is at most 2 R, and with the margins (rb_abs covers the
    // rounding of the positions and of every component's computed distance,
    // +inf where coordinates are unbounded) at most this computed bound, so
    // it is a threshold the scans may cull against without changing R or cls
    if (kBound) s.rb = Math<T>::fma(R, T(2.001953125), p->rb_abs);  // 2 (1 + 2^-10)
    const uint32_t k = s.k;
    if (R < p->eps) {
        const T g = boundary_value<T, D>(p, x, cls);
        const bool first = (k == 0);
        e.steps = k + 1;
        e.cls = cls;
        e.status = first ? kDegenerate : kAbsorbed;
        e.ex = s.ex;
        e.u = s.W * g;
        e.gs = first ? T(0) : s.gfac * s.W1 * g;
        e.S = s.S;
        e.goal_w = (cls == kGoal) ? s.W : T(0);
        if (SRC) {
            e.ubd = e.u;
            e.u += s.src;
            e.gs = first ? T(0) : s.gfac * (s.W1 * g + s.src1);
            e.gs0 = s.gs0;
            e.srcS = s.srcS;
        }
        return true;
    }
    if (k + 1 >= p->max_steps) {
        e.steps = k + 1;
        e.cls = cls;
        e.status = kTruncated;
        e.ex = 0;
        e.u = T(0);
        e.gs = T(0);
        e.S = T(0);
        e.goal_w = T(0);
        if (SRC) e.gs0 = e.ubd = e.srcS = T(0);
        return true;
    }
    if (SRC && p->has_src) {  // the ball around x_k holds the source: volume term
        T dz2 = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const T t = p->src_z[i] - x[i];
            dz2 = Math<T>::fma(t, t, dz2);
        }
        if (dz2 < R * R) {
            const T r = Math<T>::sqrt(dz2);
            const SourceTerm<T> st = ball_green<T, D, BWD>(p, r, R);
            p = fresh(p0);
            const T Ga = p->src_amp * st.G;
            if (BWD) s.srcS = Math<T>::fma(s.W, Math<T>::fma(s.S, Ga, p->src_amp * st.dG), s.srcS);
            s.src = Math<T>::fma(s.W, Ga, s.src);
            if (k > 0) s.src1 = Math<T>::fma(s.W1, Ga, s.src1);
            else if (r > T(0)) s.gs0 = p->c_imp * p->src_amp * st.gm / r;
        }
        p = fresh(p0);
    }
    const T R2 = R * R;
    const T y = p->qsigma * R2;
    const T C = Math<T>::rcp(horner<T>(p->cC, p->nt_C, y));
    p = fresh(p0);
    s.W *= C;
    s.W1 *= (k > 0) ? C : T(1);
    renormalize<SRC, BWD>(s);
    if (BWD) {
        const T p1 = horner<T>(p->cC1, p->nt_C1, y);
        s.S = Math<T>::fma(T(-0.5 / D) * R2 * p1, C, s.S);
        if (k == 0) s.gfac = T(D) * Math<T>::rcp(R * p1);
    } else if (k == 0) {
        s.gfac = T(D) * Math<T>::rcp(R * horner<T>(p->cC1, p->nt_C1, y));
    }
    T v[D];
    direction<T, D>(k, s.w, q, fresh(p0)->env_id, key0, key1, v);
    if (k == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) s.v0[i] = v[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) s.x[i] = Math<T>::fma(R, v[i], s.x[i]);
    s.k = k + 1;
    return false;
}

// ------------------------------------------------------------------------
// Wave-level sums (64 lanes) of FP64 accumulators.
// ------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace wos

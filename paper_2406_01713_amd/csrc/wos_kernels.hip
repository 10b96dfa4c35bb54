// wos_kernels.hip -- Walk-on-Spheres kernels for gfx950 (CDNA4, wave64).
//
//   plain_kernel       one walk per lane, one wave per (query, 64-walk chunk);
//                      the wave runs until its longest walk ends (forward, or
//                      forward + backward sums when BWD: the backward pass
//                      regenerates the same walks from their Philox counters)
//   persistent_kernel  ragged batch of environments in one launch: resident
//                      waves pull work units (env, query, walk range) from a
//                      device counter, and a lane whose walk ends starts the
//                      unit's next walk at once (lane refill), so a wave is not
//                      held by its longest walk
//   finalize_*         per-query means, standard errors and backward products
//                      from per-wave partial sums, in a fixed order
//   plan_update        one gradient-ascent step of the planning loop
//
// All walk arithmetic lives in wos_device.hpp; the estimator is Sec. IV-A of
// the paper (screened WoS, first-sphere gradient), the step rule Sec. VII.
#include <hip/hip_runtime.h>

#include <cmath>

#include "wos_device.hpp"
#include "wos_launch.hpp"

namespace wos {

namespace {

constexpr int kBlock = 256;  // 4 waves per block for the plain / finalize kernels

__device__ __forceinline__ void apply_key_add(uint32_t& k0, uint32_t& k1, const uint64_t* key_add)
{
    if (key_add) {
        const uint64_t key = (((uint64_t)k1 << 32) | k0) + *to_const(key_add);
        k0 = (uint32_t)key;
        k1 = (uint32_t)(key >> 32);
    }
}

// Sum the accumulators of a wave and let lane 0 store them.
template <int N>
__device__ __forceinline__ void wave_store(double (&a)[N], double* out)
{
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = wave_sum(a[i]);
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = a[i];
    }
}

// 2^ex: the factor between a finished walk's stored weighted terms and their
// values (the FP32 walk keeps the weight's exponent apart; FP64 does not).
template <typename T>
__device__ __forceinline__ double walk_scale(const WalkEnd<T>& e)
{
    if (sizeof(T) == 8) return 1.0;
    return ::ldexp(1.0, e.ex);
}

// One-point gradient of a finished walk: gs v0, plus gs0 (z - x_0) when a
// point source lies in the first ball (gs0 carries no weight, so no scale).
template <typename T, int D, int DA, bool SRC>
__device__ __forceinline__ double walk_grad(const WalkEnd<T>& e, const T (&v0)[DA], cenv<T> p, const T* xq, int i,
                                            double sc)
{
    const double g = (double)(e.gs * v0[i]) * sc;
    if (SRC) return g + (double)(e.gs0 * (p->src_z[i] - xq[i]));
    return g;
}

// d u_hat / d sigma of a finished walk: (W g) S, plus the source part.
template <typename T, bool SRC>
__device__ __forceinline__ double walk_dsigma(const WalkEnd<T>& e, double sc)
{
    if (SRC) return ((double)e.ubd * (double)e.S + (double)e.srcS) * sc;
    return (double)e.u * (double)e.S * sc;
}

// Contribution of one finished walk to an accumulator row laid out for DA
// coordinates (nacc(DA) entries), of which the first D are in use.
template <typename T, int D, int DA, bool SRC>
__device__ __forceinline__ void accumulate(double (&a)[nacc(DA)], const WalkEnd<T>& e, const T (&v0)[DA],
                                           cenv<T> p, const T* xq)
{
    const double sc = walk_scale(e);
    const double u = (double)e.u * sc;
    a[0] += u;
    a[1] += u * u;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double g = walk_grad<T, D, DA, SRC>(e, v0, p, xq, i, sc);
        a[2 + i] += g;
        a[2 + DA + i] += g * g;
    }
    a[2 + 2 * DA] += (double)e.steps;
    a[3 + 2 * DA] += (e.status == kTruncated) ? 1.0 : 0.0;
    a[4 + 2 * DA] += (e.status == kDegenerate) ? 1.0 : 0.0;
    a[5 + 2 * DA] += walk_dsigma<T, SRC>(e, sc);
    a[6 + 2 * DA] += (double)e.goal_w * sc;
}

// The wave's work tally goes into lane 0's accumulators before the wave sum.
template <int N>
__device__ __forceinline__ void add_work(double (&a)[N], int at, const WorkCount& wc)
{
    if ((threadIdx.x & (kWave - 1)) == 0) {
        a[at] += (double)wc.sph;
        a[at + 1] += (double)wc.box;
        a[at + 2] += (double)wc.cbox;
    }
}

// ------------------------------------------------------------------------
// Plain kernel.  FP32: at least 4 waves per SIMD (at most 128 registers per
// lane) where that needs no scratch memory (d <= 6, and d = 7 without a
// point source), else at least 3 (168 registers); left free, the allocator
// may take a few more and fall a wave lower.
// ------------------------------------------------------------------------
template <typename T, int D, bool SRC>
constexpr int plain_waves()
{
    return sizeof(T) != 4 ? 1 : (D < 7 || (D == 7 && !SRC)) ? 4 : 3;
}

template <typename T, int D, bool BWD, bool SRC>
__global__ void __launch_bounds__(kBlock, (plain_waves<T, D, SRC>()))
plain_kernel(const EnvP<T>* penv, const T* __restrict__ queries, int64_t n_units, int32_t chunks,
             int64_t n_walks, int64_t w_base, uint32_t q_base, const uint64_t* __restrict__ key_add,
             double* __restrict__ partials, double* __restrict__ records)
{
    __shared__ uint32_t pair_lds[kBlock / kWave][kPairLds];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / kWave) + wv;
    if (unit >= n_units) return;
    const int64_t q = unit / chunks;
    const int64_t wi = (unit - q * chunks) * kWave + lane;
    const cenv<T> p = (cenv<T>)penv;
    uint32_t k0 = p->key0, k1 = p->key1;
    apply_key_add(k0, k1, key_add);

    T xq[D];
    cptr<T> qrow = to_const(queries) + q * D;
#pragma unroll
    for (int i = 0; i < D; ++i) xq[i] = qrow[i];

    const bool active = wi < n_walks;
    Walker<T, D> s;
    walker_start<T, D, D>(s, xq, (uint32_t)(w_base + wi));
    WalkEnd<T> e;
    e.u = e.gs = e.S = e.goal_w = T(0);
    e.ex = 0;
    e.steps = 0;
    e.status = kTruncated;
    e.cls = kOuter;
    WorkCount wc(pair_lds[wv]);
    // every lane steps until the wave's last walk ends (a finished lane runs
    // along idle), so the obstacle scans and the work tally stay wave-uniform
    bool done = !active;
    while (__builtin_amdgcn_ballot_w64(!done) != 0) {
        WalkEnd<T> ek;
        const bool fin = walker_step<T, D, BWD, D, SRC>(p, s, q_base + (uint32_t)q, k0, k1, ek, wc, !done);
        if (fin && !done) {
            e = ek;
            done = true;
        }
    }

    double a[nacc(D)];
#pragma unroll
    for (int i = 0; i < nacc(D); ++i) a[i] = 0.0;
    if (active) accumulate<T, D, D, SRC>(a, e, s.v0, p, xq);
    add_work(a, 7 + 2 * D, wc);
    wave_store<nacc(D)>(a, partials + unit * nacc(D));

    if (records != nullptr && active) {
        double* r = records + wi * (D + 7);
        const double sc = walk_scale(e);
        r[0] = (double)e.u * sc;
#pragma unroll
        for (int i = 0; i < D; ++i) r[1 + i] = walk_grad<T, D, D, SRC>(e, s.v0, p, xq, i, sc);
        r[D + 1] = (double)e.S;
        r[D + 2] = (double)e.goal_w * sc;
        r[D + 3] = (double)e.steps;
        r[D + 4] = (double)e.status;
        r[D + 5] = (double)e.cls;
        r[D + 6] = walk_dsigma<T, SRC>(e, sc);
    }
}

__device__ __forceinline__ double se_of(double s, double s2, double n)
{
    if (n < 2.0) return 0.0;
    const double m = s / n;
    const double var = (s2 - n * m * m) / (n - 1.0);
    return var > 0.0 ? ::sqrt(var / n) : 0.0;
}

template <typename T, int D, bool BWD>
__global__ void __launch_bounds__(kBlock)
finalize_plain(const double* __restrict__ partials, int64_t n_q, int32_t chunks, int64_t n_walks,
               T* __restrict__ out_u, T* __restrict__ out_grad, double* __restrict__ out_stats,
               const T* __restrict__ ubar, T* __restrict__ out_dx, double* __restrict__ out_dq,
               double* __restrict__ prod)
{
    // one block per query: thread t sums chunks t, t + kBlock, ... in order,
    // then a butterfly over each wave and the waves in index order, so the
    // result does not depend on timing
    const int64_t q = blockIdx.x;
    if (q >= n_q) return;
    constexpr int NA = nacc(D);
    constexpr int NW = kBlock / kWave;
    __shared__ double wsum[NW][NA];
    double a[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = 0.0;
    const double* row = partials + q * chunks * NA;
    for (int c = threadIdx.x; c < chunks; c += kBlock) {
#pragma unroll
        for (int i = 0; i < NA; ++i) a[i] += row[(int64_t)c * NA + i];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = wave_sum(a[i]);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) wsum[wv][i] = a[i];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        a[i] = wsum[0][i];
        for (int w = 1; w < NW; ++w) a[i] += wsum[w][i];
    }
    const double n = (double)n_walks;
    out_u[q] = (T)(a[0] / n);
    if (out_grad) {
#pragma unroll
        for (int i = 0; i < D; ++i) out_grad[q * D + i] = (T)(a[2 + i] / n);
    }
    if (out_stats) {
        double* st = out_stats + q * (D + 4);
        st[0] = se_of(a[0], a[1], n);
#pragma unroll
        for (int i = 0; i < D; ++i) st[1 + i] = se_of(a[2 + i], a[2 + D + i], n);
        st[D + 1] = a[2 + 2 * D] / n;
        st[D + 2] = a[3 + 2 * D];
        st[D + 3] = a[4 + 2 * D];
    }
    if (BWD) {
        const double ub = (double)ubar[q];
        const double dqs = a[5 + 2 * D] / n, dqg = a[6 + 2 * D] / n;
        if (out_dq) {
            out_dq[2 * q] = dqs;
            out_dq[2 * q + 1] = dqg;
        }
        prod[2 * q] = ub * dqs;
        prod[2 * q + 1] = ub * dqg;
#pragma unroll
        for (int i = 0; i < D; ++i) out_dx[q * D + i] = (T)(ub * (a[2 + i] / n));
    }
}

// Fixed-order block reduction (deterministic run to run).
__global__ void __launch_bounds__(kBlock)
reduce_pairs(const double* __restrict__ prod, int64_t n, double* out0, double* out1)
{
    __shared__ double s0[kBlock], s1[kBlock];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        a += prod[2 * i];
        b += prod[2 * i + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out0 = s0[0];
        *out1 = s1[0];
    }
}

// ------------------------------------------------------------------------
// Persistent ragged-batch kernel (FP32).
// ------------------------------------------------------------------------
typedef __attribute__((address_space(4))) const BatchEnv CBatch;

constexpr int kNAccBatch = nacc(kMaxDim);

// One walk step of an env of dimension d on the shared 8-wide walker state.
template <bool BWD, bool SRC>
__device__ __forceinline__ bool step_any_d(int d, cenv<float> p, Walker<float, kMaxDim>& s, uint32_t q,
                                           uint32_t k0, uint32_t k1, WalkEnd<float>& e, WorkCount& wc,
                                           bool live)
{
    switch (d) {
    case 2: return walker_step<float, 2, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    case 3: return walker_step<float, 3, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    case 4: return walker_step<float, 4, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    case 5: return walker_step<float, 5, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    case 6: return walker_step<float, 6, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    case 7: return walker_step<float, 7, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    default: return walker_step<float, 8, BWD, kMaxDim, SRC>(p, s, q, k0, k1, e, wc, live);
    }
}

// Gradient sums and sums of squares of a work unit (2 x kMaxDim doubles per
// lane) live in LDS: they change only when a walk ends, and keeping them out
// of registers leaves the walk loop without register spills.  Layout per
// wave: [entry][lane], so a wave's accesses to one entry are contiguous.
constexpr int kLdsAcc = 2 * kMaxDim;

// One work unit: walks [w_begin, w_end) of one query, with lane refill.  The
// walker state is 8 wide for every d, so the dimension only selects the step
// code.  Accumulators other than the gradient ones stay in registers.
template <bool BWD, bool SRC>
__device__ __forceinline__ void run_unit(cenv<float> p, CBatch& be, int64_t local, const float* queries,
                                         uint32_t k0, uint32_t k1, double* lds, uint32_t* pairs, double* out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int d = be.d;
    const int64_t n_walks = be.n_walks;
    const int64_t ql = local / be.splits;
    const int64_t sp = local - ql * be.splits;
    const int64_t w_begin = sp * (int64_t)be.wps;
    const int64_t w_end = (w_begin + be.wps < n_walks) ? w_begin + be.wps : n_walks;
    // walks of the unit counted from w_begin in 32 bits (a unit holds at
    // most wps < 2^31 walks); walk ids are taken modulo 2^32 as before
    const int32_t n_unit = (int32_t)(w_end - w_begin);
    const uint32_t id0 = (uint32_t)w_begin;

    float xq[kMaxDim];
    cptr<float> qrow = to_const(queries) + (be.q_off + ql) * be.q_stride;
#pragma unroll
    for (int i = 0; i < kMaxDim; ++i) xq[i] = (i < d) ? qrow[i < d ? i : 0] : 0.0f;

    // registers: [0] u, [1] u^2, then steps, truncated, degenerate, u S,
    // goal weight, sphere and box distances and cluster boxes (the nacc
    // layout without the gradient entries; the last three from the wave's
    // work tally)
    constexpr int NR = kNAccBatch - kLdsAcc;
    double a[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) a[i] = 0.0;
    double* g = lds + lane;
#pragma unroll
    for (int i = 0; i < kLdsAcc; ++i) g[i * kWave] = 0.0;

    // lanes [0, be.lanes) carry walks; the rest (with more than one lane per
    // walker) only take part in the member scans of the pair rounds
    const int lanes = be.lanes;
    Walker<float, kMaxDim> s;
    bool active = lane < lanes && lane < n_unit;
    walker_start<float, kMaxDim, kMaxDim>(s, xq, id0 + (uint32_t)lane);
    int32_t base = lanes;
    const uint32_t qi = (uint32_t)ql;
    WorkCount wc(pairs);

    while (__builtin_amdgcn_ballot_w64(active) != 0) {
        WalkEnd<float> e;
        // idle lanes (the unit has no walks left for them) step along
        bool fin = step_any_d<BWD, SRC>(d, p, s, qi, k0, k1, e, wc, active);
        fin = fin && active;
        {
            if (fin) {
                const double sc = walk_scale(e);
                const double u = (double)e.u * sc;
                a[0] += u;
                a[1] += u * u;
                a[2] += (double)e.steps;
                a[3] += (e.status == kTruncated) ? 1.0 : 0.0;
                a[4] += (e.status == kDegenerate) ? 1.0 : 0.0;
                a[5] += walk_dsigma<float, SRC>(e, sc);
                a[6] += (double)e.goal_w * sc;
                // static indices (unrolled, guarded by d) keep the walker in
                // registers; a runtime loop bound would index it dynamically
                // and move it to scratch memory
#pragma unroll
                for (int i = 0; i < kMaxDim; ++i) {
                    if (i < d) {
                        const double gi = walk_grad<float, kMaxDim, kMaxDim, SRC>(e, s.v0, p, xq, i, sc);
                        g[i * kWave] += gi;
                        g[(kMaxDim + i) * kWave] += gi * gi;
                    }
                }
            }
        }
        // lane refill: finished lanes take the unit's next walks in lane order
        const uint64_t m = __builtin_amdgcn_ballot_w64(fin);
        if (m) {
            if (fin) {
                const uint32_t rank =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const int32_t wn = base + (int32_t)rank;
                if (wn < n_unit) {
                    walker_start<float, kMaxDim, kMaxDim>(s, xq, id0 + (uint32_t)wn);
                } else {
                    active = false;
                }
            }
            base += __popcll(m);
        }
    }
    add_work(a, 7, wc);
    // back to the nacc(kMaxDim) layout for the partial row
    double row[kNAccBatch];
    row[0] = a[0];
    row[1] = a[1];
#pragma unroll
    for (int i = 0; i < kLdsAcc; ++i) row[2 + i] = g[i * kWave];
#pragma unroll
    for (int i = 2; i < NR; ++i) row[kLdsAcc + i] = a[i];
    wave_store<kNAccBatch>(row, out);
}

// Launch shape: WPB waves per block (1, 2 or 4; the LDS slices scale with
// it) and at least 4 resident waves per SIMD in every shape (the second
// launch bound: at most 128 registers per lane).  4 waves per SIMD measured
// faster than 3 (6 %) or 5 (18 %, spills).
template <bool BWD, bool SRC, int WPB>
__global__ void __launch_bounds__(WPB * kWave, 4)
persistent_kernel(const EnvP<float>* envs, const BatchEnv* benv, int n_benv,
                  const float* __restrict__ queries, int64_t total_units,
                  uint32_t key0, uint32_t key1, const uint64_t* __restrict__ key_add,
                  unsigned* counter, double* __restrict__ partials)
{
    __shared__ double lds_acc[WPB][kLdsAcc * kWave];
    __shared__ uint32_t pair_lds[WPB][kPairLds];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    double* lds = lds_acc[wv];
    uint32_t* pairs = pair_lds[wv];
    uint32_t k0 = key0, k1 = key1;
    apply_key_add(k0, k1, key_add);
    CBatch* B = (CBatch*)benv;
    const unsigned one = ((threadIdx.x & (kWave - 1)) == 0) ? 1u : 0u;
    // A wave takes at most total_units units, so the loop is bounded even if
    // the counter were wrong.  Every lane issues the atomic (lane 0 adds 1,
    // the others 0): no lane-dependent branch around it, so the loop stays
    // wave-uniform; lane 0's old value is the unit index.
    for (int64_t taken = 0; taken < total_units; ++taken) {
        const unsigned u = __builtin_amdgcn_readfirstlane(atomicAdd(counter, one));
        if ((int64_t)u >= total_units) break;
        // last env whose first unit is <= u (empty envs share the next offset)
        int lo = 0, hi = n_benv - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B[mid].unit_off <= (int64_t)u) lo = mid;
            else hi = mid - 1;
        }
        CBatch& be = B[lo];
        const cenv<float> p = (cenv<float>)(envs + be.slot);
        run_unit<BWD, SRC>(p, be, (int64_t)u - be.unit_off, queries, k0, k1, lds, pairs,
                           partials + (int64_t)u * kNAccBatch);
    }
}

template <bool BWD>
__global__ void __launch_bounds__(kBlock)
finalize_batch(const BatchEnv* __restrict__ benv, const double* __restrict__ partials,
               const float* __restrict__ ubar, float* __restrict__ out_u,
               float* __restrict__ out_grad, int grad_stride, double* __restrict__ out_stats,
               float* __restrict__ out_dx, double* __restrict__ out_dsigma,
               double* __restrict__ out_dg, float* __restrict__ out_dir, unsigned* counter)
{
    __shared__ double s0[kBlock], s1[kBlock];
    const BatchEnv be = benv[blockIdx.x];
    const int d = be.d;
    const double n = (double)be.n_walks;
    double bs = 0.0, bg = 0.0;
    // a thread per query, or, with 64 or more walk ranges per query (one
    // planning start with 1e5 walks has about 800), a wave per query whose
    // lanes stride over the ranges and are then summed across the wave
    const bool by_wave = be.splits >= kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int q0 = by_wave ? (int)(threadIdx.x / kWave) : (int)threadIdx.x;
    const int dq = by_wave ? kBlock / kWave : kBlock;
    for (int ql = q0; ql < be.n_q; ql += dq) {  // wave-uniform when by_wave
        double a[kNAccBatch];
#pragma unroll
        for (int i = 0; i < kNAccBatch; ++i) a[i] = 0.0;
        const double* row = partials + (be.unit_off + (int64_t)ql * be.splits) * kNAccBatch;
        if (by_wave) {
            for (int c = lane; c < be.splits; c += kWave)
#pragma unroll
                for (int i = 0; i < kNAccBatch; ++i) a[i] += row[c * kNAccBatch + i];
#pragma unroll
            for (int i = 0; i < kNAccBatch; ++i) a[i] = wave_sum(a[i]);
            if (lane != 0) continue;
        } else {
            for (int c = 0; c < be.splits; ++c)
#pragma unroll
                for (int i = 0; i < kNAccBatch; ++i) a[i] += row[c * kNAccBatch + i];
        }
        const int64_t qg = be.q_off + ql;
        out_u[qg] = (float)(a[0] / n);
        // partial rows use the 8-wide layout of nacc(kMaxDim)
        constexpr int M = kMaxDim;
        if (out_grad)
#pragma unroll
            for (int i = 0; i < M; ++i) out_grad[qg * grad_stride + i] = (i < d) ? (float)(a[2 + i] / n) : 0.0f;
        if (out_dir) {  // unit direction from the FP64 sums, scaled by the largest entry first
            double m = 0.0, g2 = 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i) m = (i < d) ? ::fmax(m, ::fabs(a[2 + i])) : m;
            if (m > 0.0)
#pragma unroll
                for (int i = 0; i < M; ++i) g2 += (i < d) ? (a[2 + i] / m) * (a[2 + i] / m) : 0.0;
            const double r = (g2 > 0.0) ? 1.0 / ::sqrt(g2) : 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i)
                out_dir[qg * grad_stride + i] = (i < d && m > 0.0) ? (float)((a[2 + i] / m) * r) : 0.0f;
        }
        if (out_stats) {
            double* st = out_stats + qg * kBatchStats;
            st[0] = se_of(a[0], a[1], n);
#pragma unroll
            for (int i = 0; i < M; ++i) st[1 + i] = (i < d) ? se_of(a[2 + i], a[2 + M + i], n) : 0.0;
            st[M + 1] = a[2 + 2 * M] / n;
            st[M + 2] = a[3 + 2 * M];
            st[M + 3] = a[4 + 2 * M];
            st[M + 4] = a[7 + 2 * M] / n;                    // sphere distances per walk
            st[M + 5] = a[8 + 2 * M] / n;                    // box distances per walk
            st[M + 6] = (a[2 + 2 * M] / n) * (double)be.n_cl;  // cluster bounds per walk
            st[M + 7] = a[9 + 2 * M] / n;                    // cluster boxes per walk
        }
        if (BWD) {
            const double ub = (double)ubar[qg];
            bs += ub * (a[5 + 2 * M] / n);
            bg += ub * (a[6 + 2 * M] / n);
#pragma unroll
            for (int i = 0; i < kMaxDim; ++i)
                out_dx[qg * kBatchStride + i] = (i < d) ? (float)(ub * (a[2 + i] / n)) : 0.0f;
        }
    }
    if (BWD) {
        s0[threadIdx.x] = bs;
        s1[threadIdx.x] = bg;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                s0[threadIdx.x] += s0[threadIdx.x + w];
                s1[threadIdx.x] += s1[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out_dsigma[be.slot] = s0[0];
            out_dg[be.slot] = s1[0];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;  // ready for the next launch
}

// ------------------------------------------------------------------------
// Planning update (Sec. III gradient ascent, Sec. VII step rule).
// ------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(kBlock)
plan_update(const EnvP<float>* penv, float* __restrict__ x, int64_t n, const float* __restrict__ dir,
            int grad_stride, float s_ub, double* __restrict__ path_len, int32_t* __restrict__ stalls,
            int32_t* __restrict__ status, uint64_t* step)
{
    __shared__ uint32_t pair_lds[kBlock / kWave][kPairLds];
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const cenv<float> p = (cenv<float>)penv;
    // every lane evaluates the distance (the matrix-core cluster test needs
    // the whole wave); lanes past n use start 0 (or the origin) and write nothing
    const bool valid = s < n;
    const int64_t si = valid ? s : 0;
    float xs[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xs[i] = (n > 0) ? x[si * D + i] : 0.0f;
    int cls;
    WorkCount wc(pair_lds[__builtin_amdgcn_readfirstlane(threadIdx.x / kWave)]);
    const float R = distance<float, D>(p, xs, cls, wc, valid);
    if (valid) {
        float dz2 = 0.0f;
        if (p->has_src) {
#pragma unroll
            for (int i = 0; i < D; ++i) dz2 = Math<float>::fma(xs[i] - p->src_z[i], xs[i] - p->src_z[i], dz2);
        }
        if (R < p->eps) {
            status[s] = (cls == kGoal) ? 1 : 2;
        } else if (p->has_src && dz2 < s_ub * s_ub) {
            status[s] = 1;  // a point-source goal is reached within one nominal step
        } else {
            status[s] = 0;
            float g[D];
            float g2 = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                g[i] = dir[s * grad_stride + i];
                g2 = Math<float>::fma(g[i], g[i], g2);
            }
            if (g2 == 0.0f) {
                stalls[s] += 1;
            } else {
                const float h = Math<float>::min(s_ub, 0.5f * R);
                const float f = h / ::sqrtf(g2);
#pragma unroll
                for (int i = 0; i < D; ++i) x[s * D + i] = Math<float>::fma(f, g[i], xs[i]);
                path_len[s] += (double)h;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
}

// ------------------------------------------------------------------------
// Varadhan read-out (Sec. III, eq. transformation_varadhan): w = -sqrt(t) ln u,
// t = 1 / sigma, grad w = -sqrt(t) grad u / u; u <= 0 (no signal) gives
// w = +inf and grad w = 0.  One thread per query.
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
varadhan_kernel(const T* __restrict__ u, const T* __restrict__ grad, int64_t n, int d, int stride,
                T sqrt_t, T* __restrict__ w, T* __restrict__ grad_w)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const T uq = u[q];
    const bool ok = uq > T(0);
    w[q] = ok ? -sqrt_t * ::log(uq) : Math<T>::inf();
    if (grad_w) {
        const T f = ok ? -sqrt_t / uq : T(0);
        for (int i = 0; i < d; ++i) grad_w[q * stride + i] = f * grad[q * stride + i];
    }
}

__global__ void fill_u32(unsigned* p, int64_t n, unsigned v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_f64(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------
template <typename T, int D, bool BWD, bool SRC>
static void plain_go(unsigned grid, const EnvP<T>* p, const T* queries, int64_t units, int32_t chunks,
                     int64_t n_walks, int64_t w_base, uint32_t q_base, const uint64_t* key_add, double* partials,
                     double* records, hipStream_t st)
{
    hipLaunchKernelGGL((plain_kernel<T, D, BWD, SRC>), dim3(grid), dim3(kBlock), 0, st, p, queries, units, chunks,
                       n_walks, w_base, q_base, key_add, partials, records);
}

template <typename T, int D>
static hipError_t plain_d(bool bwd, bool src, const EnvP<T>* p, const T* queries, int64_t n_q, int64_t n_walks,
                          int64_t w_base, uint32_t q_base, const uint64_t* key_add, double* partials,
                          double* records, hipStream_t st)
{
    const int32_t chunks = (int32_t)((n_walks + kWave - 1) / kWave);
    const int64_t units = n_q * chunks;
    if (units == 0) return hipSuccess;
    const unsigned grid = blocks_for(units, kBlock / kWave);
    if (bwd && src)
        plain_go<T, D, true, true>(grid, p, queries, units, chunks, n_walks, w_base, q_base, key_add, partials, records, st);
    else if (bwd)
        plain_go<T, D, true, false>(grid, p, queries, units, chunks, n_walks, w_base, q_base, key_add, partials, records, st);
    else if (src)
        plain_go<T, D, false, true>(grid, p, queries, units, chunks, n_walks, w_base, q_base, key_add, partials, records, st);
    else
        plain_go<T, D, false, false>(grid, p, queries, units, chunks, n_walks, w_base, q_base, key_add, partials, records, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_plain(int d, bool bwd, bool src, const EnvP<T>* p, const T* queries, int64_t n_q,
                        int64_t n_walks, int64_t w_base, uint32_t q_base, const uint64_t* key_add,
                        double* partials, double* records, hipStream_t st)
{
    switch (d) {
    case 2: return plain_d<T, 2>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 3: return plain_d<T, 3>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 4: return plain_d<T, 4>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 5: return plain_d<T, 5>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 6: return plain_d<T, 6>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 7: return plain_d<T, 7>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    case 8: return plain_d<T, 8>(bwd, src, p, queries, n_q, n_walks, w_base, q_base, key_add, partials, records, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int D>
static hipError_t fin_d(bool bwd, const double* partials, int64_t n_q, int32_t chunks, int64_t n_walks,
                        T* out_u, T* out_grad, double* out_stats, const T* ubar, T* out_dx,
                        double* out_dq, double* prod, hipStream_t st)
{
    if (n_q == 0) return hipSuccess;
    const unsigned grid = (unsigned)n_q;  // one block per query
    if (bwd)
        hipLaunchKernelGGL((finalize_plain<T, D, true>), dim3(grid), dim3(kBlock), 0, st, partials, n_q,
                           chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod);
    else
        hipLaunchKernelGGL((finalize_plain<T, D, false>), dim3(grid), dim3(kBlock), 0, st, partials, n_q,
                           chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize_plain(int d, bool bwd, const double* partials, int64_t n_q, int32_t chunks,
                                 int64_t n_walks, T* out_u, T* out_grad, double* out_stats,
                                 const T* ubar, T* out_dx, double* out_dq, double* prod,
                                 hipStream_t st)
{
    switch (d) {
    case 2: return fin_d<T, 2>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 3: return fin_d<T, 3>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 4: return fin_d<T, 4>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 5: return fin_d<T, 5>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 6: return fin_d<T, 6>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 7: return fin_d<T, 7>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    case 8: return fin_d<T, 8>(bwd, partials, n_q, chunks, n_walks, out_u, out_grad, out_stats, ubar, out_dx, out_dq, prod, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_plain<float>(int, bool, bool, const EnvP<float>*, const float*, int64_t, int64_t,
                                        int64_t, uint32_t, const uint64_t*, double*, double*, hipStream_t);
template hipError_t launch_plain<double>(int, bool, bool, const EnvP<double>*, const double*, int64_t, int64_t,
                                         int64_t, uint32_t, const uint64_t*, double*, double*, hipStream_t);
template hipError_t launch_finalize_plain<float>(int, bool, const double*, int64_t, int32_t, int64_t, float*,
                                                 float*, double*, const float*, float*, double*, double*,
                                                 hipStream_t);
template hipError_t launch_finalize_plain<double>(int, bool, const double*, int64_t, int32_t, int64_t,
                                                  double*, double*, double*, const double*, double*,
                                                  double*, double*, hipStream_t);

hipError_t launch_reduce_pairs(const double* prod, int64_t n, double* out0, double* out1, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_pairs, dim3(1), dim3(kBlock), 0, st, prod, n, out0, out1);
    return hipGetLastError();
}

template <bool BWD, bool SRC>
static hipError_t persistent_go(int grid, int block, const EnvP<float>* envs, const BatchEnv* benv, int n_benv,
                                const float* queries, int64_t total_units, uint32_t key0, uint32_t key1,
                                const uint64_t* key_add, unsigned* counter, double* partials, hipStream_t st)
{
#define WOS_PERSISTENT_CASE(W)                                                                                  \
    case W * kWave:                                                                                             \
        hipLaunchKernelGGL((persistent_kernel<BWD, SRC, W>), dim3(grid), dim3(block), 0, st, envs, benv, n_benv, \
                           queries, total_units, key0, key1, key_add, counter, partials);                       \
        return hipSuccess;
    switch (block) {
        WOS_PERSISTENT_CASE(1)
        WOS_PERSISTENT_CASE(2)
        WOS_PERSISTENT_CASE(4)
    default: return hipErrorInvalidValue;
    }
#undef WOS_PERSISTENT_CASE
}

hipError_t launch_persistent(bool bwd, bool src, int grid, int block, const EnvP<float>* envs,
                             const BatchEnv* benv, int n_benv, const float* queries, int64_t total_units,
                             uint32_t key0, uint32_t key1, const uint64_t* key_add, unsigned* counter,
                             double* partials, hipStream_t st)
{
    if (total_units == 0) return hipSuccess;
    hipError_t e;
    if (bwd && src)
        e = persistent_go<true, true>(grid, block, envs, benv, n_benv, queries, total_units, key0, key1, key_add, counter, partials, st);
    else if (bwd)
        e = persistent_go<true, false>(grid, block, envs, benv, n_benv, queries, total_units, key0, key1, key_add, counter, partials, st);
    else if (src)
        e = persistent_go<false, true>(grid, block, envs, benv, n_benv, queries, total_units, key0, key1, key_add, counter, partials, st);
    else
        e = persistent_go<false, false>(grid, block, envs, benv, n_benv, queries, total_units, key0, key1, key_add, counter, partials, st);
    return e != hipSuccess ? e : hipGetLastError();
}

template <bool BWD, bool SRC>
static int resident_per_cu(int block)
{
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (block) {
    case 1 * kWave: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<BWD, SRC, 1>, block, 0); break;
    case 2 * kWave: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<BWD, SRC, 2>, block, 0); break;
    case 4 * kWave: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<BWD, SRC, 4>, block, 0); break;
    default: break;
    }
    return (e == hipSuccess && per_cu > 0) ? per_cu : 1;
}

int persistent_resident_blocks(bool bwd, bool src, int block)
{
    const int per_cu = (bwd && src) ? resident_per_cu<true, true>(block)
                       : bwd        ? resident_per_cu<true, false>(block)
                       : src        ? resident_per_cu<false, true>(block)
                                    : resident_per_cu<false, false>(block);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return per_cu;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    return per_cu * cus;
}

hipError_t launch_finalize_batch(bool bwd, const BatchEnv* benv, int n_benv, const double* partials,
                                 const float* ubar, float* out_u, float* out_grad,
                                 int grad_stride, double* out_stats, float* out_dx, double* out_dsigma,
                                 double* out_dg, float* out_dir, unsigned* counter, hipStream_t st)
{
    if (n_benv == 0) return hipSuccess;
    if (bwd)
        hipLaunchKernelGGL(finalize_batch<true>, dim3(n_benv), dim3(kBlock), 0, st, benv, partials, ubar, out_u,
                           out_grad, grad_stride, out_stats, out_dx, out_dsigma, out_dg, out_dir, counter);
    else
        hipLaunchKernelGGL(finalize_batch<false>, dim3(n_benv), dim3(kBlock), 0, st, benv, partials, ubar, out_u,
                           out_grad, grad_stride, out_stats, out_dx, out_dsigma, out_dg, out_dir, counter);
    return hipGetLastError();
}

hipError_t launch_plan_update(int d, const EnvP<float>* p, float* x, int64_t n, const float* dir,
                              int grad_stride, float s_ub, double* path_len, int32_t* stalls,
                              int32_t* status, uint64_t* step, hipStream_t st)
{
    const unsigned grid = n > 0 ? blocks_for(n, kBlock) : 1u;
#define WOS_PLAN_CASE(DD)                                                                              \
    case DD:                                                                                           \
        hipLaunchKernelGGL(plan_update<DD>, dim3(grid), dim3(kBlock), 0, st, p, x, n, dir, grad_stride,  \
                           s_ub, path_len, stalls, status, step);                                      \
        break;
    switch (d) {
        WOS_PLAN_CASE(2)
        WOS_PLAN_CASE(3)
        WOS_PLAN_CASE(4)
        WOS_PLAN_CASE(5)
        WOS_PLAN_CASE(6)
        WOS_PLAN_CASE(7)
        WOS_PLAN_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef WOS_PLAN_CASE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_varadhan(const T* u, const T* grad, int64_t n, int d, int stride, double sigma, T* w,
                           T* grad_w, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const T sqrt_t = (T)(1.0 / std::sqrt(sigma));
    hipLaunchKernelGGL((varadhan_kernel<T>), dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, u, grad, n, d,
                       stride, sqrt_t, w, grad_w);
    return hipGetLastError();
}
template hipError_t launch_varadhan<float>(const float*, const float*, int64_t, int, int, double, float*, float*,
                                           hipStream_t);
template hipError_t launch_varadhan<double>(const double*, const double*, int64_t, int, int, double, double*,
                                            double*, hipStream_t);

hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace wos

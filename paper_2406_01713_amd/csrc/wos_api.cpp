// wos_api.cpp -- the C ABI of libwos (include/wos.h): argument checks, device
// copies of the domain, weight-series coefficients, launch decomposition, the
// batched scheduler's work-unit table, the HIP-graph planning loop and the
// launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <limits>
#include <vector>

#include "../../include/wos.h"
#include "wos_launch.hpp"
#include "wos_params.hpp"

using namespace wos;

namespace {

thread_local std::string g_err;

// Outer-box faces of unbounded coordinates (extruded geometry): far enough
// never to be the nearest face, finite in FP32.
constexpr double kFarFace = 1e30;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(WOS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define WOS_HIP(call, what)                       \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool finite_all(const double* p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

struct wos_domain {
    int d = 0;
    int geom_d = 0;  // obstacles and the outer boundary use the first geom_d coordinates
    int64_t n_arm = 0;  // planar arm: task-plane obstacle points (0: no arm)
    double arm_l[kMaxDim] = {0};
    double arm_K = 0;
    float* arm_f = nullptr;
    double* arm_d = nullptr;
    int device = 0;
    int64_t n_sph = 0, n_box = 0;
    float* sph_f = nullptr;
    double* sph_d = nullptr;
    float* box_f = nullptr;
    double* box_d = nullptr;
    bool has_goal = false;
    double goal_c[kMaxDim] = {0};
    double goal_r = 0;
    int outer_kind = 0;
    double lo[kMaxDim] = {0}, hi[kMaxDim] = {0}, oc[kMaxDim] = {0};
    double orad = 0;
    int mode = 0;
    double g_goal = 1, g_obs = 0, g_outer = 0, b = 0;
    double ak[kMaxDim] = {0};
    double r_max = 0;  // largest possible empty-ball radius (bounds sigma R^2 / 4)
    double coord_scale = 0;  // largest coordinate magnitude (plus radius) of the geometry
    // clustered copies of the obstacle tables (see EnvP): one buffer per
    // precision, [sphere rows | sphere bounds | box rows | box bounds]
    int32_t n_cl_sph = 0, n_cl_box = 0;
    bool has_src = false;  // point source amp delta_z
    double src_z[kMaxDim] = {0};
    double src_amp = 0, c_imp = 1;
    float* cl_f = nullptr;
    double* cl_d = nullptr;
    size_t off_sph_bnd = 0, off_box_cl = 0, off_box_bnd = 0;
    size_t off_sph_mf = 0, off_box_mf = 0;  // matrix-core features (FP32 buffer only)
    size_t off_sph_cb = 0, off_box_cb = 0;  // cluster bounding boxes (FP32 buffer only)
};

namespace {

// Horner coefficients c_k = 1 / ((b)_k k!) of 0F1(; b; y) up to the first k
// whose term at y_max falls below tol times the sum (all terms are positive).
int series_coeffs(double b, double y_max, double tol, double* c)
{
    c[0] = 1.0;
    double term = 1.0, sum = 1.0;
    int k = 1;
    for (; k < kMaxTerms; ++k) {
        c[k] = c[k - 1] / ((b + k - 1.0) * (double)k);
        term *= y_max / ((b + k - 1.0) * (double)k);
        sum += term;
        if (term <= tol * sum && (double)k * k > y_max) return k + 1;
        if (y_max == 0.0) return 1;
    }
    return -1;
}

template <typename T>
int make_env(const wos_domain* D, double sigma, double eps, uint64_t seed, uint32_t env_id,
             const wos_options& o, EnvP<T>& p)
{
    std::memset(&p, 0, sizeof(p));
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(WOS_EINVAL, "sigma must be finite and >= 0 (got %g)", sigma);
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(WOS_EINVAL, "eps must be finite and > 0 (got %g)", eps);
    if (D->mode == WOS_BDATA_AFFINE && sigma != 0.0)
        return fail(WOS_ENOTSUP, "affine boundary data solves the equation only at sigma = 0");
    if (D->mode == WOS_BDATA_PLANE) {
        double k2 = 0;
        for (int i = 0; i < D->d; ++i) k2 += D->ak[i] * D->ak[i];
        if (std::fabs(k2 - sigma) > 1e-9 * std::max(1.0, sigma))
            return fail(WOS_ENOTSUP, "plane-wave data needs |k|^2 = sigma (|k|^2 = %g, sigma = %g)", k2, sigma);
    }
    const double y_max = 0.25 * sigma * D->r_max * D->r_max;
    const double tol = sizeof(T) == 4 ? 1e-9 : 1e-18;
    double cC[kMaxTerms], cC1[kMaxTerms];
    const int nC = series_coeffs(0.5 * D->d, y_max, tol, cC);
    const int nC1 = series_coeffs(0.5 * D->d + 1.0, y_max, tol, cC1);
    if (nC < 0 || nC1 < 0)
        return fail(WOS_ENOTSUP, "sigma R_max^2 / 4 = %g needs more than %d series terms", y_max, kMaxTerms);
    // Horner runs on c_k 2^(m k) and y 2^-m: every step is the unscaled one
    // times an exact power of two, so the value is the same bit for bit, and
    // the scaled coefficients stay in T's normal range (unscaled, FP32's c_k
    // leave it from k ~ 20, and at sigma R^2 / 4 ~ 200 the lost terms hold
    // about 1e-3 of the sum).  m: the largest with 2^m <= y_max whose scaled
    // coefficients stay below 2^120 (FP32) or 2^1000 (FP64).
    const double c_lim = std::ldexp(1.0, sizeof(T) == 4 ? 120 : 1000);
    int m = (y_max > 1.0) ? (int)std::floor(std::log2(y_max)) : 0;
    for (; m > 0; --m) {
        bool ok = true;
        for (int k = 0; k < nC && ok; ++k) ok = std::ldexp(cC[k], m * k) <= c_lim;
        for (int k = 0; k < nC1 && ok; ++k) ok = std::ldexp(cC1[k], m * k) <= c_lim;
        if (ok) break;
    }
    p.sph = nullptr;
    p.box = nullptr;
    if (sizeof(T) == 4) {
        p.sph = (const T*)D->sph_f;
        p.box = (const T*)D->box_f;
    } else {
        p.sph = (const T*)D->sph_d;
        p.box = (const T*)D->box_d;
    }
    p.n_sph = (int32_t)D->n_sph;
    p.n_box = (int32_t)D->n_box;
    const bool full = (o.flags & WOS_FULL_SCAN) != 0;
    p.n_cl_sph = full ? 0 : D->n_cl_sph;
    p.n_cl_box = full ? 0 : D->n_cl_box;
    const T* cl = sizeof(T) == 4 ? (const T*)D->cl_f : (const T*)D->cl_d;
    p.sph_cl = cl;
    p.sph_bnd = cl ? cl + D->off_sph_bnd : nullptr;
    p.box_cl = cl ? cl + D->off_box_cl : nullptr;
    p.box_bnd = cl ? cl + D->off_box_bnd : nullptr;
    p.sph_mf = D->cl_f ? D->cl_f + D->off_sph_mf : nullptr;
    p.box_mf = D->cl_f ? D->cl_f + D->off_box_mf : nullptr;
    p.sph_cb = D->cl_f ? D->cl_f + D->off_sph_cb : nullptr;
    p.box_cb = D->cl_f ? D->cl_f + D->off_box_cb : nullptr;
    p.use_mfma = (sizeof(T) != 4 || (o.flags & WOS_SCALAR_CULL)) ? 0 : (o.flags & WOS_WAVE_SCAN) ? 1 : 2;
    p.box_test = (o.flags & WOS_BOX_TEST) ? 1 : (o.flags & WOS_NO_BOX_TEST) ? 0 : D->geom_d >= kBoxTestMinDim;
    // a pair-queue entry holds the cluster index in 26 bits
    if (p.use_mfma == 2 && (D->n_cl_sph >= (1 << 26) || D->n_cl_box >= (1 << 26))) p.use_mfma = 1;
    p.d = D->d;
    p.geom_d = D->geom_d;
    p.pad_g = 0;
    if (D->n_arm > 0) {
        p.arm_pts = sizeof(T) == 4 ? (const T*)D->arm_f : (const T*)D->arm_d;
        p.n_arm = (int32_t)D->n_arm;
        for (int i = 0; i < kMaxDim; ++i) p.arm_l[i] = (T)D->arm_l[i];
        p.arm_invK = (T)(1.0 / D->arm_K);
    }
    p.has_goal = D->has_goal ? 1 : 0;
    p.outer_kind = D->outer_kind;
    p.mode = D->mode;
    p.nt_C = nC;
    p.nt_C1 = nC1;
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    p.env_id = env_id;
    p.max_steps = o.max_steps ? o.max_steps : kDefaultMaxSteps;
    for (int i = 0; i < kMaxDim; ++i) {
        p.goal_c[i] = (T)D->goal_c[i];
        p.lo[i] = (T)D->lo[i];
        p.hi[i] = (T)D->hi[i];
        p.oc[i] = (T)D->oc[i];
        p.ak[i] = (T)D->ak[i];
    }
    p.goal_r = (T)D->goal_r;
    p.orad = (T)D->orad;
    p.g_goal = (T)D->g_goal;
    p.g_obs = (T)D->g_obs;
    p.g_outer = (T)D->g_outer;
    p.b = (T)D->b;
    p.sigma = (T)sigma;
    p.eps = (T)eps;
    // margin of the step-to-step bound R_next <= 2 R: 2^-14 of the geometry's
    // size exceeds the rounding of the positions and of every component's
    // distance (a few units of 2^-24 of that size in FP32) many times over;
    // unbounded (extruded) coordinates let |x| grow without limit, so there
    // the bound is off
    p.rb_abs = D->geom_d == D->d ? (T)(0x1p-14 * (1.0 + D->coord_scale)) : std::numeric_limits<T>::infinity();
    p.qsigma = (T)std::ldexp(0.25 * sigma, -m);
    for (int i = 0; i < kMaxTerms; ++i) {
        p.cC[i] = (T)(i < nC ? std::ldexp(cC[i], m * i) : 0.0);
        p.cC1[i] = (T)(i < nC1 ? std::ldexp(cC1[i], m * i) : 0.0);
    }
    if (D->has_src) {
        // Green's-function constants (see ball_green): nu = d/2 - 1
        const int d = D->d;
        const double nu = 0.5 * d - 1.0, pi = 3.14159265358979323846;
        const double area = 2.0 * std::pow(pi, 0.5 * d) / std::tgamma(0.5 * d);
        p.has_src = 1;
        for (int i = 0; i < d; ++i) p.src_z[i] = (T)D->src_z[i];
        p.src_amp = (T)D->src_amp;
        p.c_imp = (T)D->c_imp;
        p.nu = (T)nu;
        p.sqrt_sigma = (T)std::sqrt(sigma);
        if (sigma > 0.0) {
            p.phi_c = (T)(std::pow(2.0 * pi, -0.5 * d) * std::pow(sigma, 0.5 * nu));
            p.grad_c = (T)(std::pow(2.0 * pi, -0.5 * d) * std::pow(sigma, 0.5 * (nu + 1.0)));
        } else {
            p.phi_c = (T)(d == 2 ? 1.0 / (2.0 * pi) : 1.0 / ((d - 2.0) * area));
            p.grad_c = (T)(1.0 / area);
        }
    }
    return WOS_OK;
}

// Leaves of a k-d split of obstacle centres: the widest axis of the centres
// in idx[lo, hi) is split at a multiple of kCluster near the median, so every
// leaf but the last in order holds exactly kCluster obstacles.
void kd_leaves(const double* c, int d, std::vector<int64_t>& idx, int64_t lo, int64_t hi)
{
    const int64_t n = hi - lo;
    if (n <= kCluster) return;
    double mn[kMaxDim], mx[kMaxDim];
    for (int i = 0; i < d; ++i) {
        mn[i] = INFINITY;
        mx[i] = -INFINITY;
    }
    for (int64_t k = lo; k < hi; ++k)
        for (int i = 0; i < d; ++i) {
            mn[i] = std::min(mn[i], c[idx[k] * d + i]);
            mx[i] = std::max(mx[i], c[idx[k] * d + i]);
        }
    int ax = 0;
    for (int i = 1; i < d; ++i)
        if (mx[i] - mn[i] > mx[ax] - mn[ax]) ax = i;
    std::stable_sort(idx.begin() + lo, idx.begin() + hi,
                     [&](int64_t a, int64_t b) { return c[a * d + ax] < c[b * d + ax]; });
    int64_t half = (int64_t)std::llround((double)n / (2.0 * kCluster)) * kCluster;
    half = std::min(std::max<int64_t>(half, kCluster), n - 1);
    kd_leaves(c, d, idx, lo, lo + half);
    kd_leaves(c, d, idx, lo + half, hi);
}

// Reach of member k of a cluster from centre C: |c_k - C| + r_k (spheres)
// or + |h_k| (boxes).
template <typename T>
double reach(int d, const T* row, bool box, const double* C)
{
    double dc = 0.0, rad = 0.0;
    for (int i = 0; i < d; ++i) {
        const double t = (double)row[i] - C[i];
        dc += t * t;
    }
    if (box) {
        for (int i = 0; i < d; ++i) rad += (double)row[d + i] * (double)row[d + i];
        rad = std::sqrt(rad);
    } else {
        rad = (double)row[d];
    }
    return std::sqrt(dc) + rad;
}

// Centre that (nearly) minimises the bounding radius max_k reach_k(C), a
// convex function of C: from the start point, step towards the member of
// largest reach, keeping a step only when it lowers the maximum and
// shrinking the step otherwise.  Any centre is valid; a smaller radius only
// makes the bound tighter.
template <typename T>
void minimax_centre(int d, const T* rows, int S, bool box, const int64_t* members, int n, double* C)
{
    auto fmax = [&](const double* P, int* arg) {
        double f = -1.0;
        for (int k = 0; k < n; ++k) {
            const double r = reach(d, rows + members[k] * S, box, P);
            if (r > f) {
                f = r;
                *arg = k;
            }
        }
        return f;
    };
    int far = 0;
    double f = fmax(C, &far);
    double step = 0.5 * f;
    for (int it = 0; it < 64 && step > 0.0; ++it) {
        const T* row = rows + members[far] * S;
        double dir[kMaxDim], nrm = 0.0;
        for (int i = 0; i < d; ++i) {
            dir[i] = (double)row[i] - C[i];
            nrm += dir[i] * dir[i];
        }
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) break;
        double P[kMaxDim];
        for (int i = 0; i < d; ++i) P[i] = C[i] + step * dir[i] / nrm;
        int farP = 0;
        const double fP = fmax(P, &farP);
        if (fP < f) {
            for (int i = 0; i < d; ++i) C[i] = P[i];
            f = fP;
            far = farP;
        } else {
            step *= 0.7;
        }
    }
}

// Clustered rows and bounding spheres of one obstacle table in precision T.
// rows: the caller-order table (stride S, values already rounded to T).  The
// bounding radius is computed in FP64 from the rounded centres and radii
// (spheres: r_j; boxes: |h_j|), enlarged by the relative margin 2 m of the
// device bound (m = 2^-16 in FP32, 2^-45 in FP64) plus a tiny absolute term,
// and rounded up to T.
template <typename T>
void build_clusters(int d, int64_t n, bool box, const std::vector<int64_t>& idx, const T* rows, int S,
                    T* cl, T* bnd)
{
    const double m2 = sizeof(T) == 4 ? 0x1p-15 : 0x1p-44;
    const double tiny = sizeof(T) == 4 ? 0x1p-100 : 0x1p-900;
    const int SB = sph_stride(d);
    const int64_t n_cl = (n + kCluster - 1) / kCluster;
    for (int64_t g = 0; g < n_cl; ++g) {
        const int64_t j0 = g * kCluster, j1 = std::min<int64_t>(n, j0 + kCluster);
        double mn[kMaxDim], mx[kMaxDim];
        for (int i = 0; i < d; ++i) {
            mn[i] = INFINITY;
            mx[i] = -INFINITY;
        }
        for (int64_t k = j0; k < j0 + kCluster; ++k) {
            T* out = cl + k * S;
            if (k < j1) {
                const T* in = rows + idx[k] * S;
                for (int i = 0; i < S; ++i) out[i] = in[i];
                for (int i = 0; i < d; ++i) {
                    mn[i] = std::min(mn[i], (double)in[i]);
                    mx[i] = std::max(mx[i], (double)in[i]);
                }
            } else {
                // padding: a point obstacle far outside any domain
                for (int i = 0; i < S; ++i) out[i] = T(0);
                for (int i = 0; i < d; ++i) out[i] = T(1e18);
            }
        }
        T* b = bnd + g * SB;
        for (int i = 0; i < SB; ++i) b[i] = T(0);
        double C[kMaxDim];
        for (int i = 0; i < d; ++i) C[i] = 0.5 * (mn[i] + mx[i]);
        minimax_centre(d, rows, S, box, idx.data() + j0, (int)(j1 - j0), C);
        for (int i = 0; i < d; ++i) b[i] = (T)C[i];
        double rho = 0.0;
        double Cr[kMaxDim];
        for (int i = 0; i < d; ++i) Cr[i] = (double)b[i];  // the centre as stored
        for (int64_t k = j0; k < j1; ++k) rho = std::max(rho, reach(d, rows + idx[k] * S, box, Cr));
        const double want = rho * (1.0 + m2) + tiny;
        T r = (T)want;
        if ((double)r < want) r = std::nextafter(r, std::numeric_limits<T>::infinity());
        b[d] = r;
    }
}

// Bounding boxes of the clusters (FP32 kernels, see kClusterBox) from the
// caller-order FP32 rows, in cluster order: per cluster lo[kMaxDim] then
// hi[kMaxDim], the box of its members (centres -+ radius, or -+ half-widths)
// enlarged by delta = 2^-16 times its diagonal (plus a tiny absolute term) on
// every side, computed in FP64 and rounded outwards to FP32.  The margin
// covers the rounding of the kernel's box and member distances (see
// box_round); padding rows of the last cluster are not members.
void build_cluster_boxes(int d, int64_t n, bool box, const std::vector<int64_t>& idx, const float* rows, int S,
                         float* out)
{
    const int64_t n_cl = (n + kCluster - 1) / kCluster;
    for (int64_t g = 0; g < n_cl; ++g) {
        const int64_t j0 = g * kCluster, j1 = std::min<int64_t>(n, j0 + kCluster);
        double lo[kMaxDim], hi[kMaxDim];
        for (int i = 0; i < d; ++i) {
            lo[i] = INFINITY;
            hi[i] = -INFINITY;
        }
        for (int64_t k = j0; k < j1; ++k) {
            const float* row = rows + idx[k] * S;
            for (int i = 0; i < d; ++i) {
                const double ext = box ? (double)row[d + i] : (double)row[d];
                lo[i] = std::min(lo[i], (double)row[i] - ext);
                hi[i] = std::max(hi[i], (double)row[i] + ext);
            }
        }
        double diag = 0.0;
        for (int i = 0; i < d; ++i) diag += (hi[i] - lo[i]) * (hi[i] - lo[i]);
        const double delta = std::sqrt(diag) * 0x1p-16 + 0x1p-100;
        float* o = out + g * kClusterBox;
        for (int i = 0; i < kClusterBox; ++i) o[i] = 0.0f;
        for (int i = 0; i < d; ++i) {
            const double l = lo[i] - delta, h = hi[i] + delta;
            float lf = (float)l, hf = (float)h;
            if ((double)lf > l) lf = std::nextafter(lf, -std::numeric_limits<float>::infinity());
            if ((double)hf < h) hf = std::nextafter(hf, std::numeric_limits<float>::infinity());
            o[i] = lf;
            o[kMaxDim + i] = hf;
        }
    }
}

int check_obstacles(int d, const wos_spheres* spheres, const wos_boxes* boxes)
{
    const int64_t ns = spheres ? spheres->n : 0, nb = boxes ? boxes->n : 0;
    if (ns < 0 || nb < 0 || ns > (1 << 24) || nb > (1 << 24)) return fail(WOS_EINVAL, "bad obstacle counts");
    if (ns > 0 && (!spheres->centers || !spheres->radii)) return fail(WOS_EINVAL, "sphere arrays are NULL");
    if (nb > 0 && (!boxes->centers || !boxes->half_widths)) return fail(WOS_EINVAL, "box arrays are NULL");
    if (ns > 0 && (!finite_all(spheres->centers, ns * d) || !finite_all(spheres->radii, ns)))
        return fail(WOS_EINVAL, "non-finite sphere data");
    if (nb > 0 && (!finite_all(boxes->centers, nb * d) || !finite_all(boxes->half_widths, nb * d)))
        return fail(WOS_EINVAL, "non-finite box data");
    for (int64_t j = 0; j < ns; ++j)
        if (spheres->radii[j] < 0) return fail(WOS_EINVAL, "negative sphere radius");
    for (int64_t j = 0; j < nb * d; ++j)
        if (boxes->half_widths[j] < 0) return fail(WOS_EINVAL, "negative box half-width");
    return WOS_OK;
}

// Caller-order device rows of the obstacle tables in FP32 and FP64.
void obstacle_rows(int d, const wos_spheres* spheres, const wos_boxes* boxes, std::vector<float>& sf,
                   std::vector<double>& sd, std::vector<float>& bf, std::vector<double>& bd)
{
    const int64_t ns = spheres ? spheres->n : 0, nb = boxes ? boxes->n : 0;
    const int ss = sph_stride(d), bs = box_stride(d);
    sf.assign((size_t)std::max<int64_t>(ns, 1) * ss, 0.f);
    sd.assign((size_t)std::max<int64_t>(ns, 1) * ss, 0.0);
    for (int64_t j = 0; j < ns; ++j) {
        for (int i = 0; i < d; ++i) {
            sd[j * ss + i] = spheres->centers[j * d + i];
            sf[j * ss + i] = (float)spheres->centers[j * d + i];
        }
        sd[j * ss + d] = spheres->radii[j];
        sf[j * ss + d] = (float)spheres->radii[j];
    }
    bf.assign((size_t)std::max<int64_t>(nb, 1) * bs, 0.f);
    bd.assign((size_t)std::max<int64_t>(nb, 1) * bs, 0.0);
    for (int64_t j = 0; j < nb; ++j) {
        for (int i = 0; i < d; ++i) {
            bd[j * bs + i] = boxes->centers[j * d + i];
            bf[j * bs + i] = (float)boxes->centers[j * d + i];
            bd[j * bs + d + i] = boxes->half_widths[j * d + i];
            bf[j * bs + d + i] = (float)boxes->half_widths[j * d + i];
        }
    }
}

// Cluster order of n obstacles (k-d leaves of kCluster), or none below
// kClusterMin; returns the number of clusters.
int64_t cluster_order(int d, int64_t n, const double* centers, std::vector<int64_t>& idx)
{
    idx.clear();
    if (n < kClusterMin) return 0;
    idx.resize(n);
    for (int64_t j = 0; j < n; ++j) idx[j] = j;
    kd_leaves(centers, d, idx, 0, n);
    return (n + kCluster - 1) / kCluster;
}

// Matrix-core cluster features (see kMfmaTile) from the FP32 bound rows:
// out holds ceil(n_cl / 16) + 1 tiles of 64 x 4 floats, the last a spare
// all-skip tile that the kernel reads ahead into and never tests.
void build_mfma_features(int d, int64_t n_cl, const float* bnd, float* out)
{
    const int SB = sph_stride(d);
    const double m = 0x1p-12;
    const int64_t n_tiles = (n_cl + kMfmaTile - 1) / kMfmaTile + 1;  // + the spare tile
    for (int64_t t = 0; t < n_tiles; ++t)
        for (int lane = 0; lane < 64; ++lane) {
            const int j = lane % kMfmaTile, k = lane / kMfmaTile;
            const int64_t g = t * kMfmaTile + j;
            double f[kMfmaFeat];
            if (g < n_cl) {
                const float* b = bnd + g * SB;
                double cc = 0.0;
                for (int i = 0; i < d; ++i) cc += (double)b[i] * (double)b[i];
                const double rho = (double)b[d];
                for (int i = 0; i < 8; ++i) f[i] = i < d ? -2.0 * (double)b[i] : 0.0;
                f[8] = 1.0;
                f[9] = cc * (1.0 - m) - rho * rho * (1.0 + m);
                f[10] = -1.0;
                f[11] = -2.0 * rho;
            } else {
                for (int i = 0; i < kMfmaFeat; ++i) f[i] = 0.0;
                f[9] = 1e30;  // always skipped
            }
            float* o = out + (t * 64 + lane) * 4;
            for (int s = 0; s < 3; ++s) o[s] = (float)f[4 * s + k];
            o[3] = 0.0f;
        }
}

int check_device(const wos_domain* D)
{
    int dev = -1;
    WOS_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != D->device) return fail(WOS_EINVAL, "domain lives on device %d, current device is %d", D->device, dev);
    return WOS_OK;
}

int read_opts(const wos_options* opt, wos_options& o)
{
    o = wos_options{WOS_FP32, 0u, 0u, 0u};
    if (opt) o = *opt;
    if ((o.flags & WOS_BOX_TEST) && (o.flags & WOS_NO_BOX_TEST))
        return fail(WOS_EINVAL, "WOS_BOX_TEST and WOS_NO_BOX_TEST together");
    if (o.flags & ~(WOS_FP64 | WOS_FULL_SCAN | WOS_SCALAR_CULL | WOS_WAVE_SCAN | WOS_OUT_FP64 | WOS_NO_BOX_TEST |
                    WOS_BOX_TEST))
        return fail(WOS_EINVAL, "unknown flags 0x%x", o.flags);
    if (o.reserved != 0) return fail(WOS_EINVAL, "wos_options.reserved must be 0");
    return WOS_OK;
}

// Device scratch allocated in stream order and freed the same way; where the
// device has no stream-ordered allocator, plain allocations are freed after
// the stream drains.
struct Scratch {
    std::vector<void*> ptrs;
    hipStream_t st;
    bool sync_free = false;
    explicit Scratch(hipStream_t s) : st(s) {}
    template <typename T>
    int get(T** p, size_t n)
    {
        *p = nullptr;
        if (n == 0) n = 1;
        hipError_t e = sync_free ? hipErrorNotSupported : hipMallocAsync((void**)p, n * sizeof(T), st);
        if (e == hipErrorNotSupported) {
            (void)hipGetLastError();
            sync_free = true;
            e = hipMalloc((void**)p, n * sizeof(T));
        }
        if (e != hipSuccess) return fail(WOS_ENOMEM, "device scratch of %zu bytes: %s", n * sizeof(T), hipGetErrorString(e));
        ptrs.push_back((void*)*p);
        return WOS_OK;
    }
    ~Scratch()
    {
        if (sync_free) {
            (void)hipStreamSynchronize(st);
            for (void* p : ptrs) (void)hipFree(p);
        } else {
            for (void* p : ptrs) (void)hipFreeAsync(p, st);
        }
    }
};

// Pinned staging of host tables for asynchronous upload; the next upload waits
// for the previous copy to finish before reusing the buffer.
struct Staging {
    std::mutex mu;
    void* buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
Staging g_stage;

int upload(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_stage.mu);
    if (g_stage.pending) {
        WOS_HIP(hipEventSynchronize(g_stage.ev), "staging wait");
        g_stage.pending = false;
    }
    if (!g_stage.ev) WOS_HIP(hipEventCreateWithFlags(&g_stage.ev, hipEventDisableTiming), "hipEventCreate");
    if (bytes > g_stage.cap) {
        if (g_stage.buf) (void)hipHostFree(g_stage.buf);
        g_stage.buf = nullptr;
        g_stage.cap = 0;
        hipError_t e = hipHostMalloc(&g_stage.buf, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return fail(WOS_ENOMEM, "pinned staging of %zu bytes", bytes);
        g_stage.cap = bytes;
    }
    std::memcpy(g_stage.buf, src, bytes);
    WOS_HIP(hipMemcpyAsync(dst, g_stage.buf, bytes, hipMemcpyHostToDevice, st), "upload");
    WOS_HIP(hipEventRecord(g_stage.ev, st), "hipEventRecord");
    g_stage.pending = true;
    return WOS_OK;
}

// ------------------------------------------------------------------------
// Autotune cache: launch shapes of the persistent kernel keyed by the batch
// mix (the multiset of its environments' dimension and log2 buckets of
// obstacle, query and walk counts) or, from the synthetic single-scene
// tuner, by the (d, obstacle bucket, query bucket) of the heaviest env.
// ------------------------------------------------------------------------
struct Tune {
    int units_per_wave = 4;
    int grid_mult = 1;
    int walks_per_lane = 2;   // least walks per lane in a work unit (lane refill needs 2)
    int waves_per_block = 4;  // block of 64, 128 or 256 threads
    int lanes_per_walker = 1; // 64 / walks a wave carries at once (1, 2, 4, ..., 64)
};
std::mutex g_tune_mu;
std::map<std::string, Tune, std::less<>> g_tune;  // transparent: lookups by char* allocate nothing
bool g_tune_loaded = false;
std::string g_tune_path;

int log2_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

void tune_key(char (&k)[48], int d, int64_t M, int64_t Q)
{
    snprintf(k, sizeof(k), "d%d_m%d_q%d", d, log2_bucket(std::max<int64_t>(M, 1)), log2_bucket(std::max<int64_t>(Q, 1)));
}

uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

bool valid_tune(const Tune& t)
{
    return t.units_per_wave > 0 && t.units_per_wave <= 64 && t.grid_mult > 0 && t.grid_mult <= 8 &&
           t.walks_per_lane > 0 && t.walks_per_lane <= 64 &&
           (t.waves_per_block == 1 || t.waves_per_block == 2 || t.waves_per_block == 4) &&
           t.lanes_per_walker > 0 && t.lanes_per_walker <= kWave && (t.lanes_per_walker & (t.lanes_per_walker - 1)) == 0;
}

void load_tune_locked(const char* path)
{
    g_tune.clear();
    g_tune_loaded = true;
    g_tune_path = path ? path : "";
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[320];
    while (fgets(line, sizeof(line), f)) {
        char key[64];
        Tune t;
        // one entry per line: "key": {"units_per_wave": U, "grid_mult": G,
        // "walks_per_lane": W, "waves_per_block": B, "lanes_per_walker": L}
        // (W, B, L absent in older files: 2, 4, 1)
        const int n = sscanf(line,
                             " \"%63[^\"]\": {\"units_per_wave\": %d, \"grid_mult\": %d, \"walks_per_lane\": %d, "
                             "\"waves_per_block\": %d, \"lanes_per_walker\": %d}",
                             key, &t.units_per_wave, &t.grid_mult, &t.walks_per_lane, &t.waves_per_block,
                             &t.lanes_per_walker);
        if (n < 4) t.walks_per_lane = 2;
        if (n < 5) t.waves_per_block = 4;
        if (n < 6) t.lanes_per_walker = 1;
        if (n >= 3 && valid_tune(t)) g_tune[key] = t;
    }
    fclose(f);
}

// The batch mix's entry, else the heaviest env's bucket, else the defaults.
Tune lookup_tune(const char* mix, int d, int64_t M, int64_t Q)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_locked(getenv("WOS_AUTOTUNE_CACHE"));
    auto it = g_tune.find(mix);
    if (it != g_tune.end()) return it->second;
    char k[48];
    tune_key(k, d, M, Q);
    it = g_tune.find(k);
    if (it != g_tune.end()) return it->second;
    return Tune{};
}

int save_tune_locked(const char* path)
{
    FILE* f = fopen(path, "w");
    if (!f) return fail(WOS_EINVAL, "cannot write autotune cache %s", path);
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : g_tune) {
        fprintf(f, "  \"%s\": {\"units_per_wave\": %d, \"grid_mult\": %d, \"walks_per_lane\": %d, "
                   "\"waves_per_block\": %d, \"lanes_per_walker\": %d}%s\n",
                kv.first.c_str(), kv.second.units_per_wave, kv.second.grid_mult, kv.second.walks_per_lane,
                kv.second.waves_per_block, kv.second.lanes_per_walker, (++i < g_tune.size()) ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return WOS_OK;
}

// Relative cost of one work unit of an env: obstacle work per walk step
// times a typical walk length times the walks of the unit.
double unit_cost(const wos_domain* D, int64_t wps)
{
    static const double steps[9] = {0, 0, 12, 25, 40, 55, 71, 85, 95};
    const int d = D->d;
    const double per_step = (double)D->n_sph * (2 * d + 3) + (double)D->n_box * (5 * d + 4) +
                            (double)D->n_arm * d * 12 + 150.0 * ((d + 3) / 4);
    return per_step * steps[d] * (double)wps;
}

// Key of a batch mix: the sum over envs of a hash of (d, log2 buckets of
// obstacles, queries and walks, point source), so the order of the envs does
// not matter and nothing is allocated.
void mix_key(char (&k)[48], const wos_domain* const* envs, const int64_t* q_off, int n_envs, const int64_t* n_walks)
{
    uint64_t h = 0;
    for (int e = 0; e < n_envs; ++e) {
        const wos_domain* D = envs[e];
        const uint64_t v = (uint64_t)D->d | ((uint64_t)log2_bucket(std::max<int64_t>(D->n_sph + D->n_box + D->n_arm, 1)) << 8) |
                           ((uint64_t)log2_bucket(std::max<int64_t>(q_off[e + 1] - q_off[e], 1)) << 16) |
                           ((uint64_t)log2_bucket(n_walks[e]) << 24) | ((uint64_t)(D->has_src ? 1 : 0) << 32);
        h += mix64(v);
    }
    snprintf(k, sizeof(k), "mix_%d_%016llx", n_envs, (unsigned long long)h);
}

struct BatchLayout {
    int64_t total_units = 0;
    int grid = 0;
    int block = 256;
};

// Work units: each query's walks are split into `splits` ranges so that the
// launch has about units_per_wave units per resident wave; envs are ordered
// by decreasing unit cost (longest-processing-time first, ties in caller
// order).  order (n_envs ints) is working storage; benv receives the
// n_envs rows of the unit table.  force: launch-shape fields > 0 override
// the tuned ones.
void plan_batch(const wos_domain* const* envs, const int64_t* q_off, int n_envs, const int64_t* n_walks,
                int q_stride, const Tune* force, bool full_scan, bool src, int* order, BatchEnv* benv,
                BatchLayout& L)
{
    int64_t sumQW = 0, maxM = 0, heavyQ = 0, maxW = 1;
    int heavy_d = 2;
    double heavy = -1;
    for (int e = 0; e < n_envs; ++e) {
        const int64_t q = q_off[e + 1] - q_off[e];
        sumQW += q * n_walks[e];
        maxW = std::max(maxW, n_walks[e]);
        const double c = unit_cost(envs[e], n_walks[e]) * (double)q;
        if (c > heavy) {
            heavy = c;
            heavy_d = envs[e]->d;
            maxM = envs[e]->n_sph + envs[e]->n_box;
            heavyQ = q;
        }
    }
    char mk[48];
    mix_key(mk, envs, q_off, n_envs, n_walks);
    Tune t = lookup_tune(mk, heavy_d, maxM, heavyQ);
    if (force && force->units_per_wave > 0) t.units_per_wave = force->units_per_wave;
    if (force && force->grid_mult > 0) t.grid_mult = force->grid_mult;
    if (force && force->walks_per_lane > 0) t.walks_per_lane = force->walks_per_lane;
    if (force && force->waves_per_block > 0) t.waves_per_block = force->waves_per_block;
    if (force && force->lanes_per_walker > 0) t.lanes_per_walker = force->lanes_per_walker;
    // walks a wave carries at once; the other lanes only share the member
    // scans of those walks (the pair rounds spread over all 64 lanes)
    const int64_t lanes = kWave / t.lanes_per_walker;
    const int block = t.waves_per_block * kWave;
    const int resident_blocks = persistent_resident_blocks(true, src, block);
    L.block = block;
    L.grid = std::max(1, resident_blocks * t.grid_mult);
    const int64_t waves = (int64_t)L.grid * (block / kWave);
    const int64_t target = waves * t.units_per_wave;
    // one walk-range length for the launch: total walks / target units, a
    // multiple of the walk-carrying lanes, at least walks_per_lane walks per
    // such lane
    // (default 2, so lanes refill).  Measured: on the 7-D planning step
    // (524288 walks, 4096 resident waves) 2 per lane beat 4 by 25 % (half the
    // waves had been idle) and 1 by 7 %; on one-start planning with 1e5 walks
    // 2 beat 1 by 5-20 % (a wave with one walk per lane waits for its longest
    // of 64 walks).
    int64_t wps = std::max<int64_t>((int64_t)t.walks_per_lane * lanes, sumQW / std::max<int64_t>(target, 1));
    wps = std::min(wps, maxW);
    wps = ((wps + lanes - 1) / lanes) * lanes;

    auto env_wps = [&](int e) { return std::min<int64_t>(wps, ((n_walks[e] + lanes - 1) / lanes) * lanes); };
    auto cost = [&](int e) {
        return q_off[e + 1] > q_off[e] ? unit_cost(envs[e], env_wps(e)) : -1.0;
    };
    for (int e = 0; e < n_envs; ++e) order[e] = e;
    // std::sort with the caller index as tie-break: the order of a stable
    // sort, without the temporary buffer std::stable_sort allocates
    std::sort(order, order + n_envs, [&](int a, int b) {
        const double ca = cost(a), cb = cost(b);
        return ca > cb || (ca == cb && a < b);
    });
    int64_t uoff = 0;
    for (int i = 0; i < n_envs; ++i) {
        const int e = order[i];
        BatchEnv& b = benv[i];
        const int64_t w = env_wps(e);
        const int64_t splits = (n_walks[e] + w - 1) / w;
        b.q_off = q_off[e];
        b.n_q = (int32_t)(q_off[e + 1] - q_off[e]);
        b.n_walks = n_walks[e];
        b.splits = (int32_t)splits;
        b.wps = (int32_t)w;
        b.d = envs[e]->d;
        b.q_stride = q_stride;
        b.slot = e;
        b.n_cl = full_scan ? 0 : envs[e]->n_cl_sph + envs[e]->n_cl_box;
        b.lanes = (int32_t)lanes;
        b.unit_off = uoff;
        uoff += (int64_t)b.n_q * splits;
    }
    L.total_units = uoff;
}

}  // namespace

// ----------------------------------------------------------------------------
// Scratch of wos_estimate_batch_noalloc: one array per device, reserved when
// the library's device code loads there and held until the process ends.  In
// host code its name is only a stand-in: the device address comes from
// hipGetSymbolAddress, resolved once per device with that device current.
// Layout per call: [work-unit counter | env and unit tables | partial sums],
// each part 256-byte aligned.
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[WOS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocMaxDevices = 64;
constexpr size_t kNoAllocHostBytes =
    (size_t)WOS_NOALLOC_MAX_ENVS * (sizeof(EnvP<float>) + sizeof(BatchEnv));

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Host side of the no-allocation call: the device addresses of `scratch`,
// one upload event per device, and static host staging for the tables (the
// next call waits for the previous upload before rewriting it).  The mutex
// serialises callers on the host; calls that overlap on one device's streams
// still share that device's array.
struct NoAlloc {
    std::mutex mu;
    unsigned char* dev[kNoAllocMaxDevices] = {};
    hipEvent_t ev[kNoAllocMaxDevices] = {};
    hipEvent_t pending = nullptr;
};
NoAlloc g_na;
alignas(256) unsigned char g_na_host[kNoAllocHostBytes];
int g_na_order[WOS_NOALLOC_MAX_ENVS];

// Set-up on the current device, once: resolve the array's device address
// and create the upload event.
int noalloc_setup(int dev)
{
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(WOS_EINVAL, "device %d: the no-allocation call supports devices 0..%d", dev, kNoAllocMaxDevices - 1);
    if (g_na.dev[dev]) return WOS_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    e = hipEventCreateWithFlags(&g_na.ev[dev], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "scratch upload event");
    g_na.dev[dev] = (unsigned char*)ptr;
    return WOS_OK;
}

// Batched launch.  fixed = false: tables and partial sums in stream-ordered
// device allocations.  fixed = true: everything in the device's `scratch`
// array, nothing allocated (wos_estimate_batch_noalloc).
int run_batch(const wos_domain* const* envs, int n_envs, const float* queries, const int64_t* q_offsets,
              const double* sigma, const double* eps, const int64_t* n_walks, uint64_t seed, float* out_u,
              float* out_grad, double* out_stats, const float* grad_u, float* out_dx, double* out_dsigma,
              double* out_dg, const wos_options* opt, hipStream_t st, const Tune* force, bool fixed)
{
    wos_options o;
    int rc = read_opts(opt, o);
    if (rc) return rc;
    if (o.flags & WOS_FP64) return fail(WOS_ENOTSUP, "the batched kernel computes in FP32 only");
    if (o.flags & WOS_OUT_FP64) return fail(WOS_ENOTSUP, "WOS_OUT_FP64 applies to wos_estimate only");
    if (n_envs < 0 || (n_envs > 0 && (!envs || !q_offsets || !sigma || !eps || !n_walks)))
        return fail(WOS_EINVAL, "envs, q_offsets, sigma, eps and n_walks are required");
    if (n_envs == 0) return WOS_OK;
    if (fixed && n_envs > WOS_NOALLOC_MAX_ENVS)
        return fail(WOS_EINVAL, "%d environments: the no-allocation call takes at most %d", n_envs,
                    WOS_NOALLOC_MAX_ENVS);
    for (int e = 0; e < n_envs; ++e)
        if (n_walks[e] < 1 || n_walks[e] > (int64_t)1 << 31) return fail(WOS_EINVAL, "n_walks[%d] must be in [1, 2^31]", e);
    if (q_offsets[0] != 0) return fail(WOS_EINVAL, "q_offsets[0] must be 0");
    for (int e = 0; e < n_envs; ++e) {
        if (!envs[e]) return fail(WOS_EINVAL, "envs[%d] is NULL", e);
        if (q_offsets[e + 1] < q_offsets[e]) return fail(WOS_EINVAL, "q_offsets must be non-decreasing");
        // a query's index is a 32-bit Philox counter word and an int32 count
        if (q_offsets[e + 1] - q_offsets[e] > INT32_MAX)
            return fail(WOS_EINVAL, "env %d has more than 2^31 - 1 queries", e);
        if ((rc = check_device(envs[e]))) return rc;
    }
    const int64_t sumQ = q_offsets[n_envs];
    if (sumQ > 0 && (!queries || !out_u)) return fail(WOS_EINVAL, "queries and out_u are required");
    const bool bwd = grad_u != nullptr;
    if (bwd && (!out_dx || !out_dsigma || !out_dg))
        return fail(WOS_EINVAL, "out_dx, out_dsigma and out_dg are required with grad_u");

    // host tables, contiguous: [EnvP x n_envs][BatchEnv x n_envs]
    const size_t env_bytes = (size_t)n_envs * sizeof(EnvP<float>);
    const size_t tab_bytes = env_bytes + (size_t)n_envs * sizeof(BatchEnv);
    std::unique_lock<std::mutex> na_lock;
    std::vector<unsigned char> host_vec;
    std::vector<int> order_vec;
    unsigned char* host_tab;
    int* order;
    int dev = 0;
    if (fixed) {
        na_lock = std::unique_lock<std::mutex>(g_na.mu);
        WOS_HIP(hipGetDevice(&dev), "hipGetDevice");
        if ((rc = noalloc_setup(dev))) return rc;
        if (g_na.pending) {  // the previous call's upload still reads the staging
            WOS_HIP(hipEventSynchronize(g_na.pending), "staging wait");
            g_na.pending = nullptr;
        }
        host_tab = g_na_host;
        order = g_na_order;
    } else {
        host_vec.resize(tab_bytes);
        order_vec.resize(n_envs);
        host_tab = host_vec.data();
        order = order_vec.data();
    }
    EnvP<float>* hp = reinterpret_cast<EnvP<float>*>(host_tab);
    BatchEnv* hb = reinterpret_cast<BatchEnv*>(host_tab + env_bytes);
    bool src = false;
    for (int e = 0; e < n_envs; ++e) {
        if ((rc = make_env<float>(envs[e], sigma[e], eps[e], seed, (uint32_t)e, o, hp[e]))) return rc;
        src = src || envs[e]->has_src;
        if (bwd && envs[e]->has_src && !(sigma[e] > 0.0))
            return fail(WOS_ENOTSUP, "env %d: the sigma derivative of a point source is provided for sigma > 0 only", e);
    }

    BatchLayout L;
    plan_batch(envs, q_offsets, n_envs, n_walks, kBatchStride, force, (o.flags & WOS_FULL_SCAN) != 0, src, order, hb,
               L);
    // the kernel hands out units with a 32-bit device counter
    if (L.total_units >= ((int64_t)1 << 32) - 1)
        return fail(WOS_EINVAL, "the batch splits into %lld work units; at most 2^32 - 2", (long long)L.total_units);
    const size_t part_bytes = (size_t)std::max<int64_t>(L.total_units, 1) * nacc(kMaxDim) * sizeof(double);

    Scratch S(st);
    unsigned char* d_tab;
    double* partials;
    unsigned* counter;
    if (fixed) {
        const size_t off_tab = 256, off_part = align256(off_tab + tab_bytes);
        const size_t need = off_part + part_bytes;
        if (need > (size_t)WOS_NOALLOC_SCRATCH_BYTES)
            return fail(WOS_EINVAL,
                        "the batch needs %zu bytes of scratch (%lld work units); the no-allocation call holds %zu",
                        need, (long long)L.total_units, (size_t)WOS_NOALLOC_SCRATCH_BYTES);
        unsigned char* base = g_na.dev[dev];
        counter = reinterpret_cast<unsigned*>(base);
        d_tab = base + off_tab;
        partials = reinterpret_cast<double*>(base + off_part);
        WOS_HIP(hipMemcpyAsync(d_tab, host_tab, tab_bytes, hipMemcpyHostToDevice, st), "table upload");
        WOS_HIP(hipEventRecord(g_na.ev[dev], st), "hipEventRecord");
        g_na.pending = g_na.ev[dev];
    } else {
        if ((rc = S.get(&d_tab, tab_bytes)) || (rc = S.get(&partials, part_bytes / sizeof(double))) ||
            (rc = S.get(&counter, 1)))
            return rc;
        if ((rc = upload(d_tab, host_tab, tab_bytes, st))) return rc;
    }
    const EnvP<float>* d_env = (const EnvP<float>*)d_tab;
    const BatchEnv* d_benv = (const BatchEnv*)(d_tab + env_bytes);
    // the counter starts at 0 (a fill kernel: no memset node if the caller captures)
    WOS_HIP(launch_fill_u32(counter, 1, 0u, st), "fill");
    WOS_HIP(launch_persistent(bwd, src, L.grid, L.block, d_env, d_benv, n_envs, queries, L.total_units,
                              (uint32_t)seed, (uint32_t)(seed >> 32), nullptr, counter, partials, st),
            "persistent walk kernel");
    WOS_HIP(launch_finalize_batch(bwd, d_benv, n_envs, partials, grad_u, out_u, out_grad, kBatchStride,
                                  out_stats, out_dx, out_dsigma, out_dg, nullptr, counter, st),
            "batch finalize");
    return WOS_OK;
}

// Launch-shape search on a batch: the persistent launch (forward + backward
// with u-bar = 1 when fused) timed with HIP events for shapes reached by
// coordinate descent from the built-in shape.  Each of waves per block,
// units per wave, grid multiple and walks per lane in turn runs over its
// candidate values with the others held; a shape replaces the best only when
// it is faster by more than 0.5 % (launch times repeat to about 0.1 %), and a
// second pass runs when the first moved.  One untimed launch comes first.
// Output buffers are allocated here (this is a set-up call).
struct TuneRun {
    Tune best;
    double ms_default = 0.0, ms_best = 0.0;
    int tried = 0;
};

int tune_batch(const wos_domain* const* envs, int n_envs, const float* queries, const int64_t* q_off,
               const double* sigma, const double* eps, const int64_t* n_walks, uint64_t seed, bool fused,
               TuneRun& out)
{
    const int64_t sumQ = q_off[n_envs];
    if (sumQ < 1) return fail(WOS_EINVAL, "the batch has no queries");
    float *du = nullptr, *dg = nullptr, *dub = nullptr, *ddx = nullptr;
    double *dds = nullptr, *ddg = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&du, sumQ * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&dg, sumQ * kBatchStride * sizeof(float));
    if (e == hipSuccess && fused) e = hipMalloc(&dub, sumQ * sizeof(float));
    if (e == hipSuccess && fused) e = hipMalloc(&ddx, sumQ * kBatchStride * sizeof(float));
    if (e == hipSuccess && fused) e = hipMalloc(&dds, n_envs * sizeof(double));
    if (e == hipSuccess && fused) e = hipMalloc(&ddg, n_envs * sizeof(double));
    if (e == hipSuccess && fused) e = launch_fill_u32((unsigned*)dub, sumQ, 0x3f800000u, st);  // u-bar = 1.0f
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = WOS_OK;
    auto time_one = [&](const Tune& t, double& ms) {
        if (e != hipSuccess || rc) return;
        e = hipEventRecord(e0, st);
        if (e == hipSuccess)
            rc = run_batch(envs, n_envs, queries, q_off, sigma, eps, n_walks, seed, du, dg, nullptr, dub, ddx, dds,
                           ddg, nullptr, st, &t, false);
        if (e == hipSuccess && !rc) e = hipEventRecord(e1, st);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
        float f = 0.0f;
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&f, e0, e1);
        ms = f;
    };
    Tune cur;
    double best_ms = 0.0, ms = 0.0;
    time_one(cur, ms);  // untimed: first launch of the shape
    time_one(cur, best_ms);
    out.ms_default = best_ms;
    out.tried = 1;
    std::vector<std::pair<Tune, double>> seen{{cur, best_ms}};
    auto same = [](const Tune& a, const Tune& b) {
        return a.units_per_wave == b.units_per_wave && a.grid_mult == b.grid_mult &&
               a.walks_per_lane == b.walks_per_lane && a.waves_per_block == b.waves_per_block &&
               a.lanes_per_walker == b.lanes_per_walker;
    };
    static const int wpbs[] = {1, 2, 4}, upws[] = {1, 2, 4, 8, 16}, gms[] = {1, 2}, wpls[] = {1, 2, 4};
    static const int* const vals_of[] = {wpbs, upws, gms, wpls};
    static const int n_of[] = {3, 5, 2, 3};
    auto field = [](Tune& t, int prm) -> int& {
        return prm == 0 ? t.waves_per_block : prm == 1 ? t.units_per_wave : prm == 2 ? t.grid_mult
                                                       : t.walks_per_lane;
    };
    // time candidate c (or take its earlier time); adopt it past the noise guard
    auto consider = [&](const Tune& c, bool& moved) -> bool {
        double m = -1.0;
        for (auto& s : seen)
            if (same(s.first, c)) m = s.second;
        if (m < 0.0) {
            time_one(c, m);
            seen.push_back({c, m});
            ++out.tried;
        }
        if (e == hipSuccess && !rc && m < best_ms * (1.0 - 0.005)) {
            cur = c;
            best_ms = m;
            moved = true;
            return true;
        }
        return false;
    };
    for (int pass = 0; pass < 2 && e == hipSuccess && !rc; ++pass) {
        bool moved = false;
        for (int prm = 0; prm < 4; ++prm) {
            for (int i = 0; i < n_of[prm] && e == hipSuccess && !rc; ++i) {
                Tune c = cur;
                field(c, prm) = vals_of[prm][i];
                consider(c, moved);
            }
        }
        // lanes per walker G in 1, 2, 4, ..., 64: double (then halve) while
        // the launch gets faster, so a batch that fills the device never
        // pays for the large G that only a handful of walks can use
        for (int dir = 0; dir < 2 && e == hipSuccess && !rc; ++dir) {
            for (;;) {
                const int g = dir == 0 ? 2 * cur.lanes_per_walker : cur.lanes_per_walker / 2;
                if (g < 1 || g > kWave || e != hipSuccess || rc) break;
                Tune c = cur;
                c.lanes_per_walker = g;
                if (!consider(c, moved)) break;
            }
        }
        if (!moved) break;
    }
    out.best = cur;
    out.ms_best = best_ms;
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    void* bufs[] = {du, dg, dub, ddx, dds, ddg};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (st) (void)hipStreamDestroy(st);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    return WOS_OK;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* wos_last_error(void) { return g_err.c_str(); }

int wos_create_domain(int d, const wos_spheres* spheres, const wos_boxes* boxes, const wos_arm* arm,
                      const wos_ball* goal, const wos_outer* outer, const wos_bdata* bdata,
                      const wos_source* source, wos_domain** out)
{
    if (!out) return fail(WOS_EINVAL, "out is NULL");
    *out = nullptr;
    if (d < WOS_MIN_DIM || d > WOS_MAX_DIM) return fail(WOS_EDIM, "d = %d outside [%d, %d]", d, WOS_MIN_DIM, WOS_MAX_DIM);
    if (!outer || !bdata) return fail(WOS_EINVAL, "outer and bdata are required");
    int rc = check_obstacles(d, spheres, boxes);
    if (rc) return rc;
    const int64_t ns = spheres ? spheres->n : 0, nb = boxes ? boxes->n : 0;
    if (bdata->mode < 0 || bdata->mode > 2) return fail(WOS_EINVAL, "unknown boundary-data mode %d", bdata->mode);
    if (source && (!source->z || !finite_all(source->z, d) || !std::isfinite(source->amplitude) ||
                   !std::isfinite(source->c_imp) || source->c_imp < 0.0))
        return fail(WOS_EINVAL, "bad point source (z NULL or non-finite, amplitude non-finite, c_imp < 0)");
    if (bdata->mode != 0 && !bdata->a_or_k) return fail(WOS_EINVAL, "a_or_k is required for mode %d", bdata->mode);

    const int gd = outer->geom_d == 0 ? d : outer->geom_d;
    if (gd < 1 || gd > d) return fail(WOS_EINVAL, "geom_d = %d outside [0, %d]", outer->geom_d, d);
    if (gd < d && nb > 0) return fail(WOS_EINVAL, "box obstacles need the full space (geom_d = d)");
    double arm_K = 0.0;
    if (arm) {
        if (!arm->lengths || !arm->points || arm->n_points < 1 || arm->n_points > (int64_t)INT32_MAX)
            return fail(WOS_EINVAL, "arm needs lengths and 1 <= n_points < 2^31 points");
        if (!finite_all(arm->lengths, d) || !finite_all(arm->points, 2 * arm->n_points))
            return fail(WOS_EINVAL, "non-finite arm lengths or points");
        for (int n = 0; n < d; ++n) {
            if (arm->lengths[n] < 0.0) return fail(WOS_EINVAL, "arm link lengths must be >= 0");
            double reach = 0.0;  // joint n moves every point beyond it at most this fast
            for (int i = n; i < d; ++i) reach += arm->lengths[i];
            arm_K += reach * reach;
        }
        arm_K = std::sqrt(arm_K);
        if (!(arm_K > 0.0)) return fail(WOS_EINVAL, "arm links are all of length 0");
        if (gd < d) return fail(WOS_EINVAL, "an arm needs the full space (geom_d = d)");
        if (bdata->mode != WOS_BDATA_CLASS)
            return fail(WOS_ENOTSUP, "an arm bound names no boundary point: class boundary data only");
    }
    // extruded geometry: sphere centres without their trailing coordinates
    std::vector<double> sc_ext;
    wos_spheres sph_ext;
    if (gd < d && ns > 0) {
        sc_ext.assign(spheres->centers, spheres->centers + ns * d);
        for (int64_t j = 0; j < ns; ++j)
            for (int i = gd; i < d; ++i) sc_ext[j * d + i] = 0.0;
        sph_ext = *spheres;
        sph_ext.centers = sc_ext.data();
        spheres = &sph_ext;
    }

    wos_domain* D = new wos_domain();
    D->d = d;
    D->geom_d = gd;
    D->n_sph = ns;
    D->n_box = nb;
    if (goal) {
        if (!goal->center || !(goal->radius > 0) || !finite_all(goal->center, d) || !std::isfinite(goal->radius)) {
            delete D;
            return fail(WOS_EINVAL, "bad goal ball");
        }
        D->has_goal = true;
        for (int i = 0; i < d; ++i) D->goal_c[i] = goal->center[i];
        D->goal_r = goal->radius;
    }
    D->outer_kind = outer->kind;
    if (outer->kind == WOS_OUTER_BOX) {
        if (!outer->lo || !outer->hi || !finite_all(outer->lo, gd) || !finite_all(outer->hi, gd)) {
            delete D;
            return fail(WOS_EINVAL, "bad outer box");
        }
        double rmax = INFINITY;
        for (int i = 0; i < gd; ++i) {
            if (!(outer->hi[i] > outer->lo[i])) {
                delete D;
                return fail(WOS_EINVAL, "outer box needs hi > lo");
            }
            D->lo[i] = outer->lo[i];
            D->hi[i] = outer->hi[i];
            rmax = std::min(rmax, 0.5 * (outer->hi[i] - outer->lo[i]));
        }
        // unbounded trailing coordinates: the kernels see them as 0, so these
        // faces are never the nearest
        for (int i = gd; i < d; ++i) {
            D->lo[i] = -kFarFace;
            D->hi[i] = kFarFace;
        }
        D->r_max = rmax;
    } else if (outer->kind == WOS_OUTER_BALL) {
        if (!outer->center || !(outer->radius > 0) || !finite_all(outer->center, gd) || !std::isfinite(outer->radius)) {
            delete D;
            return fail(WOS_EINVAL, "bad outer ball");
        }
        for (int i = 0; i < gd; ++i) D->oc[i] = outer->center[i];
        D->orad = outer->radius;
        D->r_max = outer->radius;
    } else {
        delete D;
        return fail(WOS_EINVAL, "unknown outer kind %d", outer->kind);
    }
    if (arm) {
        D->n_arm = arm->n_points;
        for (int i = 0; i < d; ++i) D->arm_l[i] = arm->lengths[i];
        D->arm_K = arm_K;
    }
    if (source) {
        D->has_src = true;
        for (int i = 0; i < d; ++i) D->src_z[i] = source->z[i];
        D->src_amp = source->amplitude;
        D->c_imp = source->c_imp;
    }
    D->mode = bdata->mode;
    D->g_goal = bdata->g_goal;
    D->g_obs = bdata->g_obstacle;
    D->g_outer = bdata->g_outer;
    D->b = bdata->b;
    if (bdata->mode != 0)
        for (int i = 0; i < d; ++i) D->ak[i] = bdata->a_or_k[i];
    if (!std::isfinite(D->g_goal) || !std::isfinite(D->g_obs) || !std::isfinite(D->g_outer) || !std::isfinite(D->b) ||
        !finite_all(D->ak, d)) {
        delete D;
        return fail(WOS_EINVAL, "non-finite boundary data");
    }

    // device tables, FP32 and FP64, padded rows
    const int ss = sph_stride(d), bs = box_stride(d);
    std::vector<float> sf, bf;
    std::vector<double> sd, bd;
    obstacle_rows(d, spheres, boxes, sf, sd, bf, bd);
    {
        // size of the geometry: every coordinate magnitude plus radius
        double sc = 0.0;
        if (D->has_goal)
            for (int i = 0; i < d; ++i) sc = std::max(sc, std::fabs(D->goal_c[i]) + D->goal_r);
        if (D->outer_kind == WOS_OUTER_BOX)
            for (int i = 0; i < gd; ++i) sc = std::max(sc, std::max(std::fabs(D->lo[i]), std::fabs(D->hi[i])));
        else
            for (int i = 0; i < gd; ++i) sc = std::max(sc, std::fabs(D->oc[i]) + D->orad);
        for (int64_t j = 0; j < ns; ++j)
            for (int i = 0; i < d; ++i) sc = std::max(sc, std::fabs(spheres->centers[j * d + i]) + spheres->radii[j]);
        for (int64_t j = 0; j < nb; ++j)
            for (int i = 0; i < d; ++i)
                sc = std::max(sc, std::fabs(boxes->centers[j * d + i]) + boxes->half_widths[j * d + i]);
        if (D->n_arm > 0) {
            double reach = 0.0;
            for (int i = 0; i < d; ++i) reach += std::fabs(D->arm_l[i]);
            sc = std::max(sc, reach);
            for (int64_t j = 0; j < 2 * (int64_t)D->n_arm; ++j) sc = std::max(sc, std::fabs(arm->points[j]));
        }
        D->coord_scale = sc;
    }
    hipError_t e = hipGetDevice(&D->device);
    if (e == hipSuccess) e = hipMalloc(&D->sph_f, sf.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&D->sph_d, sd.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&D->box_f, bf.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&D->box_d, bd.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(D->sph_f, sf.data(), sf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(D->sph_d, sd.data(), sd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(D->box_f, bf.data(), bf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(D->box_d, bd.data(), bd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && D->n_arm > 0) {
        const size_t na = 2 * (size_t)D->n_arm;
        std::vector<float> af(arm->points, arm->points + na);
        e = hipMalloc(&D->arm_f, na * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&D->arm_d, na * sizeof(double));
        if (e == hipSuccess) e = hipMemcpy(D->arm_f, af.data(), na * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(D->arm_d, arm->points, na * sizeof(double), hipMemcpyHostToDevice);
    }
    // clustered tables for large obstacle sets
    std::vector<int64_t> idx_s, idx_b;
    D->n_cl_sph = (int32_t)cluster_order(d, ns, ns ? spheres->centers : nullptr, idx_s);
    D->n_cl_box = (int32_t)cluster_order(d, nb, nb ? boxes->centers : nullptr, idx_b);
    // bound tables hold one zero row past the last cluster, which the scan
    // prefetches and never uses
    const int sb = sph_stride(d);
    const size_t nbs = D->n_cl_sph ? (size_t)D->n_cl_sph + 1 : 0, nbb = D->n_cl_box ? (size_t)D->n_cl_box + 1 : 0;
    D->off_sph_bnd = (size_t)D->n_cl_sph * kCluster * ss;
    D->off_box_cl = D->off_sph_bnd + nbs * sb;
    D->off_box_bnd = D->off_box_cl + (size_t)D->n_cl_box * kCluster * bs;
    const size_t cl_elems = D->off_box_bnd + nbb * sb;
    // matrix-core features live in the FP32 buffer only, after the tables
    // one spare tile after each table: the kernel loads tile t + 1 while testing tile t
    const size_t mf_s = D->n_cl_sph ? (size_t)((D->n_cl_sph + kMfmaTile - 1) / kMfmaTile + 1) * 64 * 4 : 0;
    const size_t mf_b = D->n_cl_box ? (size_t)((D->n_cl_box + kMfmaTile - 1) / kMfmaTile + 1) * 64 * 4 : 0;
    D->off_sph_mf = (cl_elems + 3) / 4 * 4;  // 16-byte aligned float4 rows
    D->off_box_mf = D->off_sph_mf + mf_s;
    // cluster bounding boxes, also FP32 only (16-byte aligned rows)
    D->off_sph_cb = D->off_box_mf + mf_b;
    D->off_box_cb = D->off_sph_cb + (size_t)D->n_cl_sph * kClusterBox;
    const size_t cf_elems = D->off_box_cb + (size_t)D->n_cl_box * kClusterBox;
    if (e == hipSuccess && cl_elems > 0) {
        std::vector<float> cf(cf_elems, 0.f);
        std::vector<double> cd(cl_elems, 0.0);
        if (D->n_cl_sph) {
            build_clusters<float>(d, ns, false, idx_s, sf.data(), ss, cf.data(), cf.data() + D->off_sph_bnd);
            build_clusters<double>(d, ns, false, idx_s, sd.data(), ss, cd.data(), cd.data() + D->off_sph_bnd);
        }
        if (D->n_cl_box) {
            build_clusters<float>(d, nb, true, idx_b, bf.data(), bs, cf.data() + D->off_box_cl,
                                  cf.data() + D->off_box_bnd);
            build_clusters<double>(d, nb, true, idx_b, bd.data(), bs, cd.data() + D->off_box_cl,
                                   cd.data() + D->off_box_bnd);
        }
        if (D->n_cl_sph)
            build_mfma_features(d, D->n_cl_sph, cf.data() + D->off_sph_bnd, cf.data() + D->off_sph_mf);
        if (D->n_cl_box)
            build_mfma_features(d, D->n_cl_box, cf.data() + D->off_box_bnd, cf.data() + D->off_box_mf);
        if (D->n_cl_sph) build_cluster_boxes(d, ns, false, idx_s, sf.data(), ss, cf.data() + D->off_sph_cb);
        if (D->n_cl_box) build_cluster_boxes(d, nb, true, idx_b, bf.data(), bs, cf.data() + D->off_box_cb);
        e = hipMalloc(&D->cl_f, cf_elems * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&D->cl_d, cl_elems * sizeof(double));
        if (e == hipSuccess) e = hipMemcpy(D->cl_f, cf.data(), cf_elems * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(D->cl_d, cd.data(), cl_elems * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        wos_destroy_domain(D);
        return fail(e == hipErrorOutOfMemory ? WOS_ENOMEM : WOS_EHIP, "domain upload: %s", hipGetErrorString(e));
    }
    *out = D;
    return WOS_OK;
}

void wos_destroy_domain(wos_domain* D)
{
    if (!D) return;
    (void)hipFree(D->sph_f);
    (void)hipFree(D->sph_d);
    (void)hipFree(D->box_f);
    (void)hipFree(D->box_d);
    (void)hipFree(D->cl_f);
    (void)hipFree(D->cl_d);
    (void)hipFree(D->arm_f);
    (void)hipFree(D->arm_d);
    delete D;
}

int wos_domain_dim(const wos_domain* D) { return D ? D->d : fail(WOS_EINVAL, "domain is NULL"); }

int wos_varadhan(const void* u, const void* grad_u, int64_t n, int d, int stride, double sigma, void* out_w,
                 void* out_grad_w, const wos_options* opt, void* stream)
{
    wos_options o;
    int rc = read_opts(opt, o);
    if (rc) return rc;
    if (o.flags & WOS_OUT_FP64) return fail(WOS_ENOTSUP, "WOS_OUT_FP64 applies to wos_estimate only (pass WOS_FP64 for double u)");
    if (n < 0) return fail(WOS_EINVAL, "n < 0");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(WOS_EINVAL, "sigma must be finite and > 0 (t = 1/sigma)");
    if (n > 0 && (!u || !out_w)) return fail(WOS_EINVAL, "u and out_w are required");
    if ((grad_u == nullptr) != (out_grad_w == nullptr)) return fail(WOS_EINVAL, "grad_u and out_grad_w go together");
    if (grad_u && (d < WOS_MIN_DIM || d > WOS_MAX_DIM)) return fail(WOS_EDIM, "d = %d outside [%d, %d]", d, WOS_MIN_DIM, WOS_MAX_DIM);
    if (grad_u && stride < d) return fail(WOS_EINVAL, "stride < d");
    hipStream_t st = (hipStream_t)stream;
    if (o.flags & WOS_FP64)
        WOS_HIP(launch_varadhan<double>((const double*)u, (const double*)grad_u, n, d, stride, sigma, (double*)out_w,
                                        (double*)out_grad_w, st),
                "varadhan");
    else
        WOS_HIP(launch_varadhan<float>((const float*)u, (const float*)grad_u, n, d, stride, sigma, (float*)out_w,
                                       (float*)out_grad_w, st),
                "varadhan");
    return WOS_OK;
}

static_assert(kCluster == WOS_CLUSTER_ROWS, "the header states the cluster size callers size their arrays by");
static_assert(kBatchStats == WOS_BATCH_STATS && kBatchStride == WOS_BATCH_STRIDE,
              "the header states the batched row widths callers size their arrays by");

int wos_debug_clusters(int d, const wos_spheres* spheres, const wos_boxes* boxes, int fp64, int64_t* out_n_cl,
                       int64_t* order_sph, double* bnd_sph, int64_t* order_box, double* bnd_box)
{
    if (d < WOS_MIN_DIM || d > WOS_MAX_DIM) return fail(WOS_EDIM, "d = %d outside [%d, %d]", d, WOS_MIN_DIM, WOS_MAX_DIM);
    if (!out_n_cl) return fail(WOS_EINVAL, "out_n_cl is NULL");
    int rc = check_obstacles(d, spheres, boxes);
    if (rc) return rc;
    const int64_t ns = spheres ? spheres->n : 0, nb = boxes ? boxes->n : 0;
    std::vector<float> sf, bf;
    std::vector<double> sd, bd;
    obstacle_rows(d, spheres, boxes, sf, sd, bf, bd);
    std::vector<int64_t> idx[2];
    const int64_t n_cl[2] = {cluster_order(d, ns, ns ? spheres->centers : nullptr, idx[0]),
                             cluster_order(d, nb, nb ? boxes->centers : nullptr, idx[1])};
    out_n_cl[0] = n_cl[0];
    out_n_cl[1] = n_cl[1];
    const int64_t n[2] = {ns, nb};
    const int S[2] = {sph_stride(d), box_stride(d)};
    const int SB = sph_stride(d);
    int64_t* order[2] = {order_sph, order_box};
    double* bnd[2] = {bnd_sph, bnd_box};
    for (int k = 0; k < 2; ++k) {
        if (!n_cl[k]) continue;
        if (order[k])
            for (int64_t j = 0; j < n_cl[k] * kCluster; ++j) order[k][j] = j < n[k] ? idx[k][j] : -1;
        if (!bnd[k]) continue;
        std::vector<double> b((size_t)n_cl[k] * SB);
        if (fp64) {
            std::vector<double> cl((size_t)n_cl[k] * kCluster * S[k]);
            build_clusters<double>(d, n[k], k == 1, idx[k], k ? bd.data() : sd.data(), S[k], cl.data(), b.data());
        } else {
            std::vector<float> cl((size_t)n_cl[k] * kCluster * S[k]), bf32((size_t)n_cl[k] * SB);
            build_clusters<float>(d, n[k], k == 1, idx[k], k ? bf.data() : sf.data(), S[k], cl.data(), bf32.data());
            for (size_t i = 0; i < b.size(); ++i) b[i] = bf32[i];
        }
        for (int64_t g = 0; g < n_cl[k]; ++g)
            for (int i = 0; i <= d; ++i) bnd[k][g * (d + 1) + i] = b[g * SB + i];
    }
    return WOS_OK;
}

int wos_debug_cluster_boxes(int d, const wos_spheres* spheres, const wos_boxes* boxes, int64_t* out_n_cl,
                            double* box_sph, double* box_box)
{
    if (d < WOS_MIN_DIM || d > WOS_MAX_DIM) return fail(WOS_EDIM, "d = %d outside [%d, %d]", d, WOS_MIN_DIM, WOS_MAX_DIM);
    if (!out_n_cl) return fail(WOS_EINVAL, "out_n_cl is NULL");
    int rc = check_obstacles(d, spheres, boxes);
    if (rc) return rc;
    const int64_t ns = spheres ? spheres->n : 0, nb = boxes ? boxes->n : 0;
    std::vector<float> sf, bf;
    std::vector<double> sd, bd;
    obstacle_rows(d, spheres, boxes, sf, sd, bf, bd);
    std::vector<int64_t> idx[2];
    const int64_t n_cl[2] = {cluster_order(d, ns, ns ? spheres->centers : nullptr, idx[0]),
                             cluster_order(d, nb, nb ? boxes->centers : nullptr, idx[1])};
    out_n_cl[0] = n_cl[0];
    out_n_cl[1] = n_cl[1];
    const int64_t n[2] = {ns, nb};
    const int S[2] = {sph_stride(d), box_stride(d)};
    double* out[2] = {box_sph, box_box};
    for (int k = 0; k < 2; ++k) {
        if (!n_cl[k] || !out[k]) continue;
        std::vector<float> cb((size_t)n_cl[k] * kClusterBox);
        build_cluster_boxes(d, n[k], k == 1, idx[k], k ? bf.data() : sf.data(), S[k], cb.data());
        for (int64_t g = 0; g < n_cl[k]; ++g)
            for (int i = 0; i < d; ++i) {
                out[k][g * 2 * d + i] = cb[g * kClusterBox + i];
                out[k][g * 2 * d + d + i] = cb[g * kClusterBox + kMaxDim + i];
            }
    }
    return WOS_OK;
}

static int estimate_impl(const wos_domain* D, const void* queries, int64_t Q, int64_t n_walks, double sigma,
                         double eps, uint64_t seed, void* out_u, void* out_grad, double* out_stats,
                         const void* grad_u, void* out_dx, double* out_dsigma, double* out_dg, double* out_dq,
                         const wos_options* opt, hipStream_t st, bool bwd)
{
    if (!D) return fail(WOS_EINVAL, "domain is NULL");
    wos_options o;
    int rc = read_opts(opt, o);
    if (rc) return rc;
    if ((rc = check_device(D))) return rc;
    if (Q < 0 || Q > ((int64_t)1 << 32)) return fail(WOS_EINVAL, "n_queries out of range");
    if (n_walks < 1 || n_walks > ((int64_t)1 << 31)) return fail(WOS_EINVAL, "n_walks must be in [1, 2^31]");
    if (bwd) {
        if (!out_dx || !out_dsigma || !out_dg) return fail(WOS_EINVAL, "out_dx, out_dsigma and out_dg are required");
        if (Q > 0 && !grad_u) return fail(WOS_EINVAL, "grad_u is required");
    } else if (Q > 0 && !out_u) {
        return fail(WOS_EINVAL, "out_u is required");
    }
    if (Q > 0 && !queries) return fail(WOS_EINVAL, "queries is NULL");
    if (bwd && (o.flags & WOS_OUT_FP64)) return fail(WOS_ENOTSUP, "WOS_OUT_FP64 applies to wos_estimate only");
    if (bwd && D->has_src && !(sigma > 0.0))
        return fail(WOS_ENOTSUP, "the sigma derivative of a point source is provided for sigma > 0 only");
    const int d = D->d;
    const int32_t chunks = (int32_t)((n_walks + kWave - 1) / kWave);
    Scratch S(st);
    double* partials = nullptr;
    double* prod = nullptr;
    if ((rc = S.get(&partials, (size_t)std::max<int64_t>(Q, 1) * chunks * nacc(d)))) return rc;
    if (bwd && (rc = S.get(&prod, (size_t)std::max<int64_t>(Q, 1) * 2))) return rc;
    if (o.flags & WOS_FP64) {
        EnvP<double> p;
        if ((rc = make_env<double>(D, sigma, eps, seed, o.env_id, o, p))) return rc;
        if (Q == 0) {
            if (bwd) {
                WOS_HIP(launch_fill_f64(out_dsigma, 1, 0.0, st), "fill");
                WOS_HIP(launch_fill_f64(out_dg, 1, 0.0, st), "fill");
            }
            return WOS_OK;
        }
        double* uo = (double*)out_u;
        double* uscratch = nullptr;
        if (bwd && !uo) {
            if ((rc = S.get(&uscratch, (size_t)Q))) return rc;
            uo = uscratch;
        }
        EnvP<double>* pd;
        if ((rc = S.get(&pd, 1)) || (rc = upload(pd, &p, sizeof(p), st))) return rc;
        WOS_HIP(launch_plain<double>(d, bwd, D->has_src, pd, (const double*)queries, Q, n_walks, 0, 0, nullptr, partials,
                                     nullptr, st),
                "plain walk kernel");
        WOS_HIP(launch_finalize_plain<double>(d, bwd, partials, Q, chunks, n_walks, uo, (double*)out_grad, out_stats,
                                              (const double*)grad_u, (double*)out_dx, out_dq, prod, st),
                "finalize");
    } else {
        EnvP<float> p;
        if ((rc = make_env<float>(D, sigma, eps, seed, o.env_id, o, p))) return rc;
        if (Q == 0) {
            if (bwd) {
                WOS_HIP(launch_fill_f64(out_dsigma, 1, 0.0, st), "fill");
                WOS_HIP(launch_fill_f64(out_dg, 1, 0.0, st), "fill");
            }
            return WOS_OK;
        }
        float* uo = (float*)out_u;
        float* uscratch = nullptr;
        if (bwd && !uo) {
            if ((rc = S.get(&uscratch, (size_t)Q))) return rc;
            uo = uscratch;
        }
        EnvP<float>* pd;
        if ((rc = S.get(&pd, 1)) || (rc = upload(pd, &p, sizeof(p), st))) return rc;
        WOS_HIP(launch_plain<float>(d, bwd, D->has_src, pd, (const float*)queries, Q, n_walks, 0, 0, nullptr, partials,
                                    nullptr, st),
                "plain walk kernel");
        if (o.flags & WOS_OUT_FP64)  // forward only: the FP64 sums written without rounding to FP32
            WOS_HIP(launch_finalize_plain<double>(d, false, partials, Q, chunks, n_walks, (double*)out_u,
                                                  (double*)out_grad, out_stats, nullptr, nullptr, nullptr, nullptr, st),
                    "finalize");
        else
            WOS_HIP(launch_finalize_plain<float>(d, bwd, partials, Q, chunks, n_walks, uo, (float*)out_grad, out_stats,
                                                 (const float*)grad_u, (float*)out_dx, out_dq, prod, st),
                    "finalize");
    }
    if (bwd) WOS_HIP(launch_reduce_pairs(prod, Q, out_dsigma, out_dg, st), "reduce");
    return WOS_OK;
}

int wos_estimate(const wos_domain* dom, const void* queries, int64_t n_queries, int64_t n_walks, double sigma,
                 double eps, uint64_t seed, void* out_u, void* out_grad, double* out_stats,
                 const wos_options* opt, void* stream)
{
    return estimate_impl(dom, queries, n_queries, n_walks, sigma, eps, seed, out_u, out_grad, out_stats, nullptr,
                         nullptr, nullptr, nullptr, nullptr, opt, (hipStream_t)stream, false);
}

int wos_backward(const wos_domain* dom, const void* queries, int64_t n_queries, int64_t n_walks, double sigma,
                 double eps, uint64_t seed, const void* grad_u, void* out_dx, double* out_dsigma,
                 double* out_dg_goal, double* out_dq, const wos_options* opt, void* stream)
{
    return estimate_impl(dom, queries, n_queries, n_walks, sigma, eps, seed, nullptr, nullptr, nullptr, grad_u,
                         out_dx, out_dsigma, out_dg_goal, out_dq, opt, (hipStream_t)stream, true);
}

int wos_estimate_batch(const wos_domain* const* envs, int n_envs, const float* queries, const int64_t* q_offsets,
                       const double* sigma, const double* eps, const int64_t* n_walks, uint64_t seed, float* out_u,
                       float* out_grad, double* out_stats, const float* grad_u, float* out_dx, double* out_dsigma,
                       double* out_dg, const wos_options* opt, void* stream)
{
    return run_batch(envs, n_envs, queries, q_offsets, sigma, eps, n_walks, seed, out_u, out_grad, out_stats,
                     grad_u, out_dx, out_dsigma, out_dg, opt, (hipStream_t)stream, nullptr, false);
}

int wos_estimate_batch_noalloc(const wos_domain* const* envs, int n_envs, const float* queries,
                               const int64_t* q_offsets, const double* sigma, const double* eps,
                               const int64_t* n_walks, uint64_t seed, float* out_u, float* out_grad,
                               double* out_stats, const float* grad_u, float* out_dx, double* out_dsigma,
                               double* out_dg, const wos_options* opt, void* stream)
{
    return run_batch(envs, n_envs, queries, q_offsets, sigma, eps, n_walks, seed, out_u, out_grad, out_stats,
                     grad_u, out_dx, out_dsigma, out_dg, opt, (hipStream_t)stream, nullptr, true);
}

int wos_debug_walks(const wos_domain* D, const double* query, uint32_t q_index, int64_t w0, int64_t n, double sigma,
                    double eps, uint64_t seed, const wos_options* opt, double* out_records)
{
    if (!D || !query || !out_records) return fail(WOS_EINVAL, "domain, query and out_records are required");
    wos_options o;
    int rc = read_opts(opt, o);
    if (rc) return rc;
    if (o.flags & WOS_OUT_FP64) return fail(WOS_ENOTSUP, "WOS_OUT_FP64 applies to wos_estimate only");
    if ((rc = check_device(D))) return rc;
    if (n < 1 || w0 < 0 || w0 + n > ((int64_t)1 << 32)) return fail(WOS_EINVAL, "bad walk range");
    const int d = D->d;
    const int32_t chunks = (int32_t)((n + kWave - 1) / kWave);
    void* dq = nullptr;
    double* part = nullptr;
    double* rec = nullptr;
    const size_t esz = (o.flags & WOS_FP64) ? sizeof(double) : sizeof(float);
    hipError_t e = hipMalloc(&dq, d * esz);
    if (e == hipSuccess) e = hipMalloc(&part, (size_t)chunks * nacc(d) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&rec, (size_t)n * (d + 7) * sizeof(double));
    if (e == hipSuccess) {
        if (o.flags & WOS_FP64) {
            e = hipMemcpy(dq, query, d * sizeof(double), hipMemcpyHostToDevice);
            EnvP<double> p;
            rc = make_env<double>(D, sigma, eps, seed, o.env_id, o, p);
            void* pd = nullptr;
            if (!rc && e == hipSuccess) e = hipMalloc(&pd, sizeof(p));
            if (!rc && e == hipSuccess) e = hipMemcpy(pd, &p, sizeof(p), hipMemcpyHostToDevice);
            if (!rc && e == hipSuccess)
                e = launch_plain<double>(d, true, D->has_src, (const EnvP<double>*)pd, (const double*)dq, 1, n, w0, q_index, nullptr,
                                         part, rec, nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            (void)hipFree(pd);
        } else {
            float qf[kMaxDim];
            for (int i = 0; i < d; ++i) qf[i] = (float)query[i];
            e = hipMemcpy(dq, qf, d * sizeof(float), hipMemcpyHostToDevice);
            EnvP<float> p;
            rc = make_env<float>(D, sigma, eps, seed, o.env_id, o, p);
            void* pd = nullptr;
            if (!rc && e == hipSuccess) e = hipMalloc(&pd, sizeof(p));
            if (!rc && e == hipSuccess) e = hipMemcpy(pd, &p, sizeof(p), hipMemcpyHostToDevice);
            if (!rc && e == hipSuccess)
                e = launch_plain<float>(d, true, D->has_src, (const EnvP<float>*)pd, (const float*)dq, 1, n, w0, q_index, nullptr,
                                        part, rec, nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            (void)hipFree(pd);
        }
    }
    if (e == hipSuccess && !rc) e = hipDeviceSynchronize();
    if (e == hipSuccess && !rc) e = hipMemcpy(out_records, rec, (size_t)n * (d + 7) * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(dq);
    (void)hipFree(part);
    (void)hipFree(rec);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "debug walks");
    return WOS_OK;
}

// ----------------------------------------------------------------------------
// Planning loop
// ----------------------------------------------------------------------------
}  // extern "C"

struct wos_plan {
    int d = 0;
    int64_t S = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* x = nullptr;
    float* u = nullptr;
    float* grad = nullptr;
    float* ubar = nullptr;
    float* dx = nullptr;
    float* dir = nullptr;
    double* dsig = nullptr;
    double* dg = nullptr;
    double* partials = nullptr;
    double* path_len = nullptr;
    int32_t* stalls = nullptr;
    int32_t* status = nullptr;
    uint64_t* step = nullptr;
    unsigned* counter = nullptr;
    EnvP<float>* env = nullptr;
    BatchEnv* benv = nullptr;
    EnvP<float> henv;
};

static void plan_free(wos_plan* P)
{
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    void* bufs[] = {P->u, P->grad, P->ubar, P->dx, P->dir, P->dsig, P->dg, P->partials, P->path_len,
                    P->stalls, P->status, P->step, P->counter, P->env, P->benv};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (P->own_stream && P->st) (void)hipStreamDestroy(P->st);
    delete P;
}

extern "C" {

int wos_plan_create(const wos_domain* D, float* x, int64_t n_starts, int64_t n_walks, double sigma, double eps,
                    double s_ub, uint64_t seed, const wos_options* opt, void* stream, wos_plan** out)
{
    if (!out) return fail(WOS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!D || !x) return fail(WOS_EINVAL, "domain and x are required");
    wos_options o;
    int rc = read_opts(opt, o);
    if (rc) return rc;
    if (o.flags & WOS_FP64) return fail(WOS_ENOTSUP, "the planning loop computes in FP32 only");
    if (o.flags & WOS_OUT_FP64) return fail(WOS_ENOTSUP, "WOS_OUT_FP64 applies to wos_estimate only");
    if ((rc = check_device(D))) return rc;
    if (n_starts < 1 || n_starts > (1 << 24)) return fail(WOS_EINVAL, "n_starts out of range");
    if (n_walks < 1 || n_walks > ((int64_t)1 << 31)) return fail(WOS_EINVAL, "n_walks must be in [1, 2^31]");
    if (!(s_ub > 0) || !std::isfinite(s_ub)) return fail(WOS_EINVAL, "s_ub must be finite and > 0");
    wos_plan* P = new wos_plan();
    P->d = D->d;
    P->S = n_starts;
    P->x = x;
    if ((rc = make_env<float>(D, sigma, eps, seed, o.env_id, o, P->henv))) {
        delete P;
        return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!st) {
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        P->own_stream = true;
    }
    P->st = st;
    const wos_domain* envs[1] = {D};
    const int64_t qoff[2] = {0, n_starts};
    const int64_t nw[1] = {n_walks};
    BatchLayout L;
    BatchEnv benv1;
    int order1;
    plan_batch(envs, qoff, 1, nw, D->d, nullptr, (o.flags & WOS_FULL_SCAN) != 0, D->has_src, &order1, &benv1, L);
    if (L.total_units >= ((int64_t)1 << 32) - 1) {
        plan_free(P);
        return fail(WOS_EINVAL, "the plan splits into %lld work units; at most 2^32 - 2", (long long)L.total_units);
    }
    const int64_t S = n_starts;
    if (e == hipSuccess) e = hipMalloc(&P->u, S * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&P->grad, S * kBatchStride * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&P->ubar, S * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&P->dx, S * kBatchStride * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&P->dir, S * kBatchStride * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&P->dsig, sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&P->dg, sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&P->partials, (size_t)std::max<int64_t>(L.total_units, 1) * nacc(kMaxDim) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&P->path_len, S * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&P->stalls, S * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&P->status, S * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&P->step, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&P->counter, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc(&P->env, sizeof(EnvP<float>));
    if (e == hipSuccess) e = hipMalloc(&P->benv, sizeof(BatchEnv));
    if (e == hipSuccess) e = hipMemcpy(P->env, &P->henv, sizeof(EnvP<float>), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->benv, &benv1, sizeof(BatchEnv), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_fill_f64(P->path_len, S, 0.0, st);
    if (e == hipSuccess) e = launch_fill_u32((unsigned*)P->stalls, S, 0u, st);
    if (e == hipSuccess) e = launch_fill_u32((unsigned*)P->status, S, 0u, st);
    if (e == hipSuccess) e = launch_fill_u32((unsigned*)P->step, 2, 0u, st);
    if (e == hipSuccess) e = launch_fill_u32(P->counter, 1, 0u, st);
    if (e == hipSuccess) e = launch_fill_u32((unsigned*)P->ubar, S, 0x3f800000u, st);  // upstream weights 1.0f
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        plan_free(P);
        return hip_fail(e, "plan set-up");
    }
    // capture [fused forward + backward walks, finalize, update]
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = launch_persistent(true, D->has_src, L.grid, L.block, P->env, P->benv, 1, x, L.total_units,
                                          P->henv.key0, P->henv.key1, P->step, P->counter, P->partials, st);
        hipError_t e2 = launch_finalize_batch(true, P->benv, 1, P->partials, P->ubar, P->u, P->grad,
                                              kBatchStride, nullptr, P->dx, P->dsig, P->dg, P->dir, P->counter, st);
        hipError_t e3 = launch_plan_update(D->d, P->env, x, S, P->dir, kBatchStride, (float)s_ub, P->path_len,
                                           P->stalls, P->status, P->step, st);
        e = hipStreamEndCapture(st, &P->graph);
        if (e == hipSuccess) e = (e1 != hipSuccess) ? e1 : (e2 != hipSuccess) ? e2 : e3;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_free(P);
        return hip_fail(e, "plan graph capture");
    }
    *out = P;
    return WOS_OK;
}

int wos_plan_step(wos_plan* P, int n_steps)
{
    if (!P) return fail(WOS_EINVAL, "plan is NULL");
    if (n_steps < 0) return fail(WOS_EINVAL, "n_steps < 0");
    for (int i = 0; i < n_steps; ++i) WOS_HIP(hipGraphLaunch(P->exec, P->st), "hipGraphLaunch");
    return WOS_OK;
}

int wos_plan_buffers(wos_plan* P, float** u, float** grad, double** path_len, int32_t** stalls, int32_t** status,
                     uint64_t** step)
{
    if (!P) return fail(WOS_EINVAL, "plan is NULL");
    if (u) *u = P->u;
    if (grad) *grad = P->grad;
    if (path_len) *path_len = P->path_len;
    if (stalls) *stalls = P->stalls;
    if (status) *status = P->status;
    if (step) *step = P->step;
    return WOS_OK;
}

int wos_plan_read(wos_plan* P, float* u, float* grad, double* path_len, int32_t* stalls, int32_t* status,
                  uint64_t* step)
{
    if (!P) return fail(WOS_EINVAL, "plan is NULL");
    WOS_HIP(hipStreamSynchronize(P->st), "plan sync");
    const int64_t S = P->S;
    if (u) WOS_HIP(hipMemcpy(u, P->u, S * sizeof(float), hipMemcpyDeviceToHost), "plan read");
    if (grad) WOS_HIP(hipMemcpy(grad, P->grad, S * kBatchStride * sizeof(float), hipMemcpyDeviceToHost), "plan read");
    if (path_len) WOS_HIP(hipMemcpy(path_len, P->path_len, S * sizeof(double), hipMemcpyDeviceToHost), "plan read");
    if (stalls) WOS_HIP(hipMemcpy(stalls, P->stalls, S * sizeof(int32_t), hipMemcpyDeviceToHost), "plan read");
    if (status) WOS_HIP(hipMemcpy(status, P->status, S * sizeof(int32_t), hipMemcpyDeviceToHost), "plan read");
    if (step) WOS_HIP(hipMemcpy(step, P->step, sizeof(uint64_t), hipMemcpyDeviceToHost), "plan read");
    return WOS_OK;
}

void wos_plan_destroy(wos_plan* P)
{
    if (!P) return;
    if (P->st) (void)hipStreamSynchronize(P->st);
    plan_free(P);
}

// ----------------------------------------------------------------------------
// Autotuner
// ----------------------------------------------------------------------------
int wos_set_autotune_cache(const char* cache_path)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_locked(cache_path);
    return WOS_OK;
}

int wos_autotune(int d, int64_t M, int64_t Q, int64_t n_walks, const char* cache_path)
{
    if (d < WOS_MIN_DIM || d > WOS_MAX_DIM) return fail(WOS_EDIM, "d = %d outside [2, 8]", d);
    if (M < 0 || Q < 1 || n_walks < 1 || !cache_path) return fail(WOS_EINVAL, "bad autotune arguments");
    // synthetic scene: M spheres r in [0.1, 0.4] in [-pi, pi]^d (64-bit LCG)
    uint64_t s = 0x9E3779B97F4A7C15ull ^ ((uint64_t)d << 32) ^ (uint64_t)M;
    auto rnd = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) * 0x1p-53;
    };
    const double pi = 3.14159265358979323846;
    std::vector<double> c((size_t)std::max<int64_t>(M, 1) * d), r((size_t)std::max<int64_t>(M, 1));
    for (int64_t j = 0; j < M; ++j) {
        for (int i = 0; i < d; ++i) c[j * d + i] = (2 * rnd() - 1) * pi;
        r[j] = 0.1 + 0.3 * rnd();
    }
    std::vector<double> lo(d, -pi), hi(d, pi), gc(d, 0.0);
    wos_spheres sp{M, c.data(), r.data()};
    wos_ball goal{gc.data(), 0.15};
    wos_outer ob{WOS_OUTER_BOX, lo.data(), hi.data(), nullptr, 0};
    wos_bdata bdv{WOS_BDATA_CLASS, 1.0, 0.0, 0.0, nullptr, 0.0};
    wos_domain* D = nullptr;
    int rc = wos_create_domain(d, &sp, nullptr, nullptr, &goal, &ob, &bdv, nullptr, &D);
    if (rc) return rc;
    std::vector<float> hq((size_t)Q * kBatchStride, 0.f);
    for (int64_t q = 0; q < Q; ++q)
        for (int i = 0; i < d; ++i) hq[q * kBatchStride + i] = (float)((2 * rnd() - 1) * (pi - 0.05));
    float* dq = nullptr;
    hipError_t e = hipMalloc(&dq, hq.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(dq, hq.data(), hq.size() * sizeof(float), hipMemcpyHostToDevice);
    TuneRun run;
    const wos_domain* envs[1] = {D};
    const int64_t qoff[2] = {0, Q};
    const int64_t nw[1] = {n_walks};
    const double sig = 2.0, ep = 1e-4;
    if (e == hipSuccess) rc = tune_batch(envs, 1, dq, qoff, &sig, &ep, nw, 1234, true, run);
    (void)hipDeviceSynchronize();
    if (dq) (void)hipFree(dq);
    wos_destroy_domain(D);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (rc) return rc;
    char k[48];
    tune_key(k, d, M, Q);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded || g_tune_path != cache_path) load_tune_locked(cache_path);
    g_tune[k] = run.best;
    return save_tune_locked(cache_path);
}

int wos_autotune_batch(const wos_domain* const* envs, int n_envs, const float* queries, const int64_t* q_offsets,
                       const double* sigma, const double* eps, const int64_t* n_walks, uint64_t seed, int fused,
                       const char* cache_path, wos_tune_result* out)
{
    if (n_envs < 1 || !envs || !queries || !q_offsets || !sigma || !eps || !n_walks)
        return fail(WOS_EINVAL, "bad autotune arguments");
    TuneRun run;
    int rc = tune_batch(envs, n_envs, queries, q_offsets, sigma, eps, n_walks, seed, fused != 0, run);
    if (rc) return rc;
    char k[48];
    mix_key(k, envs, q_offsets, n_envs, n_walks);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (cache_path && *cache_path && (!g_tune_loaded || g_tune_path != cache_path)) load_tune_locked(cache_path);
        if (!g_tune_loaded) load_tune_locked(getenv("WOS_AUTOTUNE_CACHE"));
        g_tune[k] = run.best;
        if (cache_path && *cache_path && (rc = save_tune_locked(cache_path))) return rc;
    }
    if (out) {
        out->waves_per_block = run.best.waves_per_block;
        out->units_per_wave = run.best.units_per_wave;
        out->grid_mult = run.best.grid_mult;
        out->walks_per_lane = run.best.walks_per_lane;
        out->lanes_per_walker = run.best.lanes_per_walker;
        out->ms_default = run.ms_default;
        out->ms_best = run.ms_best;
        out->tried = run.tried;
    }
    return WOS_OK;
}

}  // extern "C"

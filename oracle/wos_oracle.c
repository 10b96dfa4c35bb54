/*
 * wos_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the
 * Walk-on-Spheres estimator of the screened Poisson equation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library: it has its
 * own Philox, sampling, distance, series and estimator code.
 *
 * What it computes (Muchacho & Pokorny, "Walk on Spheres for PDE-based Path
 * Planning"):
 *   PDE (Sec. III, eq. screened_poisson_wos, with c = 1/t; we write sigma = c):
 *       Laplacian(u) - sigma u = 0 in Omega,  u = g on the boundary.
 *   Boundary data: g = g_goal on the goal ball, g_obs on obstacles and
 *   g_outer on the outer box (Sec. III, eq. screened_potential_field, with the
 *   goal set as the g = 1 part of the boundary), or, to pin the estimator,
 *   affine data a.y + b (sigma = 0) or a plane wave exp(k.y) with |k|^2 = sigma.
 *   Estimator (Sec. IV-A): u_hat(x_k) = g(xbar_k) inside the eps-shell,
 *   else C(x_k) u_hat(x_{k+1}), with x_{k+1} uniform on the largest empty
 *   sphere around x_k (Sec. IV, Fig. 2).  The paper leaves C unstated; it is
 *   the value at the centre of a ball of the solution with unit boundary data:
 *       C(R) = 1 / 0F1(; d/2; sigma R^2 / 4).
 *   Gradient (Sec. IV-A, first-sphere estimator), with the screening factor
 *   the printed formula omits for sigma > 0 (it reduces to the printed d/R
 *   form at sigma = 0):
 *       grad_hat u(x_0) = (d / R_0) C1(R_0) u_hat(x_1) v_0,
 *       C1(R) = 1 / 0F1(; d/2 + 1; sigma R^2 / 4).
 *   Backward (not in the paper): the path law does not depend on sigma (radii
 *   are distances), so d u_hat / d sigma = u_hat * sum_k d ln C(R_k) / d sigma
 *   exactly, with d ln C / d sigma = -(R^2 / 2d) 0F1(;d/2+1;y) / 0F1(;d/2;y);
 *   u is linear in the goal value, so d u_hat / d g_goal = W 1{goal}.
 *   Point source (Sec. VI and VII: a unit impulse at the goal point z with
 *   zero boundary data; Sec. IV-A: the |B| f G_c term of u_hat and the
 *   c_imp grad G_c term of the gradient): with f = amp delta_z the volume
 *   term of step k is amp G_B(x_k, z) 1{|z - x_k| < R_k}, G_B the Green's
 *   function of (-Laplacian + sigma) on the ball B(x_k, R_k) with zero data
 *   on its sphere (the sign that makes u >= 0 peak at the source).  So
 *       u_hat(x_0) = sum_k W_k amp G_B(|z - x_k|; R_k) 1{.} + W_K g(xbar_K),
 *       grad_hat u(x_0) = (d / R_0) C1(R_0) u_hat(x_1) v_0
 *                         + c_imp amp grad_x G_B(x_0, z) 1{|z - x_0| < R_0},
 *   with u_hat(x_1) the same sum over the walk from x_1 (weights W1_k).
 *   Planar arm (Sec. V-A): with joint coordinates q and task-space obstacle
 *   points, the joint-space distance to collision is replaced by the lower
 *   bound d_tau(q) / K, d_tau the planar distance between the points and the
 *   arm's links and K a Lipschitz constant of the planar forward kinematics
 *   (see or_arm_K); ties order goal, spheres, boxes, arm, outer.
 *   Extruded geometry (Sec. VI, the evaluation environment): the obstacles
 *   and the outer boundary may depend on the first geom_d coordinates only,
 *   the others being unbounded; their distances and closest points are then
 *   taken in those coordinates, the goal ball and the source stay
 *   d-dimensional.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 * 64-bit seed, counter = (2k + j, walk, query, env) for step k and block j;
 * 32-bit word x gives the uniform (2 (x >> 9) + 1) 2^-24 in (0, 1); pair p of
 * uniforms (words 2p, 2p+1) gives two normals by Box-Muller (1958); the
 * direction is the normal vector divided by its norm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 8
#define OR_PI 3.14159265358979323846

enum { OR_GOAL = 0, OR_SPHERE = 1, OR_BOX = 2, OR_OUTER = 3, OR_ARM = 4 };
enum { OR_ABSORBED = 0, OR_DEGENERATE = 1, OR_TRUNCATED = 2 };

typedef struct {
    int d;
    int has_src;         /* point source amp delta_z */
    double src_z[OR_MAXD];
    double src_amp, c_imp;
    int n_sph;
    const double* sph_c; /* n_sph x d */
    const double* sph_r; /* n_sph */
    int n_box;
    const double* box_c; /* n_box x d */
    const double* box_h; /* n_box x d */
    int has_goal;
    double goal_c[OR_MAXD];
    double goal_r;
    int outer_kind; /* 0 box [lo, hi], 1 ball (c, r) */
    double lo[OR_MAXD], hi[OR_MAXD];
    double outer_c[OR_MAXD];
    double outer_r;
    int mode; /* 0 class constants, 1 affine a.y + b, 2 plane wave exp(k.y) */
    double g_goal, g_obs, g_outer;
    double ak[OR_MAXD];
    double b;
    int geom_d; /* 0 or d: full space; else obstacles and the outer boundary
                   depend on x[0..geom_d) only (extruded, Sec. VI) */
    int n_arm;              /* task-space obstacle points of a planar arm, 0: none */
    const double* arm_pts;  /* n_arm x 2 */
    double arm_l[OR_MAXD];  /* link lengths, one link per joint coordinate */
} or_domain;

typedef struct {
    double u;                /* one-point estimate u_hat(x_0) */
    double grad[OR_MAXD];    /* one-point gradient estimate */
    double dlnC_sum;         /* sum over weighted steps of d ln C / d sigma */
    double du_dsigma;        /* d u_hat / d sigma (u_hat dlnC_sum without a source) */
    double goal_w;           /* W * 1{absorbed on the goal} */
    int steps;               /* distance evaluations made */
    int status;              /* OR_ABSORBED / OR_DEGENERATE / OR_TRUNCATED */
    int cls, idx;            /* boundary component that absorbed the walk */
} or_walk_record;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (SC'11, Sec. 3 and Table 2):  */
/* each round multiplies words 0 and 2 by fixed constants, swaps and xors the */
/* high halves into words 1 and 3 with the round key; the key is bumped by    */
/* the Weyl constants between rounds.                                         */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> uniform in (0, 1): odd multiples of 2^-24, exact in FP32. */
double or_uniform(uint32_t x)
{
    return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0);
}

/* Uniform direction on the unit sphere S^{d-1} for step k of walk (w, q, env):
 * ceil(d/2) Box-Muller pairs, then normalisation (Sec. IV: the next point is
 * uniform on the sphere around the current one). */
void or_direction(int d, uint64_t seed, uint32_t k, uint32_t w, uint32_t q, uint32_t env,
                  double v[OR_MAXD])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t words[8];
    int n_pairs = (d + 1) / 2;
    int n_blocks = (n_pairs + 1) / 2;
    for (int j = 0; j < n_blocks; ++j) {
        uint32_t ctr[4] = {2u * k + (uint32_t)j, w, q, env};
        or_philox4x32_10(ctr, key, words + 4 * j);
    }
    double n[OR_MAXD];
    for (int p = 0; p < n_pairs; ++p) {
        double u1 = or_uniform(words[2 * p]);
        double u2 = or_uniform(words[2 * p + 1]);
        double rho = sqrt(-2.0 * log(u1));
        double theta = 2.0 * OR_PI * u2;
        n[2 * p] = rho * cos(theta);
        if (2 * p + 1 < d) n[2 * p + 1] = rho * sin(theta);
    }
    double norm2 = 0.0;
    for (int i = 0; i < d; ++i) norm2 += n[i] * n[i];
    double norm = sqrt(norm2);
    for (int i = 0; i < d; ++i) v[i] = n[i] / norm;
}

/* ------------------------------------------------------------------------ */
/* Distance to the boundary (Sec. V: the walk needs d(x, boundary); exact     */
/* signed distances of the union's components, their minimum, and the first   */
/* component attaining it in the order goal, spheres, boxes, outer).          */
/* ------------------------------------------------------------------------ */
static double dist_ball_outside(int d, const double* x, const double* c, double r)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += (x[i] - c[i]) * (x[i] - c[i]);
    return sqrt(s) - r;
}

static double dist_box_signed(int d, const double* x, const double* c, const double* h)
{
    double outside2 = 0.0, inside = -INFINITY;
    for (int i = 0; i < d; ++i) {
        double q = fabs(x[i] - c[i]) - h[i];
        if (q > 0.0) outside2 += q * q;
        if (q > inside) inside = q;
    }
    return sqrt(outside2) + (inside < 0.0 ? inside : 0.0);
}

/* coordinates the obstacles and the outer boundary depend on */
static int geom_dim(const or_domain* D) { return D->geom_d > 0 ? D->geom_d : D->d; }

static double dist_outer(const or_domain* D, const double* x)
{
    int g = geom_dim(D);
    if (D->outer_kind == 0) {
        double m = INFINITY;
        for (int i = 0; i < g; ++i) {
            double a = x[i] - D->lo[i], b = D->hi[i] - x[i];
            if (a < m) m = a;
            if (b < m) m = b;
        }
        return m;
    }
    double s = 0.0;
    for (int i = 0; i < g; ++i) s += (x[i] - D->outer_c[i]) * (x[i] - D->outer_c[i]);
    return D->outer_r - sqrt(s);
}

/* Lipschitz constant of the planar forward kinematics (Sec. V-A): joint n
 * moves every point beyond it at most (l_n + ... + l_N) per radian, so the
 * Jacobian of any point of the arm has Frobenius norm at most
 * K = sqrt(sum_n (l_n + ... + l_N)^2).  (The printed sum runs over the first
 * n links; the two agree for equal links.) */
double or_arm_K(const or_domain* D)
{
    double s = 0.0;
    for (int n = 0; n < D->d; ++n) {
        double reach = 0.0;
        for (int i = n; i < D->d; ++i) reach += D->arm_l[i];
        s += reach * reach;
    }
    return sqrt(s);
}

/* Planar distance between the obstacle points and the arm at joint angles q:
 * the base joint sits at the origin, link i ends l_i further along the
 * direction q_0 + ... + q_i; each link is a segment. */
double or_arm_task_distance(const or_domain* D, const double* q)
{
    double ax = 0.0, ay = 0.0, th = 0.0, best = INFINITY;
    for (int i = 0; i < D->d; ++i) {
        th += q[i];
        double bx = ax + D->arm_l[i] * cos(th), by = ay + D->arm_l[i] * sin(th);
        double sx = bx - ax, sy = by - ay, ss = sx * sx + sy * sy;
        for (int j = 0; j < D->n_arm; ++j) {
            double px = D->arm_pts[2 * j] - ax, py = D->arm_pts[2 * j + 1] - ay;
            double t = ss > 0.0 ? (px * sx + py * sy) / ss : 0.0;
            if (t < 0.0) t = 0.0;
            if (t > 1.0) t = 1.0;
            double ex = px - t * sx, ey = py - t * sy;
            double dist = sqrt(ex * ex + ey * ey);
            if (dist < best) best = dist;
        }
        ax = bx;
        ay = by;
    }
    return best;
}

double or_distance(const or_domain* D, const double* x, int* cls, int* idx)
{
    int d = D->d, g = geom_dim(D);
    double best = INFINITY;
    int bc = OR_OUTER, bi = 0;
    if (D->has_goal) {
        best = dist_ball_outside(d, x, D->goal_c, D->goal_r);
        bc = OR_GOAL;
    }
    for (int j = 0; j < D->n_sph; ++j) {
        double dj = dist_ball_outside(g, x, D->sph_c + (size_t)j * d, D->sph_r[j]);
        if (dj < best) { best = dj; bc = OR_SPHERE; bi = j; }
    }
    for (int j = 0; j < D->n_box; ++j) {
        double dj = dist_box_signed(g, x, D->box_c + (size_t)j * d, D->box_h + (size_t)j * d);
        if (dj < best) { best = dj; bc = OR_BOX; bi = j; }
    }
    if (D->n_arm > 0) {
        double da = or_arm_task_distance(D, x) / or_arm_K(D);
        if (da < best) { best = da; bc = OR_ARM; bi = 0; }
    }
    double dout = dist_outer(D, x);
    if (dout < best) { best = dout; bc = OR_OUTER; bi = 0; }
    if (cls) *cls = bc;
    if (idx) *idx = bi;
    return best;
}

/* Closest point xbar on component (cls, idx) (Fig. 2: the boundary value is
 * read at the closest boundary point of the absorbed walker). */
void or_closest_point(const or_domain* D, const double* x, int cls, int idx, double* xbar)
{
    int d = D->d;
    /* an extruded component moves the first g coordinates, keeps the rest */
    int g = cls == OR_GOAL ? d : geom_dim(D);
    memcpy(xbar, x, sizeof(double) * (size_t)d);
    if (cls == OR_ARM) {  /* the bound names no boundary point */
        for (int i = 0; i < d; ++i) xbar[i] = NAN;
        return;
    }
    if (cls == OR_GOAL || cls == OR_SPHERE || (cls == OR_OUTER && D->outer_kind == 1)) {
        const double* c;
        double r;
        if (cls == OR_GOAL) { c = D->goal_c; r = D->goal_r; }
        else if (cls == OR_SPHERE) { c = D->sph_c + (size_t)idx * d; r = D->sph_r[idx]; }
        else { c = D->outer_c; r = D->outer_r; }
        double s = 0.0;
        for (int i = 0; i < g; ++i) s += (x[i] - c[i]) * (x[i] - c[i]);
        double n = sqrt(s);
        if (n == 0.0) {
            for (int i = 0; i < g; ++i) xbar[i] = c[i];
            xbar[0] = c[0] + r;
            return;
        }
        for (int i = 0; i < g; ++i) xbar[i] = c[i] + r * (x[i] - c[i]) / n;
        return;
    }
    if (cls == OR_BOX) {
        const double* c = D->box_c + (size_t)idx * d;
        const double* h = D->box_h + (size_t)idx * d;
        int inside = 1;
        for (int i = 0; i < g; ++i)
            if (fabs(x[i] - c[i]) > h[i]) inside = 0;
        if (!inside) {
            for (int i = 0; i < g; ++i) {
                double a = c[i] - h[i], b = c[i] + h[i];
                xbar[i] = x[i] < a ? a : (x[i] > b ? b : x[i]);
            }
            return;
        }
        /* inside: move the coordinate of the nearest face onto that face */
        int im = 0;
        double qm = -INFINITY;
        for (int i = 0; i < g; ++i) {
            double q = fabs(x[i] - c[i]) - h[i];
            if (q > qm) { qm = q; im = i; }
        }
        xbar[im] = c[im] + (x[im] >= c[im] ? h[im] : -h[im]);
        return;
    }
    /* outer box: the nearest face, lower face first on ties */
    int im = 0, hiface = 0;
    double m = INFINITY;
    for (int i = 0; i < g; ++i) {
        double a = x[i] - D->lo[i], b = D->hi[i] - x[i];
        if (a < m) { m = a; im = i; hiface = 0; }
        if (b < m) { m = b; im = i; hiface = 1; }
    }
    xbar[im] = hiface ? D->hi[im] : D->lo[im];
}

/* Boundary data g at the closest point of the absorbing component. */
double or_boundary_value(const or_domain* D, const double* x, int cls, int idx)
{
    if (D->mode == 0) {
        if (cls == OR_GOAL) return D->g_goal;
        if (cls == OR_OUTER) return D->g_outer;
        return D->g_obs;
    }
    double xbar[OR_MAXD];
    or_closest_point(D, x, cls, idx, xbar);
    double s = 0.0;
    for (int i = 0; i < D->d; ++i) s += D->ak[i] * xbar[i];
    if (D->mode == 1) return s + D->b;
    return exp(s);
}

/* ------------------------------------------------------------------------ */
/* Screening weights.  0F1(;b;y) = sum_k y^k / ((b)_k k!) (DLMF 16.2.1).      */
/* ------------------------------------------------------------------------ */
double or_hyp0f1(double b, double y)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 100000; ++k) {
        term *= y / ((b + k - 1.0) * (double)k);
        sum += term;
        if (term <= 1e-17 * sum) break;
    }
    return sum;
}

/* C(R): weight of one step of radius R (Sec. IV-A, the normalisation C(x)). */
double or_screening_C(int d, double sigma, double R)
{
    return 1.0 / or_hyp0f1(0.5 * d, 0.25 * sigma * R * R);
}

/* C1(R): screening factor of the first-sphere gradient estimator. */
double or_screening_C1(int d, double sigma, double R)
{
    return 1.0 / or_hyp0f1(0.5 * d + 1.0, 0.25 * sigma * R * R);
}

/* d ln C(R) / d sigma. */
double or_dlnC_dsigma(int d, double sigma, double R)
{
    double y = 0.25 * sigma * R * R;
    return -(R * R / (2.0 * d)) * or_hyp0f1(0.5 * d + 1.0, y) / or_hyp0f1(0.5 * d, y);
}

/* ------------------------------------------------------------------------ */
/* Point-source terms: Bessel functions and the Green's function of the ball. */
/* nu = d/2 - 1.  Free-space fundamental solution of (-Laplacian + sigma):     */
/*   sigma > 0: Phi(r) = (2 pi)^(-d/2) sigma^(nu/2) r^(-nu) K_nu(sqrt(sigma) r) */
/*   sigma = 0: Phi(r) = -ln(r) / (2 pi) (d = 2), r^(2-d) / ((d-2) |S^(d-1)|). */
/* Ball of radius R, source at distance r from the centre, zero data on the   */
/* sphere (the l = 0 mode):  G_B(r; R) = Phi(r) - Phi(R) p(r) / p(R),          */
/* p(s) = 0F1(; nu+1; sigma s^2 / 4), the regular radial solution (p = 1 at    */
/* sigma = 0).  Gradient in the centre point towards the source (the l = 1    */
/* mode, which vanishes on the sphere and has the free-space singularity):    */
/*   sigma > 0: (2 pi)^(-d/2) sigma^((nu+1)/2) r^(-nu)                         */
/*              [K_{nu+1}(sqrt(sigma) r) - K_{nu+1}(sqrt(sigma) R) (r/R)^(nu+1) */
/*               p1(r) / p1(R)],   p1(s) = 0F1(; nu+2; sigma s^2 / 4),          */
/*   sigma = 0: (r^(1-d) - r R^(-d)) / |S^(d-1)|.                              */
/* ------------------------------------------------------------------------ */

/* K_nu(z), z > 0, from its integral representation (DLMF 10.32.9)
 * K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt, by the trapezoidal rule
 * with step 1/16 (the integrand is analytic and decays doubly exponentially,
 * so the rule converges to rounding).  Terms are summed until they are
 * negligible and decreasing. */
double or_bessel_k(double nu, double z)
{
    if (!(z > 0.0)) return INFINITY;
    const double h = 1.0 / 16.0;
    double sum = 0.5 * exp(-z);
    for (int j = 1; j < 1000000; ++j) {
        double t = j * h;
        sum += exp(-z * cosh(t)) * cosh(nu * t);
        /* past the maximum of the integrand and below the smallest double */
        if (z * sinh(t) > nu && -z * cosh(t) + nu * t < -745.0) break;
    }
    return h * sum;
}

static double sphere_area(int d)
{
    return 2.0 * pow(OR_PI, 0.5 * d) / tgamma(0.5 * d);
}

/* Free-space fundamental solution Phi(r). */
double or_yukawa_free(int d, double sigma, double r)
{
    double nu = 0.5 * d - 1.0;
    if (sigma > 0.0)
        return pow(2.0 * OR_PI, -0.5 * d) * pow(sigma, 0.5 * nu) * pow(r, -nu) * or_bessel_k(nu, sqrt(sigma) * r);
    if (d == 2) return -log(r) / (2.0 * OR_PI);
    return pow(r, 2.0 - d) / ((d - 2.0) * sphere_area(d));
}

/* G_B(r; R): Green's function of the ball between its centre and a point at
 * distance r < R. */
double or_ball_green(int d, double sigma, double r, double R)
{
    double nu = 0.5 * d - 1.0;
    double ratio = or_hyp0f1(nu + 1.0, 0.25 * sigma * r * r) / or_hyp0f1(nu + 1.0, 0.25 * sigma * R * R);
    return or_yukawa_free(d, sigma, r) - or_yukawa_free(d, sigma, R) * ratio;
}

/* |grad_x G_B(x, y)| at the centre x, towards y, |y - x| = r < R. */
double or_ball_green_grad(int d, double sigma, double r, double R)
{
    double nu = 0.5 * d - 1.0;
    if (sigma > 0.0) {
        double rs = sqrt(sigma);
        double ratio = pow(r / R, nu + 1.0) * or_hyp0f1(nu + 2.0, 0.25 * sigma * r * r) /
                       or_hyp0f1(nu + 2.0, 0.25 * sigma * R * R);
        return pow(2.0 * OR_PI, -0.5 * d) * pow(sigma, 0.5 * (nu + 1.0)) * pow(r, -nu) *
               (or_bessel_k(nu + 1.0, rs * r) - or_bessel_k(nu + 1.0, rs * R) * ratio);
    }
    return (pow(r, 1.0 - d) - r * pow(R, -(double)d)) / sphere_area(d);
}

/* d Phi(r) / d sigma, sigma > 0: from d/dz (z^-nu K_nu(z)) = -z^-nu K_{nu+1}(z)
 * (DLMF 10.29.4), (2 pi)^(-d/2) r^(-nu) [nu sigma^(nu/2 - 1) K_nu(z)
 * - (r / 2) sigma^((nu - 1)/2) K_{nu+1}(z)], z = sqrt(sigma) r. */
static double yukawa_free_dsigma(int d, double sigma, double r)
{
    double nu = 0.5 * d - 1.0, z = sqrt(sigma) * r;
    return pow(2.0 * OR_PI, -0.5 * d) * pow(r, -nu) *
           (nu * pow(sigma, 0.5 * nu - 1.0) * or_bessel_k(nu, z) -
            0.5 * r * pow(sigma, 0.5 * (nu - 1.0)) * or_bessel_k(nu + 1.0, z));
}

/* d G_B(r; R) / d sigma for sigma > 0 (product and quotient rules on the
 * definition; d p(s) / d sigma = (s^2 / 4) 0F1(; nu+2; sigma s^2 / 4) / (nu + 1)). */
double or_ball_green_dsigma(int d, double sigma, double r, double R)
{
    double nu = 0.5 * d - 1.0;
    double pr = or_hyp0f1(nu + 1.0, 0.25 * sigma * r * r), pR = or_hyp0f1(nu + 1.0, 0.25 * sigma * R * R);
    double dpr = 0.25 * r * r * or_hyp0f1(nu + 2.0, 0.25 * sigma * r * r) / (nu + 1.0);
    double dpR = 0.25 * R * R * or_hyp0f1(nu + 2.0, 0.25 * sigma * R * R) / (nu + 1.0);
    double dratio = (dpr * pR - pr * dpR) / (pR * pR);
    return yukawa_free_dsigma(d, sigma, r) - yukawa_free_dsigma(d, sigma, R) * (pr / pR) -
           or_yukawa_free(d, sigma, R) * dratio;
}

/* ------------------------------------------------------------------------ */
/* One walk (Sec. IV-A recursion, unrolled: u_hat(x_0) = prod_k C(R_k) g).     */
/* ------------------------------------------------------------------------ */
void or_walk(const or_domain* D, const double* xq, double sigma, double eps, uint64_t seed,
             uint32_t w, uint32_t q, uint32_t env, int max_steps, or_walk_record* rec)
{
    int d = D->d;
    double x[OR_MAXD], v[OR_MAXD], v0[OR_MAXD];
    double W = 1.0;        /* prod_{i < k} C(R_i): weight of u_hat(x_0)            */
    double W1 = 1.0;       /* prod_{1 <= i < k} C(R_i): weight of u_hat(x_1)        */
    double R0 = 0.0, C1_0 = 0.0, S = 0.0;
    double src = 0.0;      /* sum_k W_k amp G_B(x_k, z): source part of u_hat(x_0)  */
    double src1 = 0.0;     /* the same with weights W1_k, k >= 1: of u_hat(x_1)     */
    double srcS = 0.0;     /* sum_k W_k amp (S_k G_B + d G_B / d sigma)             */
    double gsrc[OR_MAXD] = {0};
    memcpy(x, xq, sizeof(double) * (size_t)d);
    memset(rec, 0, sizeof(*rec));
    for (int k = 0;; ++k) {
        int cls, idx;
        double R = or_distance(D, x, &cls, &idx);
        rec->steps = k + 1;
        if (R < eps) { /* x_k in the eps-shell: u_hat(x_k) = g(xbar_k) */
            double g = or_boundary_value(D, x, cls, idx);
            rec->cls = cls;
            rec->idx = idx;
            if (k == 0) {
                rec->status = OR_DEGENERATE;
                rec->u = g;
                rec->goal_w = (cls == OR_GOAL) ? 1.0 : 0.0;
                return;
            }
            rec->status = OR_ABSORBED;
            rec->u = W * g + src;
            for (int i = 0; i < d; ++i)
                rec->grad[i] = (d / R0) * C1_0 * (W1 * g + src1) * v0[i] + gsrc[i];
            rec->dlnC_sum = S;
            rec->du_dsigma = W * g * S + srcS;
            rec->goal_w = (cls == OR_GOAL) ? W : 0.0;
            return;
        }
        if (k + 1 >= max_steps) { /* step cap reached: walk contributes zero */
            rec->status = OR_TRUNCATED;
            return;
        }
        if (D->has_src) { /* the ball around x_k holds the source: volume term */
            double r2 = 0.0;
            for (int i = 0; i < d; ++i) r2 += (D->src_z[i] - x[i]) * (D->src_z[i] - x[i]);
            double r = sqrt(r2);
            if (r < R) {
                double G = D->src_amp * or_ball_green(d, sigma, r, R);
                src += W * G;
                if (k > 0) src1 += W1 * G;
                if (sigma > 0.0) srcS += W * (S * G + D->src_amp * or_ball_green_dsigma(d, sigma, r, R));
                else srcS = NAN; /* d G_B / d sigma at sigma = 0 is not provided */
                if (k == 0 && r > 0.0) {
                    double gm = D->c_imp * D->src_amp * or_ball_green_grad(d, sigma, r, R) / r;
                    for (int i = 0; i < d; ++i) gsrc[i] = gm * (D->src_z[i] - x[i]);
                }
            }
        }
        double C = or_screening_C(d, sigma, R);
        W *= C;
        if (k > 0) W1 *= C;
        S += or_dlnC_dsigma(d, sigma, R);
        or_direction(d, seed, (uint32_t)k, w, q, env, v);
        if (k == 0) {
            R0 = R;
            C1_0 = or_screening_C1(d, sigma, R);
            memcpy(v0, v, sizeof(double) * (size_t)d);
        }
        for (int i = 0; i < d; ++i) x[i] += R * v[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Varadhan read-out (Sec. III, eq. transformation_varadhan):                 */
/* w = -sqrt(t) ln u with t = 1 / sigma, grad w = -sqrt(t) grad u / u.        */
/* u <= 0 (no signal) gives w = +inf and grad w = 0.                          */
/* ------------------------------------------------------------------------ */
void or_varadhan(int d, double sigma, double u, const double* grad_u, double* w, double* grad_w)
{
    double st = 1.0 / sqrt(sigma);
    if (!(u > 0.0)) {
        *w = INFINITY;
        if (grad_w) for (int i = 0; i < d; ++i) grad_w[i] = 0.0;
        return;
    }
    *w = -st * log(u);
    if (grad_w) for (int i = 0; i < d; ++i) grad_w[i] = -st * grad_u[i] / u;
}

/* ------------------------------------------------------------------------ */
/* Per-query mean of the one-point estimates (Sec. IV-A) and standard errors. */
/* stats row (d + 4): se_u, se_grad[d], mean_steps, n_trunc, n_degen.         */
/* Optional per-query backward sums: dq row (2): mean(u_hat S), mean(goal_w). */
/* ------------------------------------------------------------------------ */
static double se_two_pass(const double* a, int64_t n)
{
    if (n < 2) return 0.0;
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m += a[i];
    m /= (double)n;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (a[i] - m) * (a[i] - m);
    return sqrt(s / (double)(n - 1)) / sqrt((double)n);
}

int or_estimate(const or_domain* D, const double* queries, int64_t Q, int64_t n, double sigma,
                double eps, uint64_t seed, uint32_t env, int max_steps, double* out_u,
                double* out_grad, double* out_stats, double* out_dq)
{
    int d = D->d;
    if (n < 1 || Q < 0) return -1;
    double* uw = (double*)malloc(sizeof(double) * (size_t)n);
    double* gw = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
    if (!uw || !gw) { free(uw); free(gw); return -2; }
    for (int64_t q = 0; q < Q; ++q) {
        double su = 0.0, sg[OR_MAXD] = {0}, ssteps = 0.0, sS = 0.0, sgoal = 0.0;
        int64_t ntr = 0, ndg = 0;
        for (int64_t w = 0; w < n; ++w) {
            or_walk_record r;
            or_walk(D, queries + q * d, sigma, eps, seed, (uint32_t)w, (uint32_t)q, env,
                    max_steps, &r);
            uw[w] = r.u;
            su += r.u;
            for (int i = 0; i < d; ++i) {
                gw[i * n + w] = r.grad[i];
                sg[i] += r.grad[i];
            }
            ssteps += r.steps;
            sS += r.du_dsigma;
            sgoal += r.goal_w;
            if (r.status == OR_TRUNCATED) ++ntr;
            if (r.status == OR_DEGENERATE) ++ndg;
        }
        out_u[q] = su / (double)n;
        if (out_grad)
            for (int i = 0; i < d; ++i) out_grad[q * d + i] = sg[i] / (double)n;
        if (out_stats) {
            double* st = out_stats + q * (d + 4);
            st[0] = se_two_pass(uw, n);
            for (int i = 0; i < d; ++i) st[1 + i] = se_two_pass(gw + (size_t)i * n, n);
            st[d + 1] = ssteps / (double)n;
            st[d + 2] = (double)ntr;
            st[d + 3] = (double)ndg;
        }
        if (out_dq) {
            out_dq[2 * q] = sS / (double)n;
            out_dq[2 * q + 1] = sgoal / (double)n;
        }
    }
    free(uw);
    free(gw);
    return 0;
}

/* Backward of L(u) for upstream ubar: dL/dx_q = ubar_q grad u(x_q),
 * dL/dsigma = sum_q ubar_q du_q/dsigma, dL/dg_goal = sum_q ubar_q du_q/dg_goal,
 * all from the same walks as the forward (same seed). */
int or_backward(const or_domain* D, const double* queries, int64_t Q, int64_t n, double sigma,
                double eps, uint64_t seed, uint32_t env, int max_steps, const double* ubar,
                double* out_dx, double* out_dsigma, double* out_dg)
{
    int d = D->d;
    double* u = (double*)malloc(sizeof(double) * (size_t)(Q > 0 ? Q : 1));
    double* g = (double*)malloc(sizeof(double) * (size_t)(Q > 0 ? Q : 1) * (size_t)d);
    double* dq = (double*)malloc(sizeof(double) * (size_t)(Q > 0 ? Q : 1) * 2);
    if (!u || !g || !dq) { free(u); free(g); free(dq); return -2; }
    int rc = or_estimate(D, queries, Q, n, sigma, eps, seed, env, max_steps, u, g, NULL, dq);
    double ds = 0.0, dg = 0.0;
    for (int64_t q = 0; q < Q && rc == 0; ++q) {
        for (int i = 0; i < d; ++i) out_dx[q * d + i] = ubar[q] * g[q * d + i];
        ds += ubar[q] * dq[2 * q];
        dg += ubar[q] * dq[2 * q + 1];
    }
    *out_dsigma = ds;
    *out_dg = dg;
    free(u);
    free(g);
    free(dq);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* One step of gradient ascent along the normalised gradient (Sec. III,       */
/* screened-harmonic paths) with the adaptive step s = min(s_ub, d/2)         */
/* (Sec. VII, Table I).  Planning step t uses seed + t; start s is query s.   */
/* status: 0 moving, 1 reached the goal shell, 2 in another boundary shell.   */
/* ------------------------------------------------------------------------ */
int or_plan_step(const or_domain* D, double* x, int64_t S, int64_t n, double sigma, double eps,
                 double s_ub, uint64_t seed, uint64_t t, int max_steps, double* path_len,
                 int32_t* stalls, int32_t* status)
{
    int d = D->d;
    for (int64_t s = 0; s < S; ++s) {
        double* xs = x + s * d;
        int cls, idx;
        double R = or_distance(D, xs, &cls, &idx);
        if (R < eps) {
            status[s] = (cls == OR_GOAL) ? 1 : 2;
            continue;
        }
        if (D->has_src) { /* a point-source goal is reached within one nominal step */
            double dz2 = 0.0;
            for (int i = 0; i < d; ++i) dz2 += (xs[i] - D->src_z[i]) * (xs[i] - D->src_z[i]);
            if (sqrt(dz2) < s_ub) {
                status[s] = 1;
                continue;
            }
        }
        status[s] = 0;
        /* the walks of start s are keyed by query index s */
        double g[OR_MAXD], sg[OR_MAXD] = {0};
        for (int64_t w = 0; w < n; ++w) {
            or_walk_record r;
            or_walk(D, xs, sigma, eps, seed + t, (uint32_t)w, (uint32_t)s, 0, max_steps, &r);
            for (int i = 0; i < d; ++i) sg[i] += r.grad[i];
        }
        double gn2 = 0.0;
        for (int i = 0; i < d; ++i) {
            g[i] = sg[i] / (double)n;
            gn2 += g[i] * g[i];
        }
        if (gn2 == 0.0) {
            stalls[s] += 1;
            continue;
        }
        double step = 0.5 * R < s_ub ? 0.5 * R : s_ub;
        double gn = sqrt(gn2);
        for (int i = 0; i < d; ++i) xs[i] += step * g[i] / gn;
        path_len[s] += step;
    }
    return 0;
}

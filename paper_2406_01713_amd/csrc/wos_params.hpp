// wos_params.hpp -- parameter blocks shared by the host launcher and the walk
// kernels of libwos (internal; not part of the C ABI).
#pragma once
#include <stdint.h>

namespace wos {

constexpr int kMaxDim = 8;
constexpr int kMaxTerms = 96;      // Horner terms of the 0F1 weight series
constexpr int kBatchStride = 8;    // row stride of batched query / gradient arrays
constexpr int kWave = 64;          // CDNA wavefront width
constexpr uint32_t kDefaultMaxSteps = 1u << 16;
constexpr int kBatchStats = 16;    // columns of a batched stats row

enum Class : int32_t { kGoal = 0, kSphere = 1, kBox = 2, kOuter = 3, kArm = 4 };
enum Status : int32_t { kAbsorbed = 0, kDegenerate = 1, kTruncated = 2 };

// Row strides of the device obstacle tables (elements): a sphere row holds
// centre[d], radius; a box row holds centre[d], half_width[d].  Rows are
// padded to a multiple of 4 elements so scalar loads fetch whole rows.
__host__ __device__ constexpr int sph_stride(int d) { return ((d + 1 + 3) / 4) * 4; }
__host__ __device__ constexpr int box_stride(int d) { return ((2 * d + 3) / 4) * 4; }

// Obstacle clusters.  An environment with at least kClusterMin spheres (or
// boxes) also holds them regrouped into clusters of kCluster rows (leaves of a
// k-d split, the last one padded with rows far outside any domain), each with
// a bounding sphere in sphere-row layout.  A wave skips a cluster when the
// bound proves, for every active lane, that no member can be nearer than that
// lane's current distance, so the distance (value and component) is the one
// the full scan gives.
constexpr int kCluster = 8;
constexpr int kClusterMin = 64;

// Matrix-core form of the cluster test (FP32 kernels).  With walker features
//   a = [x (8 slots, 0 past d), |x|^2 (1 - m) - m thr^2, 1, thr^2, thr]
// and cluster features
//   b = [-2 C (8 slots), 1, |C|^2 (1 - m) - rho'^2 (1 + m), -1, -2 rho'],
// m = 2^-12, the dot product is |x - C|^2 - (thr + rho')^2 - m (|x|^2 + thr^2
// + |C|^2 + rho'^2); a cluster is skipped when it is positive for every
// walker of the wave.  The margin m (4096 units of rounding) exceeds the
// rounding of the products and of the members' own distances.  Cluster
// features are stored per tile of 16 clusters as 64 lanes x 4 floats: lane
// j + 16 k holds features k, 4 + k, 8 + k of cluster j of the tile (the B
// operand of three 16x16x4 products), the 4th float unused.  Padding
// clusters of the last tile, and one spare tile after it, have feature
// 9 = 1e30 (always skipped).
// Pair-compacted member scan: (walker, cluster) pairs that the matrix-core
// test keeps are queued per wave in LDS and taken 64 at a time, one pair per
// lane, through a second test against the cluster's bounding box; the pairs
// that pass go to a member queue and are evaluated 64 at a time (a step's
// last pairs join its last member round untested when they fit).  Between
// tiles fewer than 64 pairs wait in the first queue; a tile adds its pairs in
// one pass when they fit, else two need bits of every lane (at most 128
// pairs) at a time after the waiting ones are tested, so 256 entries never
// overflow.  The member queue holds fewer than 64 between rounds and gains
// at most 64 per round.
constexpr int kPairCap = 256;
constexpr int kBoxQueue = 2 * kWave;
// pair-scan LDS words per wave: first queue, member queue, then minima
constexpr int kPairLds = kPairCap + kBoxQueue + kWave;

// The bounding-box test runs by default where the obstacles depend on at
// least kBoxTestMinDim coordinates: below that a cluster's bounding sphere is
// nearly as tight as its box, and the test costs more than it saves.
constexpr int kBoxTestMinDim = 6;

// A walker's R at one step is at most twice its R at the step before (R is a
// minimum of 1-Lipschitz distances and the walker moves R), so that bound,
// with rounding margins, also thresholds the obstacle scans.  It pays where
// obstacles, not the outer box, are usually nearest: dense scenes in few
// dimensions (2-4x fewer clusters kept at d = 3-4, 1.3-1.5x at d = 5, under
// 5 % at d = 6-7, CPU walk simulation of the ragged batch); above
// kStepBoundMaxDim the kernels are built without it.
constexpr int kStepBoundMaxDim = 5;

// Cluster bounding boxes (FP32 kernels): per cluster lo[kMaxDim] then
// hi[kMaxDim] (zero past d), the box of the members enlarged by a margin
// (see build_cluster_boxes) and rounded outwards.
constexpr int kClusterBox = 2 * kMaxDim;

constexpr int kMfmaTile = 16;
constexpr int kMfmaFeat = 12;

// Per-environment parameters of one walk launch.  Read by every lane with
// wave-uniform addresses, so the compiler keeps them in scalar registers.
template <typename T>
struct EnvP {
    const T* sph;          // n_sph x sph_stride(d), caller's order
    const T* box;          // n_box x box_stride(d), caller's order
    const T* sph_cl;       // n_cl_sph x kCluster sphere rows, cluster order
    const T* box_cl;       // n_cl_box x kCluster box rows, cluster order
    const T* sph_bnd;      // n_cl_sph + 1 bounding spheres, sph_stride(d) each (last: unused)
    const T* box_bnd;      // n_cl_box + 1 bounding spheres, sph_stride(d) each (last: unused)
    const float* sph_mf;   // matrix-core cluster features, (ceil(n_cl_sph / 16) + 1) x 64 x 4 (FP32 only)
    const float* box_mf;
    const float* sph_cb;   // n_cl_sph x kClusterBox cluster bounding boxes (FP32 only)
    const float* box_cb;
    int32_t n_sph, n_box;
    int32_t n_cl_sph, n_cl_box;  // 0: scan the caller-order table instead
    int32_t use_mfma, box_test;  // FP32 cluster tests: 0 vector ALUs, 1 matrix cores with a
                                 // wave-uniform member scan, 2 matrix cores with pair compaction;
                                 // box_test (with 2): pairs pass the bounding-box test first
    int32_t d, has_goal;
    int32_t geom_d, pad_g;     // obstacles and the outer boundary depend on x[0..geom_d) only
    const T* arm_pts;          // planar arm: n_arm x 2 task-plane obstacle points
    int32_t n_arm, pad_arm;    // 0: no arm
    T arm_l[kMaxDim];          // link lengths, one per joint coordinate
    T arm_invK;                // 1 / K, K the arm's Lipschitz constant
    int32_t outer_kind, mode;  // outer: 0 box, 1 ball; mode: 0 class, 1 affine, 2 plane
    int32_t nt_C, nt_C1;       // Horner terms of 0F1(;d/2;y) and 0F1(;d/2+1;y)
    uint32_t key0, key1;       // Philox key (seed)
    uint32_t env_id, max_steps;
    T goal_c[kMaxDim];
    T goal_r;
    T lo[kMaxDim], hi[kMaxDim];
    T oc[kMaxDim];
    T orad;
    T g_goal, g_obs, g_outer, b;
    T ak[kMaxDim];
    T sigma, eps, qsigma;      // qsigma = 2^-m sigma / 4 (m: the series scale)
    T rb_abs;                  // absolute margin of the step-to-step bound on R (+inf: no bound)
    T cC[kMaxTerms];           // 2^(m k) c_k, c_k = 1 / ((d/2)_k k!)
    T cC1[kMaxTerms];          // 2^(m k) c_k, c_k = 1 / ((d/2 + 1)_k k!)
    // point source amp delta_z (has_src 0: none)
    int32_t has_src, pad_src;
    T src_z[kMaxDim];
    T src_amp, c_imp;
    T nu, sqrt_sigma;
    T phi_c;                   // sigma > 0: (2 pi)^(-d/2) sigma^(nu/2); sigma = 0: the Laplace constant
    T grad_c;                  // sigma > 0: (2 pi)^(-d/2) sigma^((nu+1)/2); sigma = 0: 1 / |S^(d-1)|
};

// Work decomposition of one environment inside a batched launch.
struct BatchEnv {
    int64_t q_off;      // first row of the env's queries in the batch arrays
    int64_t unit_off;   // first work-unit index of the env
    int64_t n_walks;    // walks per query of the env
    int32_t n_q;        // queries of the env
    int32_t splits;     // work units per query (walk ranges)
    int32_t wps;        // walks per work unit (last unit may be shorter)
    int32_t d;
    int32_t q_stride;   // row stride of the query array (elements)
    int32_t slot;       // position of the env in the caller's env array
    int32_t n_cl;       // cluster bounds evaluated per walk-step (spheres + boxes)
    int32_t lanes;      // lanes of a wave that carry walks (64 / lanes per walker)
};

// Accumulator layout of one work unit's partial sums (doubles):
// [0] sum u, [1] sum u^2, [2, 2+d) sum grad, [2+d, 2+2d) sum grad^2,
// [2+2d] sum steps, [3+2d] truncated, [4+2d] degenerate,
// [5+2d] sum u*S (d u/d sigma), [6+2d] sum W 1{goal} (d u/d g_goal),
// [7+2d] sphere distances evaluated, [8+2d] box distances evaluated,
// [9+2d] cluster bounding boxes tested.
__host__ __device__ constexpr int nacc(int d) { return 10 + 2 * d; }

}  // namespace wos

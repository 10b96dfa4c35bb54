// wos_launch.hpp -- host-side launchers of the libwos kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wos_params.hpp"

namespace wos {

// Plain walk kernel: one walk per lane, one wave per (query, 64-walk chunk),
// no refill.  Writes one partial-sum row per wave.  p is a device pointer;
// src selects the variant with point-source terms.
template <typename T>
hipError_t launch_plain(int d, bool bwd, bool src, const EnvP<T>* p, const T* queries, int64_t n_q,
                        int64_t n_walks, int64_t w_base, uint32_t q_base,
                        const uint64_t* key_add, double* partials, double* records,
                        hipStream_t st);

// Per-query means / standard errors (and backward products) from the plain
// kernel's partials.  prod (Q x 2) receives grad_u[q] * (du/dsigma, du/dg).
template <typename T>
hipError_t launch_finalize_plain(int d, bool bwd, const double* partials, int64_t n_q,
                                 int32_t chunks, int64_t n_walks, T* out_u, T* out_grad,
                                 double* out_stats, const T* ubar, T* out_dx, double* out_dq,
                                 double* prod, hipStream_t st);

// Deterministic sum of the Q x 2 products into two scalars.
hipError_t launch_reduce_pairs(const double* prod, int64_t n, double* out0, double* out1,
                               hipStream_t st);

// Persistent ragged-batch kernel (FP32): grid of resident waves pulling work
// units from *counter; refills lanes with the next walk of the unit.  src
// selects the variant with point-source terms (any env of the batch).
hipError_t launch_persistent(bool bwd, bool src, int grid, int block, const EnvP<float>* envs,
                             const BatchEnv* benv, int n_benv, const float* queries,
                             int64_t total_units, uint32_t key0, uint32_t key1,
                             const uint64_t* key_add, unsigned* counter, double* partials,
                             hipStream_t st);

// Resident waves of the persistent kernel for a block size (occupancy x CUs).
int persistent_resident_blocks(bool bwd, bool src, int block);

// Outputs of a batched launch; one block per env; also resets *counter.
// out_dir (optional, rows like out_grad) receives grad / |grad| formed from
// the FP64 sums, so it exists where the mean gradient is below FP32 range.
hipError_t launch_finalize_batch(bool bwd, const BatchEnv* benv, int n_benv,
                                 const double* partials, const float* ubar,
                                 float* out_u, float* out_grad, int grad_stride,
                                 double* out_stats, float* out_dx, double* out_dsigma,
                                 double* out_dg, float* out_dir, unsigned* counter, hipStream_t st);

// One planning update: x += min(s_ub, R/2) dir, dir the unit gradient
// direction (a zero row counts a stall); bumps *step.
hipError_t launch_plan_update(int d, const EnvP<float>* p, float* x, int64_t n, const float* dir,
                              int grad_stride, float s_ub, double* path_len, int32_t* stalls,
                              int32_t* status, uint64_t* step, hipStream_t st);

// Varadhan read-out w = -sqrt(1/sigma) ln u (and its gradient when grad and
// grad_w are given, rows of `stride` elements, first d used).
template <typename T>
hipError_t launch_varadhan(const T* u, const T* grad, int64_t n, int d, int stride, double sigma, T* w,
                           T* grad_w, hipStream_t st);

// Fill kernels (used instead of hipMemsetAsync so the calls are capturable).
hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);

}  // namespace wos

// Launchers of the HIP kernels (kernels.hip, apply_mfma.hip, krylov.hip),
// called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace kp {

hipError_t launch_build_blocks(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                               const double* params, double* out);
// workspace slots of the setup kernels for E elements: a multiple of 4 (one
// wave per element, four per workgroup), at most 2048
constexpr size_t kSetupWavesLdsMax = 150 * 1024;
inline int setup_slots(int64_t E) {
    const int64_t g = E < 2048 ? E : 2048;
    return (int)((g + 3) / 4 * 4);
}
hipError_t launch_setup(hipStream_t s, int grid, int64_t E, int dim, int n, int rank,
                        const Tables1D* tab, const double* params, const double* blocks,
                        const double* guess, double* factors, double* sigma, int32_t* status,
                        double* ws, int64_t ws_stride, const int32_t* skip = nullptr,
                        int32_t status_or = 0, const double* grams = nullptr);
// stage-1 Gram matrices R(A) R(A)^T of explicit blocks with n^2 <= 64, grams
// [E][n^2][n^2] (for launch_setup's grams)
hipError_t launch_explicit_gram(hipStream_t s, int64_t E, int dim, int n, const double* blocks, double* grams);
// learned setup: the judge of predicted factors `pred` against the SVD's
// (`factors` with their FP64 tables, learned.h); out [E][4] and accept [E]
// optional; use_pred: accepted predictions replace the factors (status 0),
// rejected elements' status gains status_rejected
size_t learned_judge_lds(int dim, int n);
hipError_t launch_learned_judge(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                                const double* params, const double* pred, double* factors, const double* tab64,
                                int64_t tab_stride, const int8_t* kinds, double factor, double guard,
                                double* out, int32_t* accept, int32_t* status, bool use_pred,
                                int32_t status_rejected);
// guess[e] = vec A1 (and vec B1 in 3D) of predicted factors: [E][2 or 1][n^2]; accept[e] = 0
hipError_t launch_learned_guess(hipStream_t s, int64_t E, int dim, int n, const double* factors,
                                double* guess, int32_t* accept);
// skip[e] = accept[e] || !(status[e] & KP_ELEM_LANCZOS_NOCONV)
hipError_t launch_fallback_mask(hipStream_t s, int64_t E, const int32_t* accept, const int32_t* status,
                                int32_t* skip);
// apply tables from the factors (three kernels: prepare, Schur, finish);
// prepare and finish run on four waves per element when their scratch fits
constexpr size_t kTables4LdsMax = 144 * 1024;
// apply tables from the factors (three kernels: prepare, Schur, finish)
struct MixedElem;
hipError_t launch_form_tables(hipStream_t s, int64_t E, int dim, int n, int rank,
                              const double* factors, double* tab64, int8_t* kinds,
                              int32_t* status);
// the same (rank 2) for the count elements list[0, count) of one (dim, n)
// class of a mixed batch, at the factor and table offsets of their descriptors
hipError_t launch_form_tables_list(hipStream_t s, int64_t count, const int32_t* list, const MixedElem* el,
                                   int dim, int n, const double* factors, double* tab64, int8_t* kinds,
                                   int32_t* status);
// rank-3 2D apply (inner flexible GMRES per element); LDS budget and restart length
constexpr size_t kRank3LdsMax = 150 * 1024;
int rank3_restart(int n);
// only: per-element flags, or null; with flags, only the flagged elements
// are solved (the rest of z is left as it is)
hipError_t launch_apply_rank3(hipStream_t s, int prec, int64_t E, int n, int nrhs,
                              const double* factors, const void* tabs, int64_t tab_stride,
                              const int8_t* kinds, const double* r, double* z, const int8_t* only = nullptr);
// 2D rank 3 with n = 16 on the matrix cores (apply_mfma.hip): the Neumann
// series of P2^{-1} (A3 (x) B3) over the rank-2 apply, 16 right-hand sides per
// workgroup; flags[e] (int8, zeroed by the caller) is set for an element whose
// series did not converge, for launch_apply_rank3 with only = flags.
hipError_t launch_apply16_rank3(hipStream_t s, int prec, int64_t E, int nrhs, const void* tabs,
                                int64_t tab_stride, const int8_t* kinds, const double* factors, const double* r,
                                double* z, int8_t* flags);
hipError_t launch_cast_tables(hipStream_t s, int64_t count, const double* t64, float* t32,
                              uint16_t* hi, uint16_t* lo, float* t2);
// n = 16 matrix-core apply (apply_mfma.hip); grid cap of its persistent loop.
// tabs: row-major tables of the precision.
constexpr int64_t kApply16Grid = 1 << 20;
// axes: the 3D elements' split axes (kp_setup with KP_OPT_SPLIT_AXIS), or NULL
// (every element split on x)
hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const int8_t* kinds, const double* r, double* z,
                          const int8_t* axes = nullptr);
hipError_t launch_apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs,
                                const void* tabs, int64_t tab_stride, const int8_t* kinds,
                                const double* r, double* z, const int8_t* axes = nullptr);
// the same two with z stored in FP32 (prec FP32, BF16, split BF16 only: their
// results are FP32 numbers, stored exactly; prec FP64 is refused)
hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const int8_t* kinds, const double* r, float* z,
                          const int8_t* axes = nullptr);
hipError_t launch_apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs,
                                const void* tabs, int64_t tab_stride, const int8_t* kinds,
                                const double* r, float* z, const int8_t* axes = nullptr);

// split-axis choice of the 3D setup: the records relabelled for axes 1 and 2
// (out [2][E][16]); the per-element choice by the largest stage-1 sigma_1
// (axis 0 in place, axes 1 and 2 in fac/sig/st [2][E][...]); a byte fill
hipError_t launch_permute_records(hipStream_t s, int64_t E, const double* params, double* out);
hipError_t launch_choose_axis(hipStream_t s, int64_t E, int64_t nfnn, const double* fac, const double* sig,
                              const int32_t* st, double* factors, double* sigma, int32_t* status, int8_t* axis);
hipError_t launch_fill_i8(hipStream_t s, int64_t count, int8_t* p, int8_t v);

// setup of general elements (quad.h, quad.hip): one workgroup per element,
// grid workspace slots of ws_stride = quad_setup_doubles(dim, n, mu) doubles
struct QuadTables;
hipError_t launch_setup_quad(hipStream_t s, int grid, int64_t E, int dim, int n, int mu, double tau,
                             const QuadTables* qt, const double* c, const double* a, const double* nu,
                             const double* g, double* factors, double* sigma, int32_t* status, double* ws,
                             int64_t ws_stride);

// 3D elements with n <= 8 (apply_small.hip): one wave per (element, rhs),
// the tensor as register fibres; the arithmetic of the generic apply
hipError_t launch_apply_small3(hipStream_t s, int prec, int64_t E, int n, int nrhs, const void* tabs,
                               int64_t tab_stride, const int8_t* kinds, const double* r, double* z,
                               const int8_t* axes);
hipError_t launch_apply_small3(hipStream_t s, int prec, int64_t E, int n, int nrhs, const void* tabs,
                               int64_t tab_stride, const int8_t* kinds, const double* r, float* z,
                               const int8_t* axes);

// systems blocks (sys.h, sys.hip): setup with one workgroup per element over
// grid workspace slots of ws_stride doubles (angle: E int32 scratch for the
// pair rotations); apply with one workgroup per
// (element, right-hand side) in FP64 (prec 0) or FP32 (prec 1) tables and
// arithmetic
hipError_t launch_setup_sys(hipStream_t s, int grid, int64_t E, int nc, int n, const double* blocks,
                            char* precond, double* ws, int64_t ws_stride, int32_t* angle);
hipError_t launch_build_sys_blocks(hipStream_t s, int64_t E, int nc, int n, const Tables1D* tab, const double* recs,
                                   double* out);
hipError_t launch_sys_operator(hipStream_t s, int64_t E, int N, const double* blocks, const double* x, double* y);
hipError_t launch_apply_sys(hipStream_t s, int64_t E, int nc, int n, int prec, int nrhs, const char* precond,
                            const double* r, double* z);

}  // namespace kp

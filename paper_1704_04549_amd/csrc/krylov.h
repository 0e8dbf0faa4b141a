// Launchers of the global operator, FGMRES vector kernels and exact block Jacobi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace kp {

constexpr int kVecBlocks = 8192;  // grid of the vector kernels (and partial-sum rows)

// strc: the elements' structure (mass n^d, then Xax 3 n^2, per element) from
// launch_structure, or null to form it from the records in every call.
// cols: 3D elements with n <= 16 and strc take the column-per-thread kernel
// (the same terms in the same order); false keeps the one-entry-per-thread
// kernel.
hipError_t launch_operator(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                           const double* params, const int32_t* nbr, const double* blocks,
                           const double* strc, const double* x, double* y, bool cols = true);
// the same with x stored in FP32
hipError_t launch_operator(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                           const double* params, const int32_t* nbr, const double* blocks,
                           const double* strc, const float* x, double* y, bool cols = true);
hipError_t launch_structure(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                            const double* params, double* strc);
hipError_t launch_mdot(hipStream_t s, const double* V, int64_t ldv, int k, const double* w,
                       int64_t N, double* partial, double* out, int accumulate);
hipError_t launch_mgs_update(hipStream_t s, const double* V, int64_t ldv, int k, const double* h,
                             double* w, int64_t N);
hipError_t launch_combine(hipStream_t s, const double* Z, int64_t ldz, int k, const double* y,
                          double* x, int64_t N);
hipError_t launch_combine(hipStream_t s, const float* Z, int64_t ldz, int k, const double* y,
                          double* x, int64_t N);
hipError_t launch_axpby(hipStream_t s, double* dst, const double* src, double a, const double* other,
                        double b, int64_t N);
// vn = w / sqrt(max(*nrm2, 0)) with the norm read on the device (zeros for a
// zero norm)
hipError_t launch_normalize(hipStream_t s, const double* nrm2, const double* w, double* vn, int64_t N);
hipError_t launch_bj_factor(hipStream_t s, int64_t E, int N, const double* blocks, double* lu,
                            int32_t* piv, int32_t* status);
hipError_t launch_bj_solve(hipStream_t s, int64_t E, int N, int nrhs, const double* lu,
                           const int32_t* piv, const double* r, double* z);

}  // namespace kp

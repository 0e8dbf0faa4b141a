// Mixed batches: elements of different dimension and degree in one batch.
//
// Every element has a descriptor (dimension, n and its offsets in the packed
// vectors, factors and tables); the persistent kernels of mixed.hip read the
// descriptor of each element they process, so one launch covers the whole
// batch.  Vectors are packed in element order: element e holds n_e^d_e values
// at vec_off[e].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "elem_ops.h"
#include "kernels.h"

namespace kp {

struct MixedElem {
    int32_t dim, n;
    int64_t vec_off;  // doubles, in the packed vectors
    int64_t fac_off;  // doubles, in the factor section (5 n^2 in 3D, 4 n^2 in 2D)
    int64_t tab_off;  // entries, in every table section ((7 + n) n^2 each)
};

// Apply work list: item i < n_block is one element processed by the whole
// workgroup (items[4 i]); the others hold up to four elements (-1: none),
// one per wave, each processed by its wave alone.
constexpr int kMixedItemWidth = 4;

// Entries of the apply's third LDS buffer for one element: the Sylvester
// sweep's 2 x 2-block right-hand sides, two n-vectors per slice (one slice in
// 2D, n in 3D).
inline long mixed_apply_h(int dim, int n) { return 2L * n * (dim == 3 ? n : 1); }

// Dynamic LDS of one apply launch: per workgroup item the tensor, one scratch
// tensor and the block buffer (2 block_nd + block_h entries); per wave of a
// wave item the same for its own element (2 wave_nd + wave_h each).  A launch
// above the limit is refused; a (dim, n) class takes the wave mode only if it
// fits at FP64, so one work list serves every precision.
constexpr size_t kMixedApplyLdsMax = 150 * 1024;
inline size_t mixed_apply_lds(size_t elem_bytes, long block_nd, long block_h, long wave_nd, long wave_h) {
    const long blk = 2 * block_nd + block_h;
    const long wav = kMixedItemWidth * (2 * wave_nd + wave_h);
    return (size_t)(blk > wav ? blk : wav) * elem_bytes;
}

hipError_t launch_mixed_setup(hipStream_t s, int grid, int64_t E, const MixedElem* el, const int32_t* order,
                              Tables1D* const* tabs, const double* params, double* factors, double* sigma,
                              int32_t* status, double* ws, int64_t ws_stride, size_t small_doubles);
// the wave form: order lists its elements only; grid4 workgroups serve
// 4 * grid4 workspace slots of ws_stride doubles; small_stride: the LDS part
// of one wave (doubles)
hipError_t launch_mixed_setup_waves(hipStream_t s, int grid4, int64_t E, const MixedElem* el,
                                    const int32_t* order, Tables1D* const* tabs, const double* params,
                                    double* factors, double* sigma, int32_t* status, double* ws,
                                    int64_t ws_stride, int64_t small_stride);
hipError_t launch_mixed_apply(hipStream_t s, int prec, int grid, int n_items, int n_block, const int32_t* items,
                              const MixedElem* el, const void* tabs, const int8_t* kinds, const double* r,
                              double* z, long block_nd, long block_h, long wave_nd, long wave_h);
hipError_t launch_mixed_operator(hipStream_t s, int64_t E, const MixedElem* el, Tables1D* const* tabs,
                                 const double* params, const double* x, double* y, int max_n, int max_nd);

}  // namespace kp

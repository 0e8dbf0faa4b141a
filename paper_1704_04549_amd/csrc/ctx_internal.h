// Internal to the library: the context behind a kp_ctx and the helpers
// shared by the entry points (argument checks, workspace, 1D tables).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <functional>

#include "../../include/kp.h"
#include "tables.h"

using namespace kp;

struct kp_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    Tables1D* d_tables[kMaxN + 1] = {};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int num_cus = 256;
    // FGMRES / operator scratch
    void* ks = nullptr;
    size_t ks_bytes = 0;
    // the matrix-free operator's per-element structure (mass tensor and axis
    // matrices), formed once per FGMRES solve
    void* strc = nullptr;
    size_t strc_bytes = 0;
    // matrix-core apply for n = 16 (KP_APPLY_GENERIC=1 in the environment selects
    // the generic per-element kernel instead, for comparison)
    bool use_mfma16 = true;
    // learned setup: MLP workspace and the model attached with kp_set_model
    void* mw = nullptr;
    size_t mw_bytes = 0;
    const void* model = nullptr;
    int model_dim = 0, model_n = 0, model_hidden = 0;
    // FGMRES steps as HIP graphs: a private stream for capture (default
    // priority) and pinned host memory for the projections
    bool use_graphs = false;
    bool fgmres_z32 = true;
    bool op_cols = true;     // column-per-thread operator kernel for 3D n <= 16 (matrix-free)  // FP32 basis Z where the preconditioner's outputs are FP32 numbers
    hipStream_t cap_stream = nullptr;
    double* pinned = nullptr;
    size_t pinned_doubles = 0;
    // device address of the allocation-free setup's scratch array on this
    // context's device (kp_setup_noalloc), or NULL if it could not be resolved
    double* scratch = nullptr;
    // 3D split-axis choice (KP_OPT_SPLIT_AXIS)
    bool split_axis = false;
    // tables of general elements per (n, mu), uploaded on first use
    void* d_quad[kMaxN + 1][kMaxN + 1] = {};
    // 3D n <= 8 apply with one wave per element (KP_OPT_APPLY_SMALL3)
    bool use_small3 = true;
    // spectral guard of the learned setup (KP_OPT_LEARNED_GUARD)
    double learned_guard = 0.01;
};

#define KP_HIP(call)                                   \
    do {                                               \
        hipError_t err_ = (call);                      \
        if (err_ != hipSuccess) return KP_ERR_HIP;     \
    } while (0)

static inline kp_status ensure_ws(kp_ctx c, size_t bytes, void** slot, size_t* cap) {
    if (*cap >= bytes && *slot) return KP_OK;
    if (*slot) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return KP_ERR_HIP;
        hipFree(*slot);
        *slot = nullptr;
        *cap = 0;
    }
    size_t want = bytes + bytes / 8 + 256;
    if (hipMalloc(slot, want) != hipSuccess) {
        *slot = nullptr;
        return KP_ERR_ALLOC;
    }
    *cap = want;
    return KP_OK;
}

static inline kp_status get_tables(kp_ctx c, int n, const Tables1D** out) {
    if (n < 2 || n > kMaxN) return KP_ERR_ARG;
    if (!c->d_tables[n]) {
        Tables1D h;
        if (!make_tables(n, &h)) return KP_ERR_ARG;
        Tables1D* d = nullptr;
        if (hipMalloc((void**)&d, sizeof(Tables1D)) != hipSuccess) return KP_ERR_ALLOC;
        if (hipMemcpy(d, &h, sizeof(Tables1D), hipMemcpyHostToDevice) != hipSuccess) {
            hipFree(d);
            return KP_ERR_HIP;
        }
        c->d_tables[n] = d;
    }
    *out = c->d_tables[n];
    return KP_OK;
}

static inline kp_status check_batch(const kp_batch* b, bool need_params = true) {
    if (!b) return KP_ERR_ARG;
    if (b->num_elems < 0) return KP_ERR_ARG;
    if (b->dim != 2 && b->dim != 3) return KP_ERR_ARG;
    if (b->n < 2 || b->n > kMaxN) return KP_ERR_ARG;
    if (need_params && !b->params && b->num_elems > 0) return KP_ERR_ARG;
    return KP_OK;
}


// a device-vector map (operator or preconditioner) for the FGMRES driver
typedef std::function<kp_status(const double*, double*)> VecFn;
// the preconditioned basis Z kept in FP32: the preconditioner writes z_j in
// FP32 and the operator reads it (used where the preconditioner's outputs are
// FP32 numbers, so that the basis holds exactly what an FP64 one would)
struct Z32Fns {
    std::function<kp_status(const double*, float*)> pc;
    std::function<kp_status(const float*, double*)> op;
};
kp_status fgmres_core(kp_ctx c, int64_t N, const VecFn& op, const VecFn& pc, const double* rhs, double* x,
                      int32_t restart, double rtol, int32_t maxit, int32_t* iters_h, double* relres_h,
                      double* hist_h, int32_t hist_len, const Z32Fns* z32 = nullptr);

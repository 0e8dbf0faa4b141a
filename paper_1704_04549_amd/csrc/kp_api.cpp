// C ABI of the KSVD preconditioner library (include/kp.h).
//
// Argument checking, workspace management, precondioner-buffer layout and
// kernel dispatch.  No numerical work happens on the host.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/kp.h"
#include "kernels.h"
#include "krylov.h"
#include "layout.h"
#include "quad.h"
#include "tables.h"
#include "ctx_internal.h"

using namespace kp;

// Scratch of the allocation-free setup (kp_setup_noalloc): the Lanczos
// workspace slots of the setup kernels, 128 MiB on every device the library
// runs on, held until the process ends.  Host code never passes the array's
// name to a kernel: kp_create resolves its device address once per device
// (hipGetSymbolAddress, with that device current) and every use goes through
// that address.
constexpr size_t kNoAllocScratchDoubles = (size_t)16 * 1024 * 1024;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device `device` (resolved once)
static double* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        double* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

// the learned setup's acceptance: residual within 1.1x the SVD's (the guard
// is a context option, KP_OPT_LEARNED_GUARD)
constexpr double kLearnedFactor = 1.1;
constexpr size_t kJudgeLdsMax = 150 * 1024;

extern "C" {

const char* kp_status_string(kp_status s) {
    switch (s) {
        case KP_OK: return "ok";
        case KP_ERR_ARG: return "invalid argument";
        case KP_ERR_ALLOC: return "device allocation failed";
        case KP_ERR_HIP: return "HIP runtime error";
        case KP_ERR_NUMERIC: return "numerical failure";
        case KP_ERR_NOCONV: return "not converged";
        case KP_ERR_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

kp_status kp_create(kp_ctx* ctx, int device, void* stream) {
    if (!ctx) return KP_ERR_ARG;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return KP_ERR_HIP;
    if (device < 0 || device >= count) return KP_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return KP_ERR_HIP;
    kp_ctx c = new (std::nothrow) kp_ctx_s();
    if (!c) return KP_ERR_ALLOC;
    c->device = device;
    c->stream = (hipStream_t)stream;
    const char* gen = getenv("KP_APPLY_GENERIC");
    c->use_mfma16 = !(gen && gen[0] == '1');
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    // the 1D tables of every supported n, so that no later call allocates them
    for (int n = 2; n <= kMaxN; ++n) {
        const Tables1D* T;
        kp_status st = get_tables(c, n, &T);
        if (st != KP_OK) {
            kp_destroy(c);
            return st;
        }
    }
    c->scratch = scratch_address(device);
    *ctx = c;
    return KP_OK;
}

kp_status kp_destroy(kp_ctx c) {
    if (!c) return KP_ERR_ARG;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (int n = 0; n <= kMaxN; ++n)
        if (c->d_tables[n]) hipFree(c->d_tables[n]);
    for (int n = 0; n <= kMaxN; ++n)
        for (int m = 0; m <= kMaxN; ++m)
            if (c->d_quad[n][m]) hipFree(c->d_quad[n][m]);
    if (c->ws) hipFree(c->ws);
    if (c->ks) hipFree(c->ks);
    if (c->strc) hipFree(c->strc);
    if (c->mw) hipFree(c->mw);
    if (c->pinned) hipHostFree(c->pinned);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
    return KP_OK;
}

kp_status kp_set_option(kp_ctx c, int32_t option, int64_t value) {
    if (!c) return KP_ERR_ARG;
    switch (option) {
        case KP_OPT_FGMRES_GRAPHS: c->use_graphs = value != 0; return KP_OK;
        case KP_OPT_APPLY_MFMA16: c->use_mfma16 = value != 0; return KP_OK;
        case KP_OPT_FGMRES_Z32: c->fgmres_z32 = value != 0; return KP_OK;
        case KP_OPT_OPERATOR_COLS: c->op_cols = value != 0; return KP_OK;
        case KP_OPT_SPLIT_AXIS: c->split_axis = value != 0; return KP_OK;
        case KP_OPT_APPLY_SMALL3: c->use_small3 = value != 0; return KP_OK;
        case KP_OPT_LEARNED_GUARD:
            if (value < 0 || value > 1000000) return KP_ERR_ARG;
            c->learned_guard = (double)value * 1e-6;
            return KP_OK;
    }
    return KP_ERR_ARG;
}

kp_status kp_set_stream(kp_ctx c, void* stream) {
    if (!c) return KP_ERR_ARG;
    c->stream = (hipStream_t)stream;
    return KP_OK;
}

size_t kp_precond_bytes(int32_t dim, int32_t n, int32_t rank, int64_t num_elems) {
    PcLayout L;
    if (!pc_layout(dim, n, rank, num_elems, &L)) return 0;
    return L.total;
}

kp_status kp_build_blocks(kp_ctx c, const kp_batch* b, double* out) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    if (!out && b->num_elems > 0) return KP_ERR_ARG;
    if (b->num_elems == 0) return KP_OK;
    const Tables1D* T;
    if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
    KP_HIP(launch_build_blocks(c->stream, b->num_elems, b->dim, b->n, T, b->params, out));
    return KP_OK;
}

static kp_status finish_tables(kp_ctx c, const kp_batch* b, int rank, char* pc, const PcLayout& L) {
    const int64_t E = b->num_elems;
    KP_HIP(launch_form_tables(c->stream, E, b->dim, b->n, rank, (const double*)(pc + L.factors),
                              (double*)(pc + L.t64), (int8_t*)(pc + L.kinds),
                              (int32_t*)(pc + L.status)));
    KP_HIP(launch_cast_tables(c->stream, E * L.ne, (const double*)(pc + L.t64), (float*)(pc + L.t32),
                              (uint16_t*)(pc + L.thi), (uint16_t*)(pc + L.tlo),
                              (float*)(pc + L.t2)));
    return KP_OK;
}

static kp_status copy_status(kp_ctx c, const kp_batch* b, const char* pc, const PcLayout& L,
                             int32_t* elem_status) {
    if (elem_status && b->num_elems > 0)
        KP_HIP(hipMemcpyAsync(elem_status, pc + L.status, b->num_elems * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_setup(kp_ctx c, const kp_batch* b, int32_t rank, int32_t mode, void* precond,
                   int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    if (!precond && b->num_elems > 0) return KP_ERR_ARG;
    if (mode != KP_SETUP_SVD && mode != KP_SETUP_LEARNED && mode != KP_SETUP_LEARNED_WARM)
        return KP_ERR_ARG;
    if (b->dim == 3 && b->blocks && b->n * b->n > 64) return KP_ERR_UNSUPPORTED;
    // the split-axis choice relabels element records (3D, records only)
    if (c->split_axis && b->dim == 3 && b->blocks) return KP_ERR_UNSUPPORTED;
    if (mode != KP_SETUP_SVD) {
        // a model for this (dim, n), rank 2, records only, the judge's scratch in LDS
        if (!c->model || c->model_dim != b->dim || c->model_n != b->n) return KP_ERR_ARG;
        if (rank != 2 || b->blocks) return KP_ERR_UNSUPPORTED;
        if (learned_judge_lds(b->dim, b->n) > kJudgeLdsMax) return KP_ERR_UNSUPPORTED;
    }
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    const Tables1D* T;
    if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
    hipSetDevice(c->device);
    const bool expl = b->blocks != nullptr;
    const int64_t wsd = setup_work_doubles(b->dim, b->n, expl, rank);
    const int grid = setup_slots(E);
    if ((st = ensure_ws(c, (size_t)wsd * grid * sizeof(double), &c->ws, &c->ws_bytes)) != KP_OK)
        return st;
    char* pc = (char*)precond;
    double* factors = (double*)(pc + L.factors);
    double* sigma = (double*)(pc + L.sigma);
    int32_t* status = (int32_t*)(pc + L.status);
    int8_t* axis = (int8_t*)(pc + L.axis);
    const bool choose_axis = c->split_axis && b->dim == 3;
    if (choose_axis && mode != KP_SETUP_SVD) return KP_ERR_UNSUPPORTED;
    if (!choose_axis) KP_HIP(launch_fill_i8(c->stream, E, axis, 0));
    if (mode == KP_SETUP_SVD && choose_axis) {
        // the two-stage KSVD split on each axis (records relabelled for y and
        // z); per element the axis whose rank-1 stage keeps the most of ||A||_F
        const size_t nfnn = (size_t)L.nf * b->n * b->n;
        if ((st = ensure_ws(c, 2 * E * (kRecLen + nfnn + 4) * sizeof(double) + 2 * E * sizeof(int32_t) + 1024,
                            &c->ks, &c->ks_bytes)) != KP_OK)
            return st;
        double* recs = (double*)c->ks;
        double* fac = recs + 2 * E * kRecLen;
        double* sig = fac + 2 * E * nfnn;
        int32_t* st2 = (int32_t*)(sig + 2 * E * 4);
        KP_HIP(launch_permute_records(c->stream, E, b->params, recs));
        KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, b->params, nullptr, nullptr, factors,
                            sigma, status, (double*)c->ws, wsd));
        for (int k = 0; k < 2; ++k)
            KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, recs + k * E * kRecLen, nullptr,
                                nullptr, fac + k * E * nfnn, sig + k * E * 4, st2 + k * E, (double*)c->ws, wsd));
        KP_HIP(launch_choose_axis(c->stream, E, nfnn, fac, sig, st2, factors, sigma, status, axis));
    } else if (mode == KP_SETUP_SVD) {
        // explicit blocks with n^2 <= 64: their stage-1 Gram matrices first, on
        // the matrix cores, each block read once
        const double* grams = nullptr;
        if (b->blocks && (long)b->n * b->n <= kGramMax) {
            const size_t gbytes = (size_t)E * b->n * b->n * b->n * b->n * sizeof(double);
            if ((st = ensure_ws(c, gbytes, &c->ks, &c->ks_bytes)) != KP_OK) return st;
            KP_HIP(launch_explicit_gram(c->stream, E, b->dim, b->n, b->blocks, (double*)c->ks));
            grams = (const double*)c->ks;
        }
        KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, b->params, b->blocks, nullptr,
                            factors, sigma, status, (double*)c->ws, wsd, nullptr, 0, grams));
    } else {
        // 1. predicted factors into the context's scratch
        const size_t nn = (size_t)b->n * b->n;
        const size_t gs = b->dim == 3 ? 2 : 1;
        const size_t pred_d = E * L.nf * nn;
        if ((st = ensure_ws(c, (pred_d + E * gs * nn) * sizeof(double) + 2 * E * sizeof(int32_t) + 1024,
                            &c->ks, &c->ks_bytes)) != KP_OK)
            return st;
        double* pred = (double*)c->ks;
        double* guess = pred + pred_d;
        int32_t* accept = (int32_t*)(guess + E * gs * nn);
        int32_t* skip = accept + E;
        if ((st = kp_mlp_predict(c, c->model, b, KP_FP32, pred)) != KP_OK) return st;
        // 2. the SVD (the judge, and the fallback): Lanczos started from the
        //    prediction (vec A1; in 3D the second stage from vec B1), then a
        //    cold Lanczos where that did not converge
        KP_HIP(launch_learned_guess(c->stream, E, b->dim, b->n, pred, guess, accept));
        KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, b->params, nullptr, guess, factors,
                            sigma, status, (double*)c->ws, wsd, nullptr, KP_ELEM_LEARNED_WARM));
        KP_HIP(launch_fallback_mask(c->stream, E, accept, status, skip));
        KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, b->params, nullptr, nullptr,
                            factors, sigma, status, (double*)c->ws, wsd, skip, 0));
        if (mode == KP_SETUP_LEARNED) {
            // 3. tables of the SVD's factors, the judge, and the tables again
            //    (those of the accepted predictions; the other elements' factors
            //    are unchanged, so are their tables)
            if ((st = finish_tables(c, b, rank, pc, L)) != KP_OK) return st;
            KP_HIP(launch_learned_judge(c->stream, E, b->dim, b->n, T, b->params, pred, factors,
                                        (const double*)(pc + L.t64), L.ne, (const int8_t*)(pc + L.kinds),
                                        kLearnedFactor, c->learned_guard, nullptr, nullptr, status, true,
                                        KP_ELEM_LEARNED_REJECTED));
        }
    }
    if ((st = finish_tables(c, b, rank, pc, L)) != KP_OK) return st;
    return copy_status(c, b, pc, L, elem_status);
}

kp_status kp_setup_noalloc(kp_ctx c, const kp_batch* b, int32_t rank, void* precond,
                           int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    if (!precond && b->num_elems > 0) return KP_ERR_ARG;
    if (b->dim == 3 && b->blocks && b->n * b->n > 64) return KP_ERR_UNSUPPORTED;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!c->scratch) return KP_ERR_HIP;
    if (c->split_axis && b->dim == 3) return KP_ERR_UNSUPPORTED;
    // the tables were built by kp_create; nothing here allocates
    const Tables1D* T = c->d_tables[b->n];
    if (!T) return KP_ERR_HIP;
    hipSetDevice(c->device);
    const bool expl = b->blocks != nullptr;
    const int64_t wsd = setup_work_doubles(b->dim, b->n, expl, rank);
    // as many workspace slots as the scratch holds (a multiple of 4), at most
    // the number kp_setup uses; fewer slots only serialise more elements per slot
    int64_t cap = (int64_t)(kNoAllocScratchDoubles / (size_t)wsd) / 4 * 4;
    if (cap < 4) return KP_ERR_UNSUPPORTED;
    int64_t grid = setup_slots(E);
    if (grid > cap) grid = cap;
    char* pc = (char*)precond;
    KP_HIP(launch_fill_i8(c->stream, E, (int8_t*)(pc + L.axis), 0));
    KP_HIP(launch_setup(c->stream, (int)grid, E, b->dim, b->n, rank, T, b->params, b->blocks, nullptr,
                        (double*)(pc + L.factors), (double*)(pc + L.sigma), (int32_t*)(pc + L.status),
                        c->scratch, wsd));
    if ((st = finish_tables(c, b, rank, pc, L)) != KP_OK) return st;
    return copy_status(c, b, pc, L, elem_status);
}

kp_status kp_learned_judge(kp_ctx c, const kp_batch* b, int32_t rank, const double* pred_factors,
                           const void* precond, double factor, double guard, double* out, int32_t* accept) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    PcLayout L;
    if (rank != 2 || !pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    if (b->blocks) return KP_ERR_UNSUPPORTED;
    if (learned_judge_lds(b->dim, b->n) > kJudgeLdsMax) return KP_ERR_UNSUPPORTED;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!pred_factors || !precond || (!out && !accept)) return KP_ERR_ARG;
    const Tables1D* T;
    if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
    const char* pc = (const char*)precond;
    KP_HIP(launch_learned_judge(c->stream, E, b->dim, b->n, T, b->params, pred_factors,
                                (double*)(pc + L.factors), (const double*)(pc + L.t64), L.ne,
                                (const int8_t*)(pc + L.kinds), factor, guard, out, accept, nullptr, false, 0));
    return KP_OK;
}

kp_status kp_setup_quad(kp_ctx c, const kp_quad_batch* q, void* precond, int32_t* elem_status) {
    if (!c || !q) return KP_ERR_ARG;
    if (q->num_elems < 0 || (q->dim != 2 && q->dim != 3)) return KP_ERR_ARG;
    if (q->n < 2 || q->mu < q->n || q->mu > kQuadMaxMu) return KP_ERR_ARG;
    PcLayout L;
    if (!pc_layout(q->dim, q->n, 2, q->num_elems, &L)) return KP_ERR_ARG;
    const int64_t E = q->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !q->c || !q->a || !q->nu || !q->g) return KP_ERR_ARG;
    hipSetDevice(c->device);
    if (!c->d_quad[q->n][q->mu]) {
        QuadTables* h = new (std::nothrow) QuadTables;
        if (!h) return KP_ERR_ALLOC;
        if (!make_quad_tables(q->n, q->mu, h)) {
            delete h;
            return KP_ERR_ARG;
        }
        void* d = nullptr;
        if (hipMalloc(&d, sizeof(QuadTables)) != hipSuccess) {
            delete h;
            return KP_ERR_ALLOC;
        }
        const hipError_t err = hipMemcpy(d, h, sizeof(QuadTables), hipMemcpyHostToDevice);
        delete h;
        if (err != hipSuccess) {
            hipFree(d);
            return KP_ERR_HIP;
        }
        c->d_quad[q->n][q->mu] = d;
    }
    const int64_t wsd = (quad_setup_doubles(q->dim, q->n, q->mu) + 31) / 32 * 32;
    const int grid = (int)(E < 2048 ? E : 2048);
    kp_status st;
    if ((st = ensure_ws(c, (size_t)wsd * grid * sizeof(double), &c->ws, &c->ws_bytes)) != KP_OK) return st;
    char* pc = (char*)precond;
    KP_HIP(launch_fill_i8(c->stream, E, (int8_t*)(pc + L.axis), 0));
    KP_HIP(launch_setup_quad(c->stream, grid, E, q->dim, q->n, q->mu, q->tau,
                             (const QuadTables*)c->d_quad[q->n][q->mu], q->c, q->a, q->nu, q->g,
                             (double*)(pc + L.factors), (double*)(pc + L.sigma), (int32_t*)(pc + L.status),
                             (double*)c->ws, wsd));
    kp_batch b{E, q->dim, q->n, nullptr, nullptr, nullptr};
    if ((st = finish_tables(c, &b, 2, pc, L)) != KP_OK) return st;
    return copy_status(c, &b, pc, L, elem_status);
}

kp_status kp_setup_from_factors(kp_ctx c, const kp_batch* b, int32_t rank, const double* factors,
                                void* precond, int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !factors) return KP_ERR_ARG;
    char* pc = (char*)precond;
    const size_t nn = (size_t)b->n * b->n;
    KP_HIP(hipMemcpyAsync(pc + L.factors, factors, E * L.nf * nn * sizeof(double),
                          hipMemcpyDeviceToDevice, c->stream));
    KP_HIP(hipMemsetAsync(pc + L.sigma, 0, E * 4 * sizeof(double), c->stream));
    KP_HIP(hipMemsetAsync(pc + L.status, 0, E * sizeof(int32_t), c->stream));
    KP_HIP(launch_fill_i8(c->stream, E, (int8_t*)(pc + L.axis), 0));
    if ((st = finish_tables(c, b, rank, pc, L)) != KP_OK) return st;
    return copy_status(c, b, pc, L, elem_status);
}

kp_status kp_get_factors(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond,
                         double* factors, double* sigma) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond) return KP_ERR_ARG;
    const char* pc = (const char*)precond;
    const size_t nn = (size_t)b->n * b->n;
    if (factors)
        KP_HIP(hipMemcpyAsync(factors, pc + L.factors, E * L.nf * nn * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    if (sigma)
        KP_HIP(hipMemcpyAsync(sigma, pc + L.sigma, E * 4 * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_get_axes(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond, int8_t* axes) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !axes) return KP_ERR_ARG;
    KP_HIP(hipMemcpyAsync(axes, (const char*)precond + L.axis, E, hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

}  // extern "C"

// z = P^{-1} r, z FP64 (Z = double) or FP32 (Z = float; rank 2, prec not FP64)
template <class Z>
static kp_status apply_impl(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond, int32_t prec,
                            int32_t nrhs, const double* r, Z* z) {
    constexpr bool z32 = sizeof(Z) == 4;
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    if (prec < KP_FP64 || prec > KP_BF16X3 || nrhs < 1) return KP_ERR_ARG;
    if (z32 && (prec == KP_FP64 || rank != 2)) return KP_ERR_UNSUPPORTED;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !r || !z) return KP_ERR_ARG;
    const char* pc = (const char*)precond;
    const void* tabs = prec == KP_FP64   ? (const void*)(pc + L.t64)
                       : prec == KP_FP32 ? (const void*)(pc + L.t32)
                       : prec == KP_BF16 ? (const void*)(pc + L.thi)
                                         : (const void*)(pc + L.t2);
    // the elements' split axes are read under KP_OPT_SPLIT_AXIS (3D)
    const int8_t* axes = (c->split_axis && b->dim == 3) ? (const int8_t*)(pc + L.axis) : nullptr;
    if (rank == 3) {
        // 2D only (pc_layout rejects rank 3 in 3D); FP64 z only (checked above)
        if constexpr (!z32) {
            const double* fac = (const double*)(pc + L.factors);
            const int8_t* kd = (const int8_t*)(pc + L.kinds);
            if (b->n == 16 && c->use_mfma16) {
                // the Neumann series on the matrix cores, then the per-element
                // GMRES for the elements it flags
                if ((st = ensure_ws(c, (size_t)E, &c->ws, &c->ws_bytes)) != KP_OK) return st;
                int8_t* flags = (int8_t*)c->ws;
                KP_HIP(launch_fill_i8(c->stream, E, flags, 0));
                KP_HIP(launch_apply16_rank3(c->stream, prec, E, nrhs, tabs, L.ne, kd, fac, r, z, flags));
                KP_HIP(launch_apply_rank3(c->stream, prec, E, b->n, nrhs, fac, tabs, L.ne, kd, r, z, flags));
            } else {
                KP_HIP(launch_apply_rank3(c->stream, prec, E, b->n, nrhs, fac, tabs, L.ne, kd, r, z));
            }
        }
    } else if (b->n == 16 && c->use_mfma16) {
        KP_HIP(launch_apply16(c->stream, prec, E, b->dim, nrhs, tabs, L.ne, (const int8_t*)(pc + L.kinds), r, z,
                              axes));
    } else if (b->dim == 3 && b->n <= 8 && c->use_small3) {
        KP_HIP(launch_apply_small3(c->stream, prec, E, b->n, nrhs, tabs, L.ne, (const int8_t*)(pc + L.kinds), r, z,
                                   axes));
    } else {
        KP_HIP(launch_apply_generic(c->stream, prec, E, b->dim, b->n, nrhs, tabs, L.ne,
                                    (const int8_t*)(pc + L.kinds), r, z, axes));
    }
    return KP_OK;
}

extern "C" {

kp_status kp_apply(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond, int32_t prec,
                   int32_t nrhs, const double* r, double* z) {
    return apply_impl(c, b, rank, precond, prec, nrhs, r, z);
}

kp_status kp_apply_z32(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond, int32_t prec,
                       int32_t nrhs, const double* r, float* z) {
    return apply_impl(c, b, rank, precond, prec, nrhs, r, z);
}

kp_status kp_blockjacobi_exact(kp_ctx c, const kp_batch* b, double* lu, int32_t* piv,
                               int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    const int N = b->dim == 2 ? b->n * b->n : b->n * b->n * b->n;
    if (!b->blocks || !lu || !piv) return KP_ERR_ARG;
    if (N > 4096) return KP_ERR_UNSUPPORTED;
    int32_t* status = elem_status;
    if (!status) {
        if ((st = ensure_ws(c, E * sizeof(int32_t), &c->ws, &c->ws_bytes)) != KP_OK) return st;
        status = (int32_t*)c->ws;
    }
    KP_HIP(launch_bj_factor(c->stream, E, N, b->blocks, lu, piv, status));
    return KP_OK;
}

kp_status kp_blockjacobi_solve(kp_ctx c, const kp_batch* b, const double* lu, const int32_t* piv,
                               int32_t nrhs, const double* r, double* z) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    const int N = b->dim == 2 ? b->n * b->n : b->n * b->n * b->n;
    if (!lu || !piv || !r || !z || nrhs < 1) return KP_ERR_ARG;
    if (N > 4096) return KP_ERR_UNSUPPORTED;
    KP_HIP(launch_bj_solve(c->stream, E, N, nrhs, lu, piv, r, z));
    return KP_OK;
}

kp_status kp_operator_apply(kp_ctx c, const kp_batch* b, const double* x, double* y) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!x || !y || x == y) return KP_ERR_ARG;
    const int nd = b->dim == 2 ? b->n * b->n : b->n * b->n * b->n;
    if (nd > 4096) return KP_ERR_UNSUPPORTED;
    const Tables1D* T;
    if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
    if (!b->blocks && b->dim == 3 && b->n <= 16 && c->op_cols) {
        // the column kernel reads the element structure: form it first
        const size_t per = (size_t)nd + 3 * (size_t)b->n * b->n;
        if ((st = ensure_ws(c, per * E * sizeof(double), &c->strc, &c->strc_bytes)) != KP_OK) return st;
        KP_HIP(launch_structure(c->stream, E, b->dim, b->n, T, b->params, (double*)c->strc));
        KP_HIP(launch_operator(c->stream, E, b->dim, b->n, T, b->params, b->nbr, b->blocks,
                               (const double*)c->strc, x, y, true));
        return KP_OK;
    }
    KP_HIP(launch_operator(c->stream, E, b->dim, b->n, T, b->params, b->nbr, b->blocks, nullptr, x, y));
    return KP_OK;
}

// the operator with its element structure formed once (into c->strc) and
// read by every application of the solve
}  // extern "C"

// (cached false: formed in every call, as kp_operator_apply does); x FP64 or
// FP32
template <class X>
static kp_status operator_run(kp_ctx c, const kp_batch* b, bool cached, const X* x, double* y) {
    const Tables1D* T;
    kp_status st = get_tables(c, b->n, &T);
    if (st != KP_OK) return st;
    KP_HIP(launch_operator(c->stream, b->num_elems, b->dim, b->n, T, b->params, b->nbr, b->blocks,
                           cached ? (const double*)c->strc : nullptr, x, y, c->op_cols));
    return KP_OK;
}

extern "C" {

// apply the selected preconditioner: z = M v
static kp_status fg_precond(kp_ctx c, const kp_batch* b, int pc_kind, int rank, const void* pc_data,
                            const void* pc_aux, int pc_prec, const double* v, double* z, int64_t N) {
    if (pc_kind == KP_PC_KSVD) return kp_apply(c, b, rank, pc_data, pc_prec, 1, v, z);
    if (pc_kind == KP_PC_BJ)
        return kp_blockjacobi_solve(c, b, (const double*)pc_data, (const int32_t*)pc_aux, 1, v, z);
    KP_HIP(launch_axpby(c->stream, z, v, 1.0, nullptr, 0.0, N));
    return KP_OK;
}

}  // extern "C"

// FGMRES(restart) from x = 0 on N unknowns with the operator op and the
// preconditioner pc (each maps a device vector to another); the driver of
// kp_fgmres and kp_mixed_fgmres.
kp_status fgmres_core(kp_ctx c, int64_t N, const VecFn& op, const VecFn& pc, const double* rhs, double* x,
                      int32_t restart, double rtol, int32_t maxit, int32_t* iters_h, double* relres_h,
                      double* hist_h, int32_t hist_len, const Z32Fns* z32) {
    kp_status st;
    const int m = restart;
    if (iters_h) *iters_h = 0;
    if (relres_h) *relres_h = 0.0;
    if (N == 0) return KP_OK;
    // workspace: V (m+1) N, Z m N (FP64, or FP32 with z32), w N, r N,
    // partial, h (2 (m+2)), y (m), and per step of a cycle its projection
    // slots (2 (m+2) each, used by the cycle graph)
    const size_t vec = (size_t)N + (N & 1);  // vector stride: even, so every vector is 16-byte aligned
    const size_t part = (size_t)kVecBlocks * (m + 2);
    const size_t zd = z32 ? ((size_t)m * vec + 1) / 2 : (size_t)m * vec;  // Z in doubles
    const size_t pslot = 2 * (size_t)(m + 2);
    const size_t need = ((m + 3) * vec + zd + part + 3 * (size_t)(m + 2) + (size_t)m * pslot) * sizeof(double);
    if ((st = ensure_ws(c, need, &c->ks, &c->ks_bytes)) != KP_OK) return st;
    double* V = (double*)c->ks;
    double* Z = V + (m + 1) * vec;
    float* Z32 = (float*)Z;
    double* w = Z + zd;
    double* r = w + vec;
    double* partial = r + vec;
    double* hd = partial + part;   // m + 2
    double* h2 = hd + (m + 2);     // m + 2
    double* yd = h2 + (m + 2);     // m + 2
    double* proj = yd + (m + 2);   // m slots of 2 (m + 2)
    hipStream_t s = c->stream;
    // host Hessenberg and Givens state
    double H[201 * 200], cs[200], sn[200], g[201], hh_local[202];
    double* hh = hh_local;
    // graph mode: a whole restart cycle (m Arnoldi steps: preconditioner,
    // operator, both Gram-Schmidt passes, the norm, the normalisation of the
    // next basis vector on the device, each step's projections in its own
    // slot, then one copy of all of them into pinned host memory) is captured
    // once per solve and replayed every cycle; the host then runs the Givens
    // rotations over the cycle's columns exactly as the step-by-step solve
    // does and stops at the same column, so the iterate is the same.  Steps
    // after that column (in the last cycle only) run without effect on it.
    bool graphs = c->use_graphs;
    hipGraphExec_t exec = nullptr;
    if (graphs) {
        const size_t pin = (size_t)m * pslot;
        if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
            graphs = false;
        if (graphs && c->pinned_doubles < pin) {
            if (c->pinned) hipHostFree(c->pinned);
            c->pinned = nullptr;
            c->pinned_doubles = 0;
            if (hipHostMalloc((void**)&c->pinned, pin * sizeof(double)) == hipSuccess)
                c->pinned_doubles = pin;
            else
                graphs = false;
        }
    }
    struct ExecGuard {
        hipGraphExec_t* e;
        ~ExecGuard() {
            if (*e) hipGraphExecDestroy(*e);
        }
    } guard{&exec};
    double nb2 = 0.0;
    KP_HIP(launch_mdot(s, rhs, 0, 1, rhs, N, partial, hd, 0));
    KP_HIP(hipMemcpyAsync(&nb2, hd, sizeof(double), hipMemcpyDeviceToHost, s));
    KP_HIP(hipStreamSynchronize(s));
    const double nb = sqrt(nb2);
    KP_HIP(launch_axpby(s, x, rhs, 0.0, nullptr, 0.0, N));
    if (!(nb > 0.0)) return KP_OK;
    KP_HIP(launch_axpby(s, r, rhs, 1.0, nullptr, 0.0, N));
    double beta = nb;
    int iters = 0;
    bool converged = false;
    // step j's device work on c->stream: z_j = M v_j, w = A z_j, CGS2 (the
    // first pass's projections in pa, the second's and then ||w||^2 in pb)
    auto step = [&](int j, double* pa, double* pb) -> kp_status {
        kp_status s2;
        hipStream_t q = c->stream;
        double* vj = V + j * vec;
        if (z32) {
            float* zj32 = Z32 + j * vec;
            if ((s2 = z32->pc(vj, zj32)) != KP_OK) return s2;
            if ((s2 = z32->op(zj32, w)) != KP_OK) return s2;
        } else {
            double* zj = Z + j * vec;
            if ((s2 = pc(vj, zj)) != KP_OK) return s2;
            if ((s2 = op(zj, w)) != KP_OK) return s2;
        }
        KP_HIP(launch_mdot(q, V, vec, j + 1, w, N, partial, pa, 0));
        KP_HIP(launch_mgs_update(q, V, vec, j + 1, pa, w, N));
        KP_HIP(launch_mdot(q, V, vec, j + 1, w, N, partial, pb, 0));
        KP_HIP(launch_mgs_update(q, V, vec, j + 1, pb, w, N));
        KP_HIP(launch_mdot(q, w, 0, 1, w, N, partial, pb + j + 1, 0));
        return KP_OK;
    };
    // column j from the two passes' projections and the norm: Givens
    // rotations, residual estimate; returns true where the cycle stops
    int k = 0;
    double hn = 0.0;
    auto column = [&](int j, const double* pa, const double* pb) -> bool {
        double* col = H + j * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = pa[i] + pb[i];
        hn = sqrt(fmax(pb[j + 1], 0.0));
        col[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        const double den = hypot(col[j], col[j + 1]);
        cs[j] = den > 0.0 ? col[j] / den : 1.0;
        sn[j] = den > 0.0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++iters;
        k = j + 1;
        if (hist_h && iters <= hist_len) hist_h[iters - 1] = fabs(g[j + 1]) / nb;
        return fabs(g[j + 1]) <= rtol * nb || iters >= maxit || hn == 0.0;
    };
    while (true) {
        KP_HIP(launch_axpby(s, V, r, 1.0 / beta, nullptr, 0.0, N));
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        k = 0;
        if (graphs && !exec) {
            // capture the cycle on the private stream (nothing runs during capture)
            c->stream = c->cap_stream;
            hipGraph_t graph = nullptr;
            bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            kp_status cst = ok ? KP_OK : KP_ERR_HIP;
            for (int j = 0; j < m && cst == KP_OK; ++j) {
                double* pa = proj + j * pslot;
                double* pb = pa + (m + 2);
                cst = step(j, pa, pb);
                if (cst == KP_OK && launch_normalize(c->cap_stream, pb + j + 1, w, V + (j + 1) * vec, N) != hipSuccess)
                    cst = KP_ERR_HIP;
            }
            if (cst == KP_OK && hipMemcpyAsync(c->pinned, proj, (size_t)m * pslot * sizeof(double),
                                               hipMemcpyDeviceToHost, c->cap_stream) != hipSuccess)
                cst = KP_ERR_HIP;
            ok = (hipStreamEndCapture(c->cap_stream, &graph) == hipSuccess) && ok && cst == KP_OK;
            c->stream = s;
            if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                exec = nullptr;
                ok = false;
            }
            if (graph) hipGraphDestroy(graph);
            if (!ok) {
                hipGetLastError();
                graphs = false;  // this solve continues without graphs
            }
        }
        if (graphs) {
            KP_HIP(hipGraphLaunch(exec, s));
            KP_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < m; ++j) {
                const double* pa = c->pinned + j * pslot;
                if (column(j, pa, pa + (m + 2))) break;
            }
        } else {
            for (int j = 0; j < m; ++j) {
                if ((st = step(j, hd, h2)) != KP_OK) return st;
                KP_HIP(hipMemcpyAsync(hh, hd, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                KP_HIP(hipMemcpyAsync(hh + j + 1, h2, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
                KP_HIP(hipStreamSynchronize(s));
                const bool stop = column(j, hh, hh + j + 1);
                if (hn > 0.0 && !stop) {
                    double* vn = V + (j + 1) * vec;
                    KP_HIP(launch_axpby(s, vn, w, 1.0 / hn, nullptr, 0.0, N));
                }
                if (stop) break;
            }
        }
        // y = H(0:k,0:k)^{-1} g, x += Z y
        double y[200];
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < k; ++q) t -= H[q * (m + 1) + i] * y[q];
            const double d = H[i * (m + 1) + i];
            y[i] = d != 0.0 ? t / d : 0.0;
        }
        KP_HIP(hipMemcpyAsync(yd, y, k * sizeof(double), hipMemcpyHostToDevice, s));
        if (z32)
            KP_HIP(launch_combine(s, Z32, vec, k, yd, x, N));
        else
            KP_HIP(launch_combine(s, Z, vec, k, yd, x, N));
        // true residual
        if ((st = op(x, w)) != KP_OK) return st;
        KP_HIP(launch_axpby(s, r, rhs, 1.0, w, -1.0, N));
        double rr = 0.0;
        KP_HIP(launch_mdot(s, r, 0, 1, r, N, partial, hd, 0));
        KP_HIP(hipMemcpyAsync(&rr, hd, sizeof(double), hipMemcpyDeviceToHost, s));
        KP_HIP(hipStreamSynchronize(s));
        beta = sqrt(fmax(rr, 0.0));
        if (beta <= rtol * nb) { converged = true; break; }
        if (iters >= maxit || !(beta > 0.0)) break;
    }
    if (iters_h) *iters_h = iters;
    if (relres_h) *relres_h = beta / nb;
    return converged ? KP_OK : KP_ERR_NOCONV;
}

extern "C" {

kp_status kp_fgmres(kp_ctx c, const kp_batch* b, int32_t pc_kind, int32_t rank, const void* pc_data,
                    const void* pc_aux, int32_t pc_prec, const double* rhs, double* x,
                    int32_t restart, double rtol, int32_t maxit, int32_t* iters_h, double* relres_h,
                    double* hist_h, int32_t hist_len) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    if (!rhs || !x || restart < 1 || restart > 200 || maxit < 1 || !(rtol > 0.0)) return KP_ERR_ARG;
    if (pc_kind < KP_PC_NONE || pc_kind > KP_PC_BJ) return KP_ERR_ARG;
    if (pc_kind != KP_PC_NONE && !pc_data) return KP_ERR_ARG;
    if (pc_kind == KP_PC_BJ && !pc_aux) return KP_ERR_ARG;
    const int nd = b->dim == 2 ? b->n * b->n : b->n * b->n * b->n;
    const int64_t N = b->num_elems * nd;
    VecFn op = [&](const double* in, double* out) { return kp_operator_apply(c, b, in, out); };
    bool cached = false;
    if (!b->blocks && nd <= 4096 && b->num_elems > 0) {
        // matrix-free: form every element's structure once for the solve
        const Tables1D* T;
        if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
        const size_t per = (size_t)nd + 3 * (size_t)b->n * b->n;
        if ((st = ensure_ws(c, per * b->num_elems * sizeof(double), &c->strc, &c->strc_bytes)) != KP_OK)
            return st;
        KP_HIP(launch_structure(c->stream, b->num_elems, b->dim, b->n, T, b->params, (double*)c->strc));
        cached = true;
        op = [&](const double* in, double* out) { return operator_run(c, b, true, in, out); };
    }
    VecFn pc = [&](const double* in, double* out) {
        return fg_precond(c, b, pc_kind, rank, pc_data, pc_aux, pc_prec, in, out, N);
    };
    // the rank-2 apply in FP32, BF16 or split BF16 ends in FP32 arithmetic:
    // its outputs are FP32 numbers, so the basis Z holds them in FP32 (the
    // same values, half the bytes)
    Z32Fns z32{[&](const double* in, float* out) { return kp_apply_z32(c, b, rank, pc_data, pc_prec, 1, in, out); },
               [&](const float* in, double* out) { return operator_run(c, b, cached, in, out); }};
    const bool use_z32 = c->fgmres_z32 && pc_kind == KP_PC_KSVD && rank == 2 && pc_prec != KP_FP64 &&
                         nd <= 4096;
    return fgmres_core(c, N, op, pc, rhs, x, restart, rtol, maxit, iters_h, relres_h, hist_h, hist_len,
                       use_z32 ? &z32 : nullptr);
}

}  // extern "C"

// C ABI of the KSVD preconditioner library (include/kp.h).
//
// Argument checking, workspace management, precondioner-buffer layout and
// kernel dispatch.  No numerical work happens on the host.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "../../include/kp.h"
#include "kernels.h"
#include "layout.h"
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
};

#define KP_HIP(call)                                   \
    do {                                               \
        hipError_t err_ = (call);                      \
        if (err_ != hipSuccess) return KP_ERR_HIP;     \
    } while (0)

static kp_status ensure_ws(kp_ctx c, size_t bytes, void** slot, size_t* cap) {
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

static kp_status get_tables(kp_ctx c, int n, const Tables1D** out) {
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

static kp_status check_batch(const kp_batch* b, bool need_params = true) {
    if (!b) return KP_ERR_ARG;
    if (b->num_elems < 0) return KP_ERR_ARG;
    if (b->dim != 2 && b->dim != 3) return KP_ERR_ARG;
    if (b->n < 2 || b->n > kMaxN) return KP_ERR_ARG;
    if (need_params && !b->params && b->num_elems > 0) return KP_ERR_ARG;
    return KP_OK;
}

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
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    *ctx = c;
    return KP_OK;
}

kp_status kp_destroy(kp_ctx c) {
    if (!c) return KP_ERR_ARG;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (int n = 0; n <= kMaxN; ++n)
        if (c->d_tables[n]) hipFree(c->d_tables[n]);
    if (c->ws) hipFree(c->ws);
    if (c->ks) hipFree(c->ks);
    delete c;
    return KP_OK;
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
    // global work slots for large n (the table kernel keeps its work in LDS otherwise);
    // the setup workspace is no longer in use once the table kernel runs
    kp_status st = ensure_ws(c, form_tables_gwork_doubles(b->n) * sizeof(double), &c->ws, &c->ws_bytes);
    if (st != KP_OK) return st;
    KP_HIP(launch_form_tables(c->stream, E, b->dim, b->n, rank, (const double*)(pc + L.factors),
                              (double*)(pc + L.t64), (int8_t*)(pc + L.kinds),
                              (int32_t*)(pc + L.status), (double*)c->ws));
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
    if (mode != KP_SETUP_SVD) return KP_ERR_UNSUPPORTED;
    if (b->dim == 3 && b->blocks && b->n * b->n > 64) return KP_ERR_UNSUPPORTED;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    const Tables1D* T;
    if ((st = get_tables(c, b->n, &T)) != KP_OK) return st;
    hipSetDevice(c->device);
    const bool expl = b->blocks != nullptr;
    const int64_t wsd = setup_work_doubles(b->dim, b->n, expl);
    int grid = (int)(E < 2048 ? E : 2048);
    if ((st = ensure_ws(c, (size_t)wsd * grid * sizeof(double), &c->ws, &c->ws_bytes)) != KP_OK)
        return st;
    char* pc = (char*)precond;
    KP_HIP(launch_setup(c->stream, grid, E, b->dim, b->n, rank, T, b->params, b->blocks, nullptr,
                        (double*)(pc + L.factors), (double*)(pc + L.sigma),
                        (int32_t*)(pc + L.status), (double*)c->ws, wsd));
    if ((st = finish_tables(c, b, rank, pc, L)) != KP_OK) return st;
    return copy_status(c, b, pc, L, elem_status);
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

kp_status kp_apply(kp_ctx c, const kp_batch* b, int32_t rank, const void* precond, int32_t prec,
                   int32_t nrhs, const double* r, double* z) {
    if (!c) return KP_ERR_ARG;
    kp_status st = check_batch(b, false);
    if (st != KP_OK) return st;
    PcLayout L;
    if (!pc_layout(b->dim, b->n, rank, b->num_elems, &L)) return KP_ERR_ARG;
    if (prec < KP_FP64 || prec > KP_BF16X3 || nrhs < 1) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !r || !z) return KP_ERR_ARG;
    if (rank == 3) return KP_ERR_UNSUPPORTED;
    const char* pc = (const char*)precond;
    const void* tabs = prec == KP_FP64   ? (const void*)(pc + L.t64)
                       : prec == KP_FP32 ? (const void*)(pc + L.t32)
                       : prec == KP_BF16 ? (const void*)(pc + L.thi)
                                         : (const void*)(pc + L.t2);
    KP_HIP(launch_apply_generic(c->stream, prec, E, b->dim, b->n, nrhs, tabs, L.ne,
                                (const int8_t*)(pc + L.kinds), r, z));
    return KP_OK;
}

kp_status kp_blockjacobi_exact(kp_ctx c, const kp_batch* b, double* lu, int32_t* piv,
                               int32_t* elem_status) {
    (void)c; (void)b; (void)lu; (void)piv; (void)elem_status;
    return KP_ERR_UNSUPPORTED;
}

kp_status kp_blockjacobi_solve(kp_ctx c, const kp_batch* b, const double* lu, const int32_t* piv,
                               int32_t nrhs, const double* r, double* z) {
    (void)c; (void)b; (void)lu; (void)piv; (void)nrhs; (void)r; (void)z;
    return KP_ERR_UNSUPPORTED;
}

kp_status kp_operator_apply(kp_ctx c, const kp_batch* b, const double* x, double* y) {
    (void)c; (void)b; (void)x; (void)y;
    return KP_ERR_UNSUPPORTED;
}

kp_status kp_fgmres(kp_ctx c, const kp_batch* b, int32_t pc_kind, int32_t rank, const void* pc_data,
                    int32_t pc_prec, const double* rhs, double* x, int32_t restart, double rtol,
                    int32_t maxit, int32_t* iters_h, double* relres_h, double* hist_h,
                    int32_t hist_len) {
    (void)c; (void)b; (void)pc_kind; (void)rank; (void)pc_data; (void)pc_prec; (void)rhs; (void)x;
    (void)restart; (void)rtol; (void)maxit; (void)iters_h; (void)relres_h; (void)hist_h;
    (void)hist_len;
    return KP_ERR_UNSUPPORTED;
}

}  // extern "C"

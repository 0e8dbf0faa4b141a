// C ABI of the systems blocks (include/kp.h: kp_sys_*): argument checks,
// workspace, buffer layout (sys.h) and kernel dispatch.
#include <hip/hip_runtime.h>

#include "../../include/kp.h"
#include "kernels.h"
#include "krylov.h"
#include "sys.h"
#include "ctx_internal.h"

using namespace kp;

static kp_status check_sys(const kp_sys_batch* b, SysLayout* L) {
    if (!b || b->num_elems < 0) return KP_ERR_ARG;
    if (!sys_layout(b->nc, b->n, b->num_elems, L)) return KP_ERR_ARG;
    return KP_OK;
}

size_t kp_sys_precond_bytes(int32_t nc, int32_t n, int64_t num_elems) {
    SysLayout L;
    if (num_elems < 0 || !sys_layout(nc, n, num_elems, &L)) return 0;
    return L.total;
}

kp_status kp_setup_sys(kp_ctx c, const kp_sys_batch* b, void* precond, int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !b->blocks) return KP_ERR_ARG;
    hipSetDevice(c->device);
    const int m = b->nc * b->n;
    const int64_t wsd = (sys_work_doubles(m, b->n) + 31) / 32 * 32;
    const int grid = (int)(E < 2048 ? E : 2048);
    if ((st = ensure_ws(c, (size_t)wsd * grid * sizeof(double) + (size_t)E * sizeof(int32_t), &c->ws,
                        &c->ws_bytes)) != KP_OK)
        return st;
    char* pc = (char*)precond;
    KP_HIP(launch_setup_sys(c->stream, grid, E, b->nc, b->n, b->blocks, pc, (double*)c->ws, wsd,
                            (int32_t*)((double*)c->ws + (size_t)wsd * grid)));
    if (elem_status)
        KP_HIP(hipMemcpyAsync(elem_status, pc + L.status, E * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              c->stream));
    return KP_OK;
}

kp_status kp_apply_sys(kp_ctx c, const kp_sys_batch* b, const void* precond, int32_t prec, int32_t nrhs,
                       const double* r, double* z) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    if (nrhs < 1) return KP_ERR_ARG;
    if (prec != KP_FP64 && prec != KP_FP32) return KP_ERR_UNSUPPORTED;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond || !r || !z) return KP_ERR_ARG;
    if (E * (int64_t)nrhs > 0x7fffffff) return KP_ERR_ARG;
    hipSetDevice(c->device);
    KP_HIP(launch_apply_sys(c->stream, E, b->nc, b->n, prec == KP_FP64 ? 0 : 1, nrhs, (const char*)precond, r,
                            z));
    return KP_OK;
}

kp_status kp_get_factors_sys(kp_ctx c, const kp_sys_batch* b, const void* precond, double* factors,
                             double* sigma) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!precond) return KP_ERR_ARG;
    const char* pc = (const char*)precond;
    if (factors)
        KP_HIP(hipMemcpyAsync(factors, pc + L.factors, E * L.nf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    if (sigma)
        KP_HIP(hipMemcpyAsync(sigma, pc + L.sigma, E * 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_build_sys_blocks(kp_ctx c, int64_t num_elems, int32_t nc, int32_t n, const double* recs,
                              double* blocks) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    if (num_elems < 0 || !sys_layout(nc, n, num_elems, &L)) return KP_ERR_ARG;
    if (num_elems == 0) return KP_OK;
    if (!recs || !blocks) return KP_ERR_ARG;
    hipSetDevice(c->device);
    const Tables1D* T;
    kp_status st = get_tables(c, n, &T);
    if (st != KP_OK) return st;
    KP_HIP(launch_build_sys_blocks(c->stream, num_elems, nc, n, T, recs, blocks));
    return KP_OK;
}

kp_status kp_sys_operator_apply(kp_ctx c, const kp_sys_batch* b, const double* x, double* y) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    if (b->num_elems == 0) return KP_OK;
    if (!b->blocks || !x || !y) return KP_ERR_ARG;
    hipSetDevice(c->device);
    KP_HIP(launch_sys_operator(c->stream, b->num_elems, b->nc * b->n * b->n, b->blocks, x, y));
    return KP_OK;
}

kp_status kp_sys_blockjacobi_exact(kp_ctx c, const kp_sys_batch* b, double* lu, int32_t* piv,
                                   int32_t* elem_status) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!b->blocks || !lu || !piv) return KP_ERR_ARG;
    hipSetDevice(c->device);
    int32_t* status = elem_status;
    if (!status) {
        if ((st = ensure_ws(c, E * sizeof(int32_t), &c->ws, &c->ws_bytes)) != KP_OK) return st;
        status = (int32_t*)c->ws;
    }
    KP_HIP(launch_bj_factor(c->stream, E, b->nc * b->n * b->n, b->blocks, lu, piv, status));
    return KP_OK;
}

kp_status kp_fgmres_sys(kp_ctx c, const kp_sys_batch* b, int32_t pc_kind, const void* pc_data, const void* pc_aux,
                        int32_t pc_prec, const double* rhs, double* x, int32_t restart, double rtol, int32_t maxit,
                        int32_t* iters_h, double* relres_h) {
    if (!c) return KP_ERR_ARG;
    SysLayout L;
    kp_status st = check_sys(b, &L);
    if (st != KP_OK) return st;
    if (!rhs || !x || restart < 1 || restart > 200 || maxit < 1 || !(rtol > 0.0)) return KP_ERR_ARG;
    if (pc_kind < KP_PC_NONE || pc_kind > KP_PC_BJ) return KP_ERR_ARG;
    if (pc_kind != KP_PC_NONE && !pc_data) return KP_ERR_ARG;
    if (pc_kind == KP_PC_BJ && !pc_aux) return KP_ERR_ARG;
    if (pc_kind == KP_PC_KSVD && pc_prec != KP_FP64 && pc_prec != KP_FP32) return KP_ERR_UNSUPPORTED;
    if (b->num_elems > 0 && !b->blocks) return KP_ERR_ARG;
    hipSetDevice(c->device);
    const int nd = b->nc * b->n * b->n;
    const int64_t N = b->num_elems * nd;
    VecFn op = [&](const double* in, double* out) { return kp_sys_operator_apply(c, b, in, out); };
    VecFn pc = [&](const double* in, double* out) -> kp_status {
        if (pc_kind == KP_PC_KSVD) return kp_apply_sys(c, b, pc_data, pc_prec, 1, in, out);
        if (pc_kind == KP_PC_BJ) {
            KP_HIP(launch_bj_solve(c->stream, b->num_elems, nd, 1, (const double*)pc_data, (const int32_t*)pc_aux,
                                   in, out));
            return KP_OK;
        }
        KP_HIP(launch_axpby(c->stream, out, in, 1.0, nullptr, 0.0, N));
        return KP_OK;
    };
    return fgmres_core(c, N, op, pc, rhs, x, restart, rtol, maxit, iters_h, relres_h, nullptr, 0, nullptr);
}

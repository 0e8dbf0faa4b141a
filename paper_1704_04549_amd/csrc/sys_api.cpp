// C ABI of the systems blocks (include/kp.h: kp_sys_*): argument checks,
// workspace, buffer layout (sys.h) and kernel dispatch.
#include <hip/hip_runtime.h>

#include "../../include/kp.h"
#include "kernels.h"
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
    if ((st = ensure_ws(c, (size_t)wsd * grid * sizeof(double), &c->ws, &c->ws_bytes)) != KP_OK) return st;
    char* pc = (char*)precond;
    KP_HIP(launch_setup_sys(c->stream, grid, E, b->nc, b->n, b->blocks, pc, (double*)c->ws, wsd));
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

// C ABI of mixed batches (include/kp.h, "mixed batches"): the plan (layout of
// the packed vectors and preconditioner, per-element descriptors, the apply
// work list), setup, apply, the block-diagonal operator, FGMRES and the
// autotuner that chooses, per (dim, n), whether an element is applied by a
// whole workgroup or by one wave.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <utility>
#include <vector>

#include "../../include/kp.h"
#include "ctx_internal.h"
#include "kernels.h"
#include "krylov.h"
#include "mixed.h"

using namespace kp;

struct kp_mixed_plan_s {
    int device = 0;
    int64_t E = 0;
    int64_t vec_len = 0;
    std::vector<MixedElem> h_el;
    MixedElem* d_el = nullptr;
    int32_t* d_order = nullptr;        // setup order: most expensive first
    Tables1D** d_tabs = nullptr;       // [kMaxN + 1] device table pointers
    // preconditioner layout (bytes)
    size_t sigma = 0, factors = 0, status = 0, kinds = 0, t64 = 0, t32 = 0, thi = 0, tlo = 0, t2 = 0, total = 0;
    int64_t fac_total = 0, tab_total = 0;
    int max_n = 2, max_nd = 4;
    int64_t ws_stride = 0;
    // setup: order[0, n_setup_block) one workgroup per element (LDS part of
    // small_doubles), the rest one wave per element (LDS part small_wave each)
    size_t small_doubles = 0, small_wave = 0;
    int64_t n_setup_block = 0;
    // elements grouped by (dim, n) class for the table kernels
    struct Class {
        int dim, n;
        int64_t start, count;
    };
    std::vector<Class> classes;
    int32_t* d_cls = nullptr;
    // side streams (default priority) over which the classes' table kernels
    // run concurrently, and the events that fork them from and join them back
    // to the context's stream; created at the first setup
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    bool side_ready = false;
    // apply work list and its launch shape
    std::map<std::pair<int, int>, int> mode;  // (dim, n) -> 0 workgroup, 1 wave
    int32_t* d_items = nullptr;
    int n_items = 0, n_block = 0;
    long block_nd = 0, wave_nd = 0;  // largest element tensor of each kind
    long block_h = 0, wave_h = 0;    // largest sweep block buffer of each kind
    bool tuned = false;
};

namespace {

#define MX_HIP(call)                                   \
    do {                                               \
        hipError_t err_ = (call);                      \
        if (err_ != hipSuccess) return KP_ERR_HIP;     \
    } while (0)

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

long elem_nd(const MixedElem& d) { return d.dim == 2 ? (long)d.n * d.n : (long)d.n * d.n * d.n; }

// work list from the current per-(dim, n) modes: workgroup items first
kp_status build_items(kp_mixed_plan p) {
    std::vector<int32_t> blk, wav;
    p->block_nd = 0;
    p->wave_nd = 0;
    p->block_h = 0;
    p->wave_h = 0;
    for (int64_t e = 0; e < p->E; ++e) {
        const MixedElem& d = p->h_el[e];
        const int md = p->mode[{d.dim, d.n}];
        if (md == 0) {
            blk.push_back((int32_t)e);
            p->block_nd = std::max(p->block_nd, elem_nd(d));
            p->block_h = std::max(p->block_h, mixed_apply_h(d.dim, d.n));
        } else {
            wav.push_back((int32_t)e);
            p->wave_nd = std::max(p->wave_nd, elem_nd(d));
            p->wave_h = std::max(p->wave_h, mixed_apply_h(d.dim, d.n));
        }
    }
    // longest first within each kind, for the tail of the persistent grid
    auto cost = [&](int32_t a, int32_t b) { return elem_nd(p->h_el[a]) > elem_nd(p->h_el[b]); };
    std::stable_sort(blk.begin(), blk.end(), cost);
    std::stable_sort(wav.begin(), wav.end(), cost);
    const int nw = (int)((wav.size() + kMixedItemWidth - 1) / kMixedItemWidth);
    std::vector<int32_t> items((blk.size() + nw) * kMixedItemWidth, -1);
    for (size_t i = 0; i < blk.size(); ++i) items[i * kMixedItemWidth] = blk[i];
    for (size_t i = 0; i < wav.size(); ++i) items[(blk.size() + i / kMixedItemWidth) * kMixedItemWidth + i % kMixedItemWidth] = wav[i];
    if (p->d_items) hipFree(p->d_items);
    p->d_items = nullptr;
    if (!items.empty()) {
        if (hipMalloc((void**)&p->d_items, items.size() * sizeof(int32_t)) != hipSuccess) return KP_ERR_ALLOC;
        MX_HIP(hipMemcpy(p->d_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    p->n_block = (int)blk.size();
    p->n_items = (int)blk.size() + nw;
    return KP_OK;
}

const void* table_section(kp_mixed_plan p, const char* pc, int prec) {
    return prec == KP_FP64 ? (const void*)(pc + p->t64)
           : prec == KP_FP32 ? (const void*)(pc + p->t32)
           : prec == KP_BF16 ? (const void*)(pc + p->thi)
                             : (const void*)(pc + p->t2);
}

kp_status mixed_apply_launch(kp_ctx c, kp_mixed_plan p, const void* precond, int prec, const double* r, double* z) {
    const char* pc = (const char*)precond;
    const int grid = p->n_items < 65536 ? p->n_items : 65536;
    MX_HIP(launch_mixed_apply(c->stream, prec, grid, p->n_items, p->n_block, p->d_items, p->d_el,
                              table_section(p, pc, prec), (const int8_t*)(pc + p->kinds), r, z, p->block_nd,
                              p->block_h, p->wave_nd, p->wave_h));
    return KP_OK;
}

}  // namespace

extern "C" {

kp_status kp_mixed_plan_create(kp_ctx c, int64_t num_elems, const int32_t* dim_n_h, kp_mixed_plan* out) {
    if (!c || !out || num_elems < 0 || (num_elems > 0 && !dim_n_h)) return KP_ERR_ARG;
    *out = nullptr;
    kp_mixed_plan p = new (std::nothrow) kp_mixed_plan_s;
    if (!p) return KP_ERR_ALLOC;
    p->device = c->device;
    p->E = num_elems;
    p->h_el.resize(num_elems);
    int64_t vo = 0, fo = 0, to = 0;
    long wsd = 0;
    size_t smd = 0;
    bool present[kMaxN + 1] = {};
    for (int64_t e = 0; e < num_elems; ++e) {
        const int dim = dim_n_h[2 * e], n = dim_n_h[2 * e + 1];
        if ((dim != 2 && dim != 3) || n < 2 || n > kMaxN) {
            delete p;
            return KP_ERR_ARG;
        }
        MixedElem& d = p->h_el[e];
        d.dim = dim;
        d.n = n;
        d.vec_off = vo;
        d.fac_off = fo;
        d.tab_off = to;
        vo += elem_nd(d);
        fo += (int64_t)(dim == 2 ? 4 : 5) * n * n;
        to += tab_entries(n);
        p->max_n = std::max(p->max_n, n);
        p->max_nd = (int)std::max<long>(p->max_nd, elem_nd(d));
        wsd = std::max(wsd, setup_work_doubles(dim, n, false, 2));
        present[n] = true;
        p->mode[{dim, n}] = 0;
    }
    p->vec_len = vo;
    p->fac_total = fo;
    p->tab_total = to;
    p->ws_stride = wsd;
    // a class is set up one wave per element when four waves' LDS parts fit
    auto wave_setup = [](int n) {
        const size_t sm = (setup_small_doubles(n, false) + 31) / 32 * 32;
        return 4 * sm * sizeof(double) <= kSetupWavesLdsMax;
    };
    size_t smw = 0;
    for (int64_t e = 0; e < num_elems; ++e) {
        const int n = p->h_el[e].n;
        const size_t sm = setup_small_doubles(n, false);
        if (wave_setup(n))
            smw = std::max(smw, (sm + 31) / 32 * 32);
        else
            smd = std::max(smd, sm);
    }
    p->small_doubles = smd;
    p->small_wave = smw;
    size_t off = 0;
    p->sigma = off; off = al256(off + num_elems * 4 * sizeof(double));
    p->factors = off; off = al256(off + fo * sizeof(double));
    p->status = off; off = al256(off + num_elems * sizeof(int32_t));
    p->kinds = off; off = al256(off + num_elems * kMaxN);
    p->t64 = off; off = al256(off + to * sizeof(double));
    p->t32 = off; off = al256(off + to * sizeof(float));
    p->thi = off; off = al256(off + to * sizeof(uint16_t));
    p->tlo = off; off = al256(off + to * sizeof(uint16_t));
    p->t2 = off; off = al256(off + to * sizeof(float));
    p->total = off;
    hipSetDevice(c->device);
    // descriptors, setup order, table pointers
    std::vector<int32_t> order(num_elems);
    for (int64_t e = 0; e < num_elems; ++e) order[e] = (int32_t)e;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const MixedElem &x = p->h_el[a], &y = p->h_el[b];
        const bool wx = wave_setup(x.n), wy = wave_setup(y.n);
        if (wx != wy) return wy;  // workgroup-mode elements first
        if (elem_nd(x) != elem_nd(y)) return elem_nd(x) > elem_nd(y);
        return x.n > y.n;
    });
    for (int64_t e = 0; e < num_elems; ++e)
        if (!wave_setup(p->h_el[e].n)) ++p->n_setup_block;
    Tables1D* tabs[kMaxN + 1] = {};
    for (int n = 2; n <= kMaxN; ++n)
        if (present[n]) {
            const Tables1D* t;
            kp_status st = get_tables(c, n, &t);
            if (st != KP_OK) {
                kp_mixed_plan_destroy(p);
                return st;
            }
            tabs[n] = (Tables1D*)t;
        }
    std::vector<int32_t> cls(num_elems);
    for (int64_t e = 0; e < num_elems; ++e) cls[e] = (int32_t)e;
    std::stable_sort(cls.begin(), cls.end(), [&](int32_t a, int32_t b) {
        const MixedElem &x = p->h_el[a], &y = p->h_el[b];
        return x.dim != y.dim ? x.dim < y.dim : x.n < y.n;
    });
    for (int64_t i = 0; i < num_elems; ++i) {
        const MixedElem& d = p->h_el[cls[i]];
        if (p->classes.empty() || p->classes.back().dim != d.dim || p->classes.back().n != d.n)
            p->classes.push_back({d.dim, d.n, i, 0});
        ++p->classes.back().count;
    }
    if (num_elems > 0) {
        if (hipMalloc((void**)&p->d_el, num_elems * sizeof(MixedElem)) != hipSuccess ||
            hipMalloc((void**)&p->d_order, num_elems * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void**)&p->d_cls, num_elems * sizeof(int32_t)) != hipSuccess) {
            kp_mixed_plan_destroy(p);
            return KP_ERR_ALLOC;
        }
        hipMemcpy(p->d_el, p->h_el.data(), num_elems * sizeof(MixedElem), hipMemcpyHostToDevice);
        hipMemcpy(p->d_order, order.data(), num_elems * sizeof(int32_t), hipMemcpyHostToDevice);
        hipMemcpy(p->d_cls, cls.data(), num_elems * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (hipMalloc((void**)&p->d_tabs, sizeof(tabs)) != hipSuccess) {
        kp_mixed_plan_destroy(p);
        return KP_ERR_ALLOC;
    }
    hipMemcpy(p->d_tabs, tabs, sizeof(tabs), hipMemcpyHostToDevice);
    kp_status st = build_items(p);
    if (st != KP_OK) {
        kp_mixed_plan_destroy(p);
        return st;
    }
    *out = p;
    return KP_OK;
}

kp_status kp_mixed_plan_destroy(kp_mixed_plan p) {
    if (!p) return KP_ERR_ARG;
    hipSetDevice(p->device);
    hipDeviceSynchronize();
    if (p->d_el) hipFree(p->d_el);
    if (p->d_order) hipFree(p->d_order);
    if (p->d_cls) hipFree(p->d_cls);
    if (p->d_tabs) hipFree(p->d_tabs);
    if (p->d_items) hipFree(p->d_items);
    for (int i = 0; i < kp_mixed_plan_s::kSide; ++i) {
        if (p->side[i]) hipStreamDestroy(p->side[i]);
        if (p->join[i]) hipEventDestroy(p->join[i]);
    }
    if (p->fork) hipEventDestroy(p->fork);
    delete p;
    return KP_OK;
}

kp_status kp_mixed_plan_info(kp_mixed_plan p, int64_t* vec_len_h, size_t* precond_bytes_h) {
    if (!p) return KP_ERR_ARG;
    if (vec_len_h) *vec_len_h = p->vec_len;
    if (precond_bytes_h) *precond_bytes_h = p->total;
    return KP_OK;
}

kp_status kp_mixed_setup(kp_ctx c, kp_mixed_plan p, const double* params, void* precond, int32_t* elem_status) {
    if (!c || !p) return KP_ERR_ARG;
    if (p->E == 0) return KP_OK;
    if (!params || !precond) return KP_ERR_ARG;
    hipSetDevice(c->device);
    // the two launches run one after the other on the stream and share the
    // workspace: at most 2048 slots each
    const int64_t eb = p->n_setup_block, ew = p->E - eb;
    const int grid = (int)(eb < 2048 ? eb : 2048);
    const int grid4 = (int)((std::min<int64_t>(ew, 2048) + 3) / 4);
    const int64_t slots = std::max<int64_t>(grid, 4 * (int64_t)grid4);
    kp_status st = ensure_ws(c, (size_t)p->ws_stride * slots * sizeof(double), &c->ws, &c->ws_bytes);
    if (st != KP_OK) return st;
    char* pc = (char*)precond;
    MX_HIP(launch_mixed_setup(c->stream, grid, eb, p->d_el, p->d_order, p->d_tabs, params,
                              (double*)(pc + p->factors), (double*)(pc + p->sigma), (int32_t*)(pc + p->status),
                              (double*)c->ws, p->ws_stride, p->small_doubles));
    MX_HIP(launch_mixed_setup_waves(c->stream, grid4, ew, p->d_el, p->d_order + eb, p->d_tabs, params,
                                    (double*)(pc + p->factors), (double*)(pc + p->sigma),
                                    (int32_t*)(pc + p->status), (double*)c->ws, p->ws_stride,
                                    (int64_t)p->small_wave));
    // the tables one (dim, n) class at a time, each in the launch shape of
    // a uniform batch of that class.  A class fills a fraction of the chip,
    // so the classes are spread over the side streams and run concurrently:
    // they read the factors and write the tables, kinds and status entries
    // of their own elements only.
    if (!p->side_ready) {
        // all or nothing: a failure releases what was created
        bool ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < kp_mixed_plan_s::kSide; ++i)
            ok = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            for (int i = 0; i < kp_mixed_plan_s::kSide; ++i) {
                if (p->side[i]) hipStreamDestroy(p->side[i]);
                if (p->join[i]) hipEventDestroy(p->join[i]);
                p->side[i] = nullptr;
                p->join[i] = nullptr;
            }
            if (p->fork) hipEventDestroy(p->fork);
            p->fork = nullptr;
            return KP_ERR_HIP;
        }
        p->side_ready = true;
    }
    MX_HIP(hipEventRecord(p->fork, c->stream));
    for (int i = 0; i < kp_mixed_plan_s::kSide; ++i) MX_HIP(hipStreamWaitEvent(p->side[i], p->fork, 0));
    // most expensive class first (count n^3), each on the least loaded stream
    std::vector<size_t> by_cost(p->classes.size());
    for (size_t k = 0; k < by_cost.size(); ++k) by_cost[k] = k;
    auto cost = [&](size_t k) {
        const double n = p->classes[k].n;
        return (double)p->classes[k].count * n * n * n;
    };
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](size_t a, size_t b) { return cost(a) > cost(b); });
    double load[kp_mixed_plan_s::kSide] = {};
    for (size_t k : by_cost) {
        const auto& cl = p->classes[k];
        const int i = (int)(std::min_element(load, load + kp_mixed_plan_s::kSide) - load);
        load[i] += cost(k);
        MX_HIP(launch_form_tables_list(p->side[i], cl.count, p->d_cls + cl.start, p->d_el, cl.dim, cl.n,
                                       (const double*)(pc + p->factors), (double*)(pc + p->t64),
                                       (int8_t*)(pc + p->kinds), (int32_t*)(pc + p->status)));
    }
    for (int i = 0; i < kp_mixed_plan_s::kSide; ++i) {
        MX_HIP(hipEventRecord(p->join[i], p->side[i]));
        MX_HIP(hipStreamWaitEvent(c->stream, p->join[i], 0));
    }
    MX_HIP(launch_cast_tables(c->stream, p->tab_total, (const double*)(pc + p->t64), (float*)(pc + p->t32),
                              (uint16_t*)(pc + p->thi), (uint16_t*)(pc + p->tlo), (float*)(pc + p->t2)));
    if (elem_status)
        MX_HIP(hipMemcpyAsync(elem_status, pc + p->status, p->E * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              c->stream));
    return KP_OK;
}

kp_status kp_mixed_get_factors(kp_ctx c, kp_mixed_plan p, const void* precond, double* factors, double* sigma) {
    if (!c || !p || !precond) return KP_ERR_ARG;
    const char* pc = (const char*)precond;
    if (factors)
        MX_HIP(hipMemcpyAsync(factors, pc + p->factors, p->fac_total * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    if (sigma)
        MX_HIP(hipMemcpyAsync(sigma, pc + p->sigma, p->E * 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_mixed_apply(kp_ctx c, kp_mixed_plan p, const void* precond, int32_t prec, const double* r, double* z) {
    if (!c || !p) return KP_ERR_ARG;
    if (prec < KP_FP64 || prec > KP_BF16X3) return KP_ERR_ARG;
    if (p->E == 0) return KP_OK;
    if (!precond || !r || !z) return KP_ERR_ARG;
    return mixed_apply_launch(c, p, precond, prec, r, z);
}

kp_status kp_mixed_autotune(kp_ctx c, kp_mixed_plan p, const void* precond, int32_t prec, const double* r,
                            double* z, int32_t* modes_h, int32_t modes_len) {
    if (!c || !p) return KP_ERR_ARG;
    if (prec < KP_FP64 || prec > KP_BF16X3) return KP_ERR_ARG;
    if (p->E == 0) return KP_OK;
    if (!precond || !r || !z) return KP_ERR_ARG;
    hipEvent_t e0, e1;
    MX_HIP(hipEventCreate(&e0));
    MX_HIP(hipEventCreate(&e1));
    kp_status st = KP_OK;
    // one (dim, n) class at a time: only its elements in the work list, both modes timed
    std::map<std::pair<int, int>, int> chosen;
    for (auto& kv : p->mode) {
        float best_t = 0.f;
        int best_m = 0;
        for (int md = 0; md < 2 && st == KP_OK; ++md) {
            // a work list of this class only
            std::vector<int32_t> items;
            long nd = 0, h = 0;
            std::vector<int32_t> members;
            for (int64_t e = 0; e < p->E; ++e)
                if (p->h_el[e].dim == kv.first.first && p->h_el[e].n == kv.first.second) {
                    members.push_back((int32_t)e);
                    nd = elem_nd(p->h_el[e]);
                    h = mixed_apply_h(p->h_el[e].dim, p->h_el[e].n);
                }
            // the wave mode holds four elements per workgroup: only for classes
            // whose four elements fit at FP64 with three full tensors each, so
            // that the wave part of a launch stays at or below the size of its
            // largest workgroup elements (n <= 40 in 2D, n <= 11 in 3D)
            if (md == 1 && 3 * kMixedItemWidth * nd * (long)sizeof(double) > (long)kMixedApplyLdsMax) break;
            const int width = md == 0 ? 1 : kMixedItemWidth;
            const int nit = (int)((members.size() + width - 1) / width);
            items.assign((size_t)nit * kMixedItemWidth, -1);
            for (size_t i = 0; i < members.size(); ++i)
                items[(i / width) * kMixedItemWidth + i % width] = members[i];
            int32_t* d_items = nullptr;
            if (hipMalloc((void**)&d_items, items.size() * sizeof(int32_t)) != hipSuccess) {
                st = KP_ERR_ALLOC;
                break;
            }
            hipMemcpy(d_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice);
            const char* pc = (const char*)precond;
            const int grid = nit < 65536 ? nit : 65536;
            float tsum = 0.f;
            for (int rep = 0; rep < 4 && st == KP_OK; ++rep) {
                hipEventRecord(e0, c->stream);
                if (launch_mixed_apply(c->stream, prec, grid, nit, md == 0 ? nit : 0, d_items, p->d_el,
                                       table_section(p, pc, prec), (const int8_t*)(pc + p->kinds), r, z,
                                       md == 0 ? nd : 0, md == 0 ? h : 0, md == 0 ? 0 : nd, md == 0 ? 0 : h) !=
                                    hipSuccess)
                    st = KP_ERR_HIP;
                hipEventRecord(e1, c->stream);
                hipEventSynchronize(e1);
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) tsum += ms;  // the first launch warms up
            }
            hipFree(d_items);
            if (md == 0 || tsum < best_t) {
                best_t = tsum;
                best_m = md;
            }
        }
        chosen[kv.first] = best_m;
        if (st != KP_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != KP_OK) {
        for (auto& q : p->mode) q.second = 0;
        build_items(p);
        return st;
    }
    p->mode = chosen;
    if ((st = build_items(p)) != KP_OK) return st;
    p->tuned = true;
    if (modes_h) {
        int i = 0;
        for (auto& kv : p->mode) {
            if (i + 3 > modes_len) break;
            modes_h[i++] = kv.first.first;
            modes_h[i++] = kv.first.second;
            modes_h[i++] = kv.second;
        }
        for (; i < modes_len; ++i) modes_h[i] = -1;
    }
    return KP_OK;
}

kp_status kp_mixed_operator_apply(kp_ctx c, kp_mixed_plan p, const double* params, const double* x, double* y) {
    if (!c || !p) return KP_ERR_ARG;
    if (p->E == 0) return KP_OK;
    if (!params || !x || !y) return KP_ERR_ARG;
    MX_HIP(launch_mixed_operator(c->stream, p->E, p->d_el, p->d_tabs, params, x, y, p->max_n, p->max_nd));
    return KP_OK;
}

kp_status kp_mixed_fgmres(kp_ctx c, kp_mixed_plan p, const double* params, int32_t pc_kind, const void* precond,
                          int32_t pc_prec, const double* rhs, double* x, int32_t restart, double rtol,
                          int32_t maxit, int32_t* iters_h, double* relres_h, double* hist_h, int32_t hist_len) {
    if (!c || !p) return KP_ERR_ARG;
    if (!rhs || !x || restart < 1 || restart > 200 || maxit < 1 || !(rtol > 0.0)) return KP_ERR_ARG;
    if (pc_kind != KP_PC_NONE && pc_kind != KP_PC_KSVD) return KP_ERR_ARG;
    if (pc_kind == KP_PC_KSVD && !precond) return KP_ERR_ARG;
    if (p->E > 0 && !params) return KP_ERR_ARG;
    VecFn op = [&](const double* in, double* out) { return kp_mixed_operator_apply(c, p, params, in, out); };
    VecFn pcf = [&](const double* in, double* out) -> kp_status {
        if (pc_kind == KP_PC_KSVD) return kp_mixed_apply(c, p, precond, pc_prec, in, out);
        MX_HIP(launch_axpby(c->stream, out, in, 1.0, nullptr, 0.0, p->vec_len));
        return KP_OK;
    };
    return fgmres_core(c, p->vec_len, op, pcf, rhs, x, restart, rtol, maxit, iters_h, relres_h, hist_h, hist_len);
}

}  // extern "C"

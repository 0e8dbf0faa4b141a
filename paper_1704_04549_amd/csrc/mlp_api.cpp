// C ABI of the learned setup (include/kp.h, "learned setup"): the model
// buffer, the forward and backward passes and the training driver.  Every
// arithmetic step runs in the kernels of mlp.hip; the host only sequences
// launches, draws the minibatch order and reads one loss per epoch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/kp.h"
#include "ctx_internal.h"
#include "mlp.h"

using namespace kp;

namespace {

#define MLP_HIP(call)                                  \
    do {                                               \
        hipError_t err_ = (call);                      \
        if (err_ != hipSuccess) return KP_ERR_HIP;     \
    } while (0)

kp_status read_header(kp_ctx c, const void* model, int hdr[8], MlpLayout* L) {
    if (!model) return KP_ERR_ARG;
    MLP_HIP(hipMemcpyAsync(hdr, model, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MLP_HIP(hipStreamSynchronize(c->stream));
    if (hdr[0] != kMlpMagic) return KP_ERR_ARG;
    if (!mlp_layout(hdr[4], hdr[5], hdr[2], L)) return KP_ERR_ARG;
    return KP_OK;
}

int gemm_prec(int prec) { return prec == KP_BF16 ? 1 : 0; }

struct Acts {
    float *Z1, *H1, *Z2, *H2, *Y;
};

// y = W3 silu(W2 silu(W1 xn + b1) + b2) + b3 for `rows` rows
kp_status forward(hipStream_t s, int bf, const MlpLayout& L, const float* P, int rows, const float* Xn,
                  const Acts& a) {
    const MlpParams o = mlp_params(L);
    MLP_HIP(launch_gemm(s, bf, rows, L.H, L.I, Xn, L.I, 0, P + o.W1, L.I, 1, a.Z1, L.H, 1.f, 0.f));
    MLP_HIP(launch_bias_silu(s, rows, L.H, a.Z1, P + o.b1, a.H1));
    MLP_HIP(launch_gemm(s, bf, rows, L.H, L.H, a.H1, L.H, 0, P + o.W2, L.H, 1, a.Z2, L.H, 1.f, 0.f));
    MLP_HIP(launch_bias_silu(s, rows, L.H, a.Z2, P + o.b2, a.H2));
    MLP_HIP(launch_gemm(s, bf, rows, L.O, L.H, a.H2, L.H, 0, P + o.W3, L.H, 1, a.Y, L.O, 1.f, 0.f));
    MLP_HIP(launch_bias(s, rows, L.O, a.Y, P + o.b3));
    return KP_OK;
}

// gradient G (param layout) from dY; a.H2 and dH are overwritten
kp_status backward(hipStream_t s, int bf, const MlpLayout& L, const float* P, int rows, const float* Xn,
                   const Acts& a, const float* dY, float* dH, float* G) {
    const MlpParams o = mlp_params(L);
    MLP_HIP(launch_gemm(s, bf, L.O, L.H, rows, dY, L.O, 1, a.H2, L.H, 0, G + o.W3, L.H, 1.f, 0.f));
    MLP_HIP(launch_colsum(s, rows, L.O, dY, G + o.b3));
    MLP_HIP(launch_gemm(s, bf, rows, L.H, L.O, dY, L.O, 0, P + o.W3, L.H, 0, dH, L.H, 1.f, 0.f));
    MLP_HIP(launch_silu_back(s, rows, L.H, dH, a.Z2));
    MLP_HIP(launch_gemm(s, bf, L.H, L.H, rows, dH, L.H, 1, a.H1, L.H, 0, G + o.W2, L.H, 1.f, 0.f));
    MLP_HIP(launch_colsum(s, rows, L.H, dH, G + o.b2));
    float* dH1 = a.H2;  // h2 is not needed any more
    MLP_HIP(launch_gemm(s, bf, rows, L.H, L.H, dH, L.H, 0, P + o.W2, L.H, 0, dH1, L.H, 1.f, 0.f));
    MLP_HIP(launch_silu_back(s, rows, L.H, dH1, a.Z1));
    MLP_HIP(launch_gemm(s, bf, L.H, L.I, rows, dH1, L.H, 1, Xn, L.I, 0, G + o.W1, L.I, 1.f, 0.f));
    MLP_HIP(launch_colsum(s, rows, L.H, dH1, G + o.b1));
    return KP_OK;
}

// carve float arrays out of the context's MLP workspace
struct Carver {
    char* p;
    template <typename T>
    T* take(size_t count) {
        T* r = (T*)p;
        p += mlp_align(count * sizeof(T));
        return r;
    }
};

size_t acts_bytes(const MlpLayout& L, size_t rows) {
    return 4 * mlp_align(rows * L.H * sizeof(float)) + mlp_align(rows * L.O * sizeof(float));
}

Acts take_acts(Carver& cv, const MlpLayout& L, size_t rows) {
    Acts a;
    a.Z1 = cv.take<float>(rows * L.H);
    a.H1 = cv.take<float>(rows * L.H);
    a.Z2 = cv.take<float>(rows * L.H);
    a.H2 = cv.take<float>(rows * L.H);
    a.Y = cv.take<float>(rows * L.O);
    return a;
}

// splitmix64 (Steele, Lea & Flood), used to draw the minibatch order
uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

size_t kp_mlp_bytes(int32_t dim, int32_t n, int32_t hidden) {
    MlpLayout L;
    if (!mlp_layout(dim, n, hidden, &L)) return 0;
    return L.total;
}

kp_status kp_mlp_init(kp_ctx c, void* model, int32_t dim, int32_t n, int32_t hidden, const float* params) {
    if (!c || !model) return KP_ERR_ARG;
    MlpLayout L;
    if (!mlp_layout(dim, n, hidden, &L)) return KP_ERR_ARG;
    int hdr[64] = {};
    hdr[0] = kMlpMagic;
    hdr[1] = L.I;
    hdr[2] = L.H;
    hdr[3] = L.O;
    hdr[4] = dim;
    hdr[5] = n;
    hdr[6] = L.nb;
    hdr[7] = 0;  // optimiser steps taken
    char* m = (char*)model;
    MLP_HIP(hipMemcpyAsync(m, hdr, sizeof(hdr), hipMemcpyHostToDevice, c->stream));
    if (params)
        MLP_HIP(hipMemcpyAsync(m + L.params, params, L.P * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    else
        MLP_HIP(hipMemsetAsync(m + L.params, 0, L.P * sizeof(float), c->stream));
    MLP_HIP(hipMemsetAsync(m + L.m, 0, L.P * sizeof(float), c->stream));
    MLP_HIP(hipMemsetAsync(m + L.v, 0, L.P * sizeof(float), c->stream));
    std::vector<float> zeros(L.I, 0.f), ones(L.I > L.nb ? L.I : L.nb, 1.f);
    MLP_HIP(hipMemcpyAsync(m + L.xmean, zeros.data(), L.I * sizeof(float), hipMemcpyHostToDevice, c->stream));
    MLP_HIP(hipMemcpyAsync(m + L.xstd, ones.data(), L.I * sizeof(float), hipMemcpyHostToDevice, c->stream));
    MLP_HIP(hipMemcpyAsync(m + L.yscale, ones.data(), L.nb * sizeof(float), hipMemcpyHostToDevice, c->stream));
    MLP_HIP(hipStreamSynchronize(c->stream));  // the host arrays go out of scope
    return KP_OK;
}

kp_status kp_mlp_get(kp_ctx c, const void* model, float* params, float* x_mean, float* x_std, float* yscale) {
    if (!c) return KP_ERR_ARG;
    int hdr[8];
    MlpLayout L;
    kp_status st = read_header(c, model, hdr, &L);
    if (st != KP_OK) return st;
    const char* m = (const char*)model;
    if (params) MLP_HIP(hipMemcpyAsync(params, m + L.params, L.P * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (x_mean) MLP_HIP(hipMemcpyAsync(x_mean, m + L.xmean, L.I * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (x_std) MLP_HIP(hipMemcpyAsync(x_std, m + L.xstd, L.I * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (yscale) MLP_HIP(hipMemcpyAsync(yscale, m + L.yscale, L.nb * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_mlp_set_norm(kp_ctx c, void* model, const float* x_mean, const float* x_std, const float* yscale) {
    if (!c) return KP_ERR_ARG;
    int hdr[8];
    MlpLayout L;
    kp_status st = read_header(c, model, hdr, &L);
    if (st != KP_OK) return st;
    char* m = (char*)model;
    if (x_mean) MLP_HIP(hipMemcpyAsync(m + L.xmean, x_mean, L.I * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (x_std) MLP_HIP(hipMemcpyAsync(m + L.xstd, x_std, L.I * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (yscale) MLP_HIP(hipMemcpyAsync(m + L.yscale, yscale, L.nb * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    return KP_OK;
}

kp_status kp_mlp_forward(kp_ctx c, const void* model, int32_t prec, int64_t rows, const float* xn, float* y) {
    if (!c || rows < 0) return KP_ERR_ARG;
    if (prec != KP_FP32 && prec != KP_BF16) return KP_ERR_ARG;
    int hdr[8];
    MlpLayout L;
    kp_status st = read_header(c, model, hdr, &L);
    if (st != KP_OK) return st;
    if (rows == 0) return KP_OK;
    if (!xn || !y || rows > (1 << 24)) return KP_ERR_ARG;
    if ((st = ensure_ws(c, acts_bytes(L, rows) + 1024, &c->mw, &c->mw_bytes)) != KP_OK) return st;
    Carver cv{(char*)c->mw};
    Acts a = take_acts(cv, L, rows);
    a.Y = y;
    const float* P = (const float*)((const char*)model + L.params);
    return forward(c->stream, gemm_prec(prec), L, P, (int)rows, xn, a);
}

kp_status kp_mlp_loss_grad(kp_ctx c, const void* model, int32_t prec, int64_t rows, const float* xn,
                           const float* t, float* grad, float* loss) {
    if (!c || rows <= 0 || !xn || !t || !grad || !loss || rows > (1 << 24)) return KP_ERR_ARG;
    if (prec != KP_FP32 && prec != KP_BF16) return KP_ERR_ARG;
    int hdr[8];
    MlpLayout L;
    kp_status st = read_header(c, model, hdr, &L);
    if (st != KP_OK) return st;
    const size_t need = acts_bytes(L, rows) + 2 * mlp_align(rows * L.O * sizeof(float)) +
                        mlp_align(rows * L.H * sizeof(float)) + mlp_align(rows * sizeof(float)) + 1024;
    if ((st = ensure_ws(c, need, &c->mw, &c->mw_bytes)) != KP_OK) return st;
    Carver cv{(char*)c->mw};
    Acts a = take_acts(cv, L, rows);
    float* dY = cv.take<float>(rows * L.O);
    float* dH = cv.take<float>(rows * L.H);
    float* rl = cv.take<float>(rows);
    const float* P = (const float*)((const char*)model + L.params);
    const int bf = gemm_prec(prec);
    if ((st = forward(c->stream, bf, L, P, (int)rows, xn, a)) != KP_OK) return st;
    MLP_HIP(launch_mlp_loss(c->stream, (int)rows, hdr[4], hdr[5], a.Y, t, dY, rl, 1.f / (float)(rows * L.O)));
    MLP_HIP(launch_sum(c->stream, (int)rows, rl, loss, 0));
    return backward(c->stream, bf, L, P, (int)rows, xn, a, dY, dH, grad);
}

kp_status kp_mlp_train(kp_ctx c, void* model, const kp_batch* b, const double* factors, int32_t epochs,
                       int32_t batch, float lr, uint64_t seed, int32_t prec, float* loss_hist_h) {
    if (!c || !b || !factors || epochs < 0 || batch < 1 || !(lr > 0.f)) return KP_ERR_ARG;
    if (prec != KP_FP32 && prec != KP_BF16) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    int hdr[8];
    MlpLayout L;
    if ((st = read_header(c, model, hdr, &L)) != KP_OK) return st;
    if (hdr[4] != b->dim || hdr[5] != b->n) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E < 1 || E > (1 << 24)) return KP_ERR_ARG;
    const int bs = batch < E ? batch : (int)E;
    const int nn = b->n * b->n;
    const size_t need = 2 * mlp_align(E * L.I * sizeof(float)) + mlp_align(E * L.O * sizeof(float)) +
                        mlp_align(E * sizeof(int32_t)) + mlp_align(bs * L.I * sizeof(float)) +
                        mlp_align(bs * L.O * sizeof(float)) * 2 + acts_bytes(L, bs) +
                        mlp_align(bs * L.H * sizeof(float)) + mlp_align(L.P * sizeof(float)) +
                        mlp_align(bs * sizeof(float)) + mlp_align(4 * sizeof(float)) + 1024;
    if ((st = ensure_ws(c, need, &c->mw, &c->mw_bytes)) != KP_OK) return st;
    Carver cv{(char*)c->mw};
    float* X = cv.take<float>(E * L.I);
    float* Xn = cv.take<float>(E * L.I);
    float* T = cv.take<float>(E * L.O);
    int32_t* idx = cv.take<int32_t>(E);
    float* Xb = cv.take<float>(bs * L.I);
    float* Tb = cv.take<float>(bs * L.O);
    float* dY = cv.take<float>(bs * L.O);
    Acts a = take_acts(cv, L, bs);
    float* dH = cv.take<float>(bs * L.H);
    float* G = cv.take<float>(L.P);
    float* rl = cv.take<float>(bs);
    float* acc = cv.take<float>(4);
    char* m = (char*)model;
    float* P = (float*)(m + L.params);
    float* Mm = (float*)(m + L.m);
    float* Vv = (float*)(m + L.v);
    float* xmean = (float*)(m + L.xmean);
    float* xstd = (float*)(m + L.xstd);
    float* ysc = (float*)(m + L.yscale);
    hipStream_t s = c->stream;
    // data: features and their normalisation, scaled targets
    MLP_HIP(launch_mlp_features(s, E, b->dim, b->params, X));
    MLP_HIP(launch_col_stats(s, E, L.I, X, xmean, xstd));
    MLP_HIP(launch_normalise(s, E, L.I, X, xmean, xstd, Xn));
    MLP_HIP(launch_block_scale(s, E, L.nb, nn, factors, ysc));
    MLP_HIP(launch_scale_targets(s, E, L.nb, nn, factors, ysc, T));
    const int bf = gemm_prec(prec);
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    int step = hdr[7];
    std::vector<int32_t> order(E);
    uint64_t rng = seed;
    const int64_t nbatch = (E + bs - 1) / bs;
    for (int ep = 0; ep < epochs; ++ep) {
        // minibatch order: Fisher-Yates with splitmix64 draws
        for (int64_t i = 0; i < E; ++i) order[i] = (int32_t)i;
        for (int64_t i = E - 1; i > 0; --i) {
            const int64_t j = (int64_t)(splitmix64(rng) % (uint64_t)(i + 1));
            const int32_t t = order[i];
            order[i] = order[j];
            order[j] = t;
        }
        MLP_HIP(hipMemcpyAsync(idx, order.data(), E * sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int64_t bi = 0; bi < nbatch; ++bi) {
            const int rows = (int)((bi + 1) * bs <= E ? bs : E - bi * bs);
            MLP_HIP(launch_gather(s, rows, idx + bi * bs, Xn, L.I, Xb, T, L.O, Tb));
            if ((st = forward(s, bf, L, P, rows, Xb, a)) != KP_OK) return st;
            MLP_HIP(launch_mlp_loss(s, rows, b->dim, b->n, a.Y, Tb, dY, rl, 1.f / (float)((long)rows * L.O)));
            MLP_HIP(launch_sum(s, rows, rl, acc, bi > 0));
            if ((st = backward(s, bf, L, P, rows, Xb, a, dY, dH, G)) != KP_OK) return st;
            ++step;
            const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
            MLP_HIP(launch_adam(s, L.P, P, G, Mm, Vv, lr, beta1, beta2, eps, c1, c2));
        }
        float h = 0.f;
        MLP_HIP(hipMemcpyAsync(&h, acc, sizeof(float), hipMemcpyDeviceToHost, s));
        MLP_HIP(hipStreamSynchronize(s));  // also keeps `order` alive for its copy
        if (loss_hist_h) loss_hist_h[ep] = h / (float)nbatch;
    }
    hdr[7] = step;
    MLP_HIP(hipMemcpyAsync(m + 7 * sizeof(int), &hdr[7], sizeof(int), hipMemcpyHostToDevice, s));
    MLP_HIP(hipStreamSynchronize(s));
    return KP_OK;
}

kp_status kp_mlp_predict(kp_ctx c, const void* model, const kp_batch* b, int32_t prec, double* factors) {
    if (!c || !b) return KP_ERR_ARG;
    if (prec != KP_FP32 && prec != KP_BF16) return KP_ERR_ARG;
    kp_status st = check_batch(b);
    if (st != KP_OK) return st;
    int hdr[8];
    MlpLayout L;
    if ((st = read_header(c, model, hdr, &L)) != KP_OK) return st;
    if (hdr[4] != b->dim || hdr[5] != b->n) return KP_ERR_ARG;
    const int64_t E = b->num_elems;
    if (E == 0) return KP_OK;
    if (!factors) return KP_ERR_ARG;
    const int64_t chunk = E < 16384 ? E : 16384;
    const size_t need = 2 * mlp_align(chunk * L.I * sizeof(float)) + acts_bytes(L, chunk) + 1024;
    if ((st = ensure_ws(c, need, &c->mw, &c->mw_bytes)) != KP_OK) return st;
    Carver cv{(char*)c->mw};
    float* X = cv.take<float>(chunk * L.I);
    float* Xn = cv.take<float>(chunk * L.I);
    Acts a = take_acts(cv, L, chunk);
    const char* m = (const char*)model;
    const float* P = (const float*)(m + L.params);
    const int nn = b->n * b->n;
    for (int64_t e0 = 0; e0 < E; e0 += chunk) {
        const int rows = (int)(e0 + chunk <= E ? chunk : E - e0);
        MLP_HIP(launch_mlp_features(c->stream, rows, b->dim, b->params + e0 * KP_REC_LEN, X));
        MLP_HIP(launch_normalise(c->stream, rows, L.I, X, (const float*)(m + L.xmean),
                                 (const float*)(m + L.xstd), Xn));
        if ((st = forward(c->stream, gemm_prec(prec), L, P, rows, Xn, a)) != KP_OK) return st;
        MLP_HIP(launch_decode(c->stream, rows, L.nb, nn, a.Y, (const float*)(m + L.yscale),
                              factors + e0 * L.O));
    }
    return KP_OK;
}

kp_status kp_set_model(kp_ctx c, const void* model) {
    if (!c) return KP_ERR_ARG;
    if (!model) {
        c->model = nullptr;
        return KP_OK;
    }
    int hdr[8];
    MlpLayout L;
    kp_status st = read_header(c, model, hdr, &L);
    if (st != KP_OK) return st;
    c->model = model;
    c->model_dim = hdr[4];
    c->model_n = hdr[5];
    c->model_hidden = hdr[2];
    return KP_OK;
}

}  // extern "C"
